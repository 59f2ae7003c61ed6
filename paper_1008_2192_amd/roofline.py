"""Roofline accounting for the detection kernel (the dominant launch).

Algorithmic work is counted with every plane computed once (the halo recomputation
of a tiled execution is overhead, not algorithm):
  * dense, per image pixel: a lower bound of med5(J) (the least of the four middle rows
    of each 2 x 5 cell's nine columns, 18 three-input minima per cell); L+; N at that bound
    (once per cell) and the upper bound of S it gives; the test of that bound against
    sigclip, which marks the pixels near which the other statistics can matter;
  * per pixel whose med5(J) is selected exactly (the cells within 4 of such a mark,
    counted by the kernel on the tile's own pixels): the med5 network, N and S;
  * per work-set pixel (within 2 of an S > sigclip pixel, S > sigfrac * sigclip):
    med5 of S, S' and the two threshold compares;
  * per contrast test (S' > sigclip): N from the pixel's estimate of S and its L+ sum
    (N = L+ / (2 S): the pixel's med5(J) was selected exactly and counted above), the 49
    med3(J) values of the med7 window (13 operations each: three sorted columns of three,
    then three column extremes and their median), and the test
    S'/F^ > objlim, decided by comparing those values with the test's switching value
    and counting them (the test holds at med7 iff it holds at 25 or more of them), which
    is less work than selecting med7.
The three sparse counts come from the kernel's own counters (crb_plan_work_counts).
Median networks count their min/max operations after dead-code elimination, per
output, from the generator; binary64 arithmetic counts one operation per IEEE add,
subtract, multiply, divide, square root and compare-select.
Peak: 256 compute units x 64 lanes x 2.4 GHz = 3.93e13 lane operations per second
(one non-packed VALU operation per lane per clock; binary64 add/mul/fma issue at
the same rate on CDNA4, which is how the published 78.6 TFLOP/s FP64 vector peak
arises from 64 lanes x 2 flops x 256 CUs x 2.4 GHz).
"""
from __future__ import annotations

import functools
import os
import sys

CU = 256
LANES = 64
CLOCK_HZ = 2.4e9
ALU_PEAK = CU * LANES * CLOCK_HZ          # lane operations per second
HBM_PEAK = 8.0e12                         # bytes per second

# binary64 operations per pixel
LPLUS_OPS = 4 * (1 + 4 + 1) + 3 + 1       # 4 sub-pixels: 4c, 4 subtractions, clip; 3 adds, /4
NOISE_OPS = 1 + 1 + 1 + 1 + 1 + 1         # +sky, floor, g*m, +rn^2, sqrt, /g
S_OPS = 2                                 # 2N, L+/(2N)
HOT_OPS = 1                               # S > sigclip
MED3_AT_OPS = 3 * 3 + 3 + 1               # one med3(J) value from its 3 x 3 window
# lower bound of med5(J): the least of the 36 values of a 2 x 5 cell's four middle rows
# (18 three-input minima per cell)
BOUND_OPS = 18 / 10
BOUND_NOISE_OPS = NOISE_OPS / 10          # N at the bound, once per 2 x 5 cell
# per work-set pixel, besides med5(S): S - med5(S), > sigclip, > sigfrac*sigclip
WORK_OPS = 3
# per contrast test: N as L+ / (2 S) from the pixel's S (2); the floor test S'/0.01 >
# objlim, N S'/objlim, the switching value and its band (6); two comparisons and two
# counts per window value (4 x 49); the two count tests (2)
CONTRAST_OPS = 2 + 6 + 4 * 49 + 2


@functools.lru_cache(maxsize=None)
def network_ops_per_output(name: str) -> float:
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    sys.path.insert(0, here)
    try:
        import gen_networks as g
    finally:
        sys.path.pop(0)
    for fn, k, ty, tx in g.TILES:
        if fn == name:
            tm = g.TileMedian(k, ty, tx).build()
            outs = list(tm.outputs.values())
            return g.count_ops(tm.net, outs) / (ty * tx)
    raise KeyError(name)


def detect_ops() -> dict:
    """Operations per image pixel (dense), per pixel of exact med5(J), per work-set
    pixel and per contrast test."""
    dense = dict(med5_bound=BOUND_OPS, lplus=LPLUS_OPS, noise_bound=BOUND_NOISE_OPS,
                 s_bound=S_OPS, hot=HOT_OPS)
    dense["total"] = sum(dense.values())
    return dict(dense=dense,
                per_exact_pixel=network_ops_per_output("med5_t2x2") + NOISE_OPS + S_OPS,
                per_work_pixel=network_ops_per_output("med5_t1x1") + WORK_OPS,
                per_contrast=CONTRAST_OPS + 49 * MED3_AT_OPS)


def detect_ops_per_launch(pixels: int, exact_pixels: float, work_pixels: float,
                          contrast_tests: float) -> float:
    """Algorithmic lane operations of one detection launch."""
    o = detect_ops()
    return (o["dense"]["total"] * pixels + o["per_exact_pixel"] * exact_pixels +
            o["per_work_pixel"] * work_pixels + o["per_contrast"] * contrast_tests)


DETECT_BYTES_PER_PIXEL = 4 + 1            # read J (FP32), write the code byte
