"""Roofline accounting for the detection kernel (the dominant launch).

Algorithmic work is counted per image pixel with every plane computed once (the
halo recomputation of a tiled execution is overhead, not algorithm):
  * median networks: the min/max operations of the networks the kernels use,
    counted from the generator after dead-code elimination, per output;
    3-input min/max/median instructions count as one operation;
  * binary64 arithmetic: one operation per IEEE add, subtract, multiply, divide,
    square root and compare-select.
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
CENTRE_OPS = 1 + 1 + 1                    # S - med5(S), > sigclip, > sigfrac*sigclip; the contrast
                                          # F^ and S'/F^ is needed only where S' > sigclip
MED3_RUN = 14
MED3_OPS = (3 * (MED3_RUN + 2) + 4 * MED3_RUN) / MED3_RUN   # column sorts of 3 ops + 4 per output


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


def detect_ops_per_pixel() -> dict:
    med5j = network_ops_per_output("med5_t2x5")
    med5s = network_ops_per_output("med5_t2x4")
    med7 = network_ops_per_output("med7_t2x4")
    parts = dict(med3=MED3_OPS, med5_J=med5j, lplus=LPLUS_OPS, noise=NOISE_OPS, s=S_OPS,
                 med7=med7, med5_S=med5s, centre=CENTRE_OPS)
    parts["total"] = sum(parts.values())
    return parts


DETECT_BYTES_PER_PIXEL = 4 + 1            # read J (FP32), write the code byte
