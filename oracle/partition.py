"""The FP64 oracle on a whole frame, run as independent subimages on the host cores.

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's CPU-baseline
leg, never by the GPU library or its binding.

This is the paper's multi-processor arrangement (Section 6.2): the frame is cut into
a 2-D grid of rectangles, each rectangle is extended by a border on every side it
shares with another, each extended subimage is cleaned by its own worker with no
communication, and only the interiors are kept.  One iteration of the method reads
at most 8 pixels away (4 for the detection statistics, 1 for each grow, 2 for the
replacement window), so a whole run of niter iterations depends on pixels at most
8 * niter away; with that border the stitched result is identical to the oracle on
the whole frame (the partition-invariance pin checks this on the oracle itself).

Workers are threads: each calls the C oracle, which runs with the interpreter lock
released, on its own subimage and owns all of its memory.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import time
from typing import Optional, Tuple

import numpy as np

from . import ref


def host_workers(cap: int = 16) -> int:
    """Worker count: the cores this process may run on, at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def grid_for(H: int, W: int, workers: int, min_side: int = 256) -> Tuple[int, int]:
    """A split with about two rectangles per worker, none below min_side pixels a side."""
    best = (1, 1)
    target = 2 * workers
    for ny in range(1, max(1, H // min_side) + 1):
        for nx in range(1, max(1, W // min_side) + 1):
            n = ny * nx
            if n > target:
                continue
            # prefer more rectangles, then squarer ones
            key = (n, -abs(H / ny - W / nx))
            if key > (best[0] * best[1], -abs(H / best[0] - W / best[1])):
                best = (ny, nx)
    return best


def lacosmic_partitioned(img: np.ndarray, gain, readnoise, sky=0.0, sigclip=4.5,
                         sigfrac=0.3, objlim=4.0, niter=4, early_stop=False,
                         split: Optional[Tuple[int, int]] = None, border: Optional[int] = None,
                         workers: Optional[int] = None) -> dict:
    """The oracle on `img` as independent bordered subimages; returns dict(clean (FP64),
    mask, wall_s, workers, split, border).  With border >= 8 * niter (the default) the
    result equals ref.lacosmic on the whole frame."""
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W = img.shape
    workers = workers or host_workers()
    border = 8 * niter if border is None else border
    ny, nx = split or grid_for(H, W, workers)
    jobs = []
    for i in range(ny):
        for j in range(nx):
            y0, y1 = H * i // ny, H * (i + 1) // ny
            x0, x1 = W * j // nx, W * (j + 1) // nx
            a0, a1 = max(0, y0 - border), min(H, y1 + border)
            b0, b1 = max(0, x0 - border), min(W, x1 + border)
            jobs.append((y0, y1, x0, x1, a0, a1, b0, b1))

    def run(job):
        y0, y1, x0, x1, a0, a1, b0, b1 = job
        r = ref.lacosmic(np.ascontiguousarray(img[a0:a1, b0:b1]), gain, readnoise, sky,
                         sigclip, sigfrac, objlim, niter, early_stop)
        return (r["clean"][y0 - a0:y1 - a0, x0 - b0:x1 - b0],
                r["mask"][y0 - a0:y1 - a0, x0 - b0:x1 - b0])

    clean = np.empty((H, W), np.float64)
    mask = np.empty((H, W), np.uint8)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        for job, (c, m) in zip(jobs, ex.map(run, jobs)):
            y0, y1, x0, x1 = job[:4]
            clean[y0:y1, x0:x1] = c
            mask[y0:y1, x0:x1] = m
    wall = time.perf_counter() - t0
    return dict(clean=clean, mask=mask, wall_s=wall, workers=workers, split=(ny, nx),
                border=border)
