"""Border (halo) sweep of the paper's partitioned run on the GPU.

CRBLASTER cleans N subimages independently, each extended by a border of 6 pixels,
which the paper reports as the smallest border without cleaning artifacts (Section
6.2).  This script measures, for several partitions and borders, how many mask and
cleaned-image pixels differ from the unpartitioned result (N = 1) on synthetic
frames.  An iteration's dependency radius is 8 pixels, so a border of 8 * niter
reproduces N = 1 exactly.

  python -m paper_1008_2192_amd.halo_sweep [--frame c2|c3] [--niter 4]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import _lib, synth

PARTITIONS = [(2, 4), (6, 6), (1, 36), (7, 7)]     # the paper's Mac Pro and TILE64 splits
BORDERS = [0, 2, 4, 6, 8, 16, 32]


def sweep(frame, niter=4, partitions=PARTITIONS, borders=BORDERS):
    img = torch.from_numpy(frame.img).to("cuda")
    c0, m0 = _lib.lacosmic(img, frame.gain, frame.readnoise, niter=niter)
    torch.cuda.synchronize()
    rows = []
    for ny, nx in partitions:
        for b in borders:
            c, m = _lib.lacosmic_partitioned(img, frame.gain, frame.readnoise, ny, nx, b,
                                             niter=niter)
            torch.cuda.synchronize()
            dm = int((m != m0).sum().item())
            dc = int((c != c0).sum().item())
            rows.append(dict(partition=f"{ny}x{nx}", border=b, mask_diff=dm, clean_diff=dc,
                             flagged=int(m0.sum().item())))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frame", default="c2", choices=["c2", "c3"])
    ap.add_argument("--niter", type=int, default=4)
    ap.add_argument("--json", action="store_true")
    a = ap.parse_args()
    f = synth.c2() if a.frame == "c2" else synth.c3()
    rows = sweep(f, a.niter)
    if a.json:
        print(json.dumps(rows))
        return
    print(f"frame {f.name} ({f.img.shape[0]}x{f.img.shape[1]}), niter {a.niter}, "
          f"flagged at N=1: {rows[0]['flagged']}")
    print("| partition | " + " | ".join(f"border {b}" for b in BORDERS) + " |")
    print("|---|" + "---|" * len(BORDERS))
    for ny, nx in PARTITIONS:
        cells = [r for r in rows if r["partition"] == f"{ny}x{nx}"]
        print(f"| {ny}x{nx} | " + " | ".join(f"{r['mask_diff']} / {r['clean_diff']}"
                                             for r in cells) + " |")
    print("(cells: mask pixels / cleaned pixels differing from the unpartitioned run)")


if __name__ == "__main__":
    sys.exit(main())
