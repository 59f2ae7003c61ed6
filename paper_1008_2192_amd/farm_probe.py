"""Framework efficiency with the paper's POISSON and WAITER work functions.

The paper measures CRBLASTER's efficiency on 1..57 TILE64 tiles with two work
functions of near-uniform per-pixel cost and no border (Section 6.3.2: POISSON on a
750x750 image of 24.3; Section 6.3.3: WAITER on a 750x750 image of 137, i.e. 137 us
per pixel).  Here the actors are the waves of a persistent farm pulling bands of
rows from atomic tickets; speedup S_n = t_1 / t_n and efficiency S_n / n.

  python -m paper_1008_2192_amd.farm_probe [--band-rows 1]
"""
from __future__ import annotations

import argparse
import json

import torch

from . import _lib

WORKERS = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096]


def time_run(kind, x, workers, band_rows, reps=3):
    best = None
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        _lib.work_run(kind, x, seed=1, workers=workers, band_rows=band_rows)
        e.record()
        torch.cuda.synchronize()
        t = s.elapsed_time(e)
        best = t if best is None else min(best, t)
    return best


def probe(band_rows=1, workers=WORKERS):
    rows = []
    for name, kind, value in (("POISSON", _lib.CRB_WORK_POISSON, 24.3),
                              ("WAITER", _lib.CRB_WORK_WAITER, 137.0)):
        x = torch.full((750, 750), value, device="cuda")
        _lib.work_run(kind, x, workers=64, band_rows=band_rows)       # warm-up
        torch.cuda.synchronize()
        t1 = None
        for n in workers:
            t = time_run(kind, x, n, band_rows)
            t1 = t if t1 is None else t1
            rows.append(dict(work=name, workers=n, ms=round(t, 4),
                             speedup=round(t1 / t, 2), efficiency=round(t1 / t / n, 4)))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--band-rows", type=int, default=1)
    ap.add_argument("--json", action="store_true")
    a = ap.parse_args()
    rows = probe(a.band_rows)
    if a.json:
        print(json.dumps(rows))
        return
    print(f"750x750 images, bands of {a.band_rows} row(s), one wave (64 lanes) per actor")
    print("| actors | POISSON ms | POISSON efficiency | WAITER ms | WAITER efficiency |")
    print("|---|---|---|---|---|")
    for n in WORKERS:
        p = next(r for r in rows if r["work"] == "POISSON" and r["workers"] == n)
        w = next(r for r in rows if r["work"] == "WAITER" and r["workers"] == n)
        print(f"| {n} | {p['ms']} | {p['efficiency']:.2%} | {w['ms']} | {w['efficiency']:.2%} |")


if __name__ == "__main__":
    main()
