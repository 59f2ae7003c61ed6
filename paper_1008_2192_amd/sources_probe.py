"""Throughput of the SOURCES work function on the tile farm.

The work function the paper gives as its example of actors returning structures
(Section 7: stellar photometry of the stars in each subimage) reads each pixel once
plus an apron of its declared radius, and writes one 40-byte record per source, so
its roofline is HBM bandwidth: algorithmic bytes per launch = 4 B x pixels +
40 B x sources.  The probe times the farm on the crowded 4096 x 4096 field (20,000
stars, 1.5% cosmic-ray coverage; peaks 5 sigma above the sky, r = 2, 7 x 7
apertures) and on that field tiled 4 x 4 into a 16384 x 16384 frame (1 GiB), over
tile shapes and actor counts (waves), with HIP events on the launch stream.

  python -m paper_1008_2192_amd.sources_probe [--json] [--tile 32x64] [--workers 4096]
                                               [--frame 16384x16384]
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import _lib, synth

HBM_PEAK_GBS = 8000.0
TILES = [(16, 64), (32, 64), (64, 64), (32, 128), (8, 256)]
WORKERS = [1024, 2048, 4096, 8192, 16384]


def field():
    f = synth.c3()
    sky = 200.0 / 1.5
    t = sky + 5.0 * np.sqrt(200.0 + 16.0) / 1.5
    return f.img, float(t), float(sky)


def time_farm(x, t, sky, th, tw, workers, out, reps=10):
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    _lib.farm_sources(x, t, sky, 2, 3, workers=workers, tile_h=th, tile_w=tw, out=out)
    for a, b in ev:
        a.record(s)
        _lib.farm_sources(x, t, sky, 2, 3, workers=workers, tile_h=th, tile_w=tw, out=out)
        b.record(s)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return ms[len(ms) // 2]


def probe(tiles=TILES, workers=WORKERS, frames=("4096x4096", "16384x16384")):
    img, t, sky = field()
    rows = []
    for name in frames:
        frame = img if name == "4096x4096" else np.tile(img, (4, 4))
        x = torch.from_numpy(frame).cuda()
        out = _lib.farm_sources(x, t, sky, 2, 3, capacity=1 << 22)
        torch.cuda.synchronize()
        n_src = int(out.count.item())
        alg = 4.0 * frame.size + 40.0 * n_src
        for th, tw in tiles:
            for w in workers:
                ms = time_farm(x, t, sky, th, tw, w, out)
                gbs = alg / (ms * 1e-3) / 1e9
                rows.append(dict(frame=name, tile=f"{th}x{tw}", workers=w, ms=round(ms, 4),
                                 sources=n_src, gbs=round(gbs, 1),
                                 frac=round(gbs / HBM_PEAK_GBS, 3)))
        del x, out
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--json", action="store_true")
    ap.add_argument("--tile", default=None, help="one tile shape, e.g. 32x64")
    ap.add_argument("--workers", type=int, default=None, help="one worker count")
    ap.add_argument("--frame", default=None, choices=["4096x4096", "16384x16384"])
    a = ap.parse_args()
    tiles = [tuple(int(v) for v in a.tile.split("x"))] if a.tile else TILES
    workers = [a.workers] if a.workers else WORKERS
    frames = [a.frame] if a.frame else ["4096x4096", "16384x16384"]
    rows = probe(tiles, workers, frames)
    if a.json:
        print(json.dumps(rows))
        return
    print("| frame | tile | workers | ms | sources | GB/s (algorithmic) | of 8 TB/s |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['frame']} | {r['tile']} | {r['workers']} | {r['ms']} | {r['sources']} | "
              f"{r['gbs']} | {r['frac']:.1%} |")
    for name in frames:
        best = min((r for r in rows if r["frame"] == name), key=lambda r: r["ms"])
        print(f"best {name}: tile {best['tile']}, {best['workers']} workers, {best['ms']} ms, "
              f"{best['gbs']} GB/s ({best['frac']:.1%})")


if __name__ == "__main__":
    main()
