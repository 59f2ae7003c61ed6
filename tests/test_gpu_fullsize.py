"""Every pixel of full-size frames against the FP64 oracle.

The frames: the 800x800 WFPC2-like frame, the 4096x4096 crowded field, and one frame of
each large size of the mixed batch (2048x4096 and 4096x2048).  Each runs through the
single-frame entry point and through one graph-captured batch plan holding all four.
The oracle runs on the host cores as independent subimages with a border of 8 pixels
per iteration (the paper's partitioned run, Section 6.2), which gives exactly the
whole-frame oracle's result (pinned on the oracle by the partition-invariance test).

Bars: masks bit-exact at every pixel, the cleaned image within 1e-5 relative at every
pixel (exactly equal where the oracle's value is 0), and the per-frame flag counts equal.
"""
import sys
import time

import numpy as np
import pytest
import torch

from oracle import partition
from paper_1008_2192_amd import _lib, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def f32(x):
    return float(np.float32(x))


def fparams(f):
    return dict(gain=f32(f.gain), readnoise=f32(f.readnoise), sky=f32(f.sky),
                sigclip=f32(f.sigclip), sigfrac=f32(f.sigfrac), objlim=f32(f.objlim))


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def full_frames():
    return [synth.c2(), synth.c3(), synth.c4_frame(32), synth.c4_frame(48)]


@pytest.fixture(scope="module")
def frames_and_oracle():
    frames = full_frames()
    refs = []
    for f in frames:
        r = partition.lacosmic_partitioned(f.img, niter=4, early_stop=False, **fparams(f))
        log(f"oracle {f.name} {f.img.shape}: {r['wall_s']:.1f} s on {r['workers']} host "
            f"threads, {r['split'][0]}x{r['split'][1]} subimages, border {r['border']}; "
            f"{int(r['mask'].sum())} flagged")
        refs.append(r)
    return frames, refs


def compare_every_pixel(what, clean, mask, r):
    gm = mask.cpu().numpy()
    gc = clean.cpu().numpy().astype(np.float64)
    em, ec = r["mask"], r["clean"]
    n_mask = int((gm != em).sum())
    zero = ec == 0.0
    rel = np.abs(gc - ec) / np.where(zero, 1.0, np.abs(ec))
    n_clean = int((rel > 1e-5).sum()) + int((gc[zero] != 0.0).sum())
    log(f"{what}: {gm.size} px, {n_mask} mask mismatches, {n_clean} cleaned pixels beyond "
        f"1e-5 relative, max relative difference {rel.max():.3g}, {int(gm.sum())} flagged")
    assert n_mask == 0, what
    assert n_clean == 0, what


def test_single_frame_entry_point_every_pixel(frames_and_oracle):
    frames, refs = frames_and_oracle
    for f, r in zip(frames, refs):
        img = torch.from_numpy(f.img).to(DEV)
        t0 = time.perf_counter()
        clean, mask = _lib.lacosmic(img, niter=4, early_stop=False, **fparams(f))
        torch.cuda.synchronize()
        log(f"crb_lacosmic {f.name}: {1e3 * (time.perf_counter() - t0):.1f} ms")
        compare_every_pixel(f"crb_lacosmic {f.name}", clean, mask, r)


def test_batch_plan_every_pixel(frames_and_oracle):
    frames, refs = frames_and_oracle
    items = []
    for f in frames:
        img = torch.from_numpy(f.img).to(DEV)
        items.append(dict(img=img, out_clean=torch.full_like(img, -1.0),
                          out_mask=torch.full(img.shape, 7, dtype=torch.uint8, device=DEV),
                          niter=4, early_stop=False, **fparams(f)))
    plan = _lib.Plan(items, use_graph=True)
    plan.run()
    stats = plan.stats()
    for f, it, r, st in zip(frames, items, refs, stats):
        compare_every_pixel(f"batch plan {f.name}", it["out_clean"], it["out_mask"], r)
        assert st["iters_run"] == 4
        assert st["n_flagged"] == int(r["mask"].sum())
    plan.close()
