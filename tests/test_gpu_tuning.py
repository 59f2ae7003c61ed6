"""Every launch shape the autotuner can pick gives bit-identical results.

The shapes: detection tiles of 16, 32 or 64 rows, launched one block per tile or as
persistent blocks taking tiles from ticket counters; grow and replacement as three
launches with first-iteration strips of 8, 16 or 32 rows, or fused into one launch per
iteration.  Each shape runs a batch of frames with ragged sizes (narrower and wider than
a strip, widths that are and are not multiples of 16, single rows and columns, and a
frame crowded enough to overflow the detection's lists) and must
reproduce the default shape's masks, cleaned images and counts exactly; the default is
checked against the FP64 oracle.  Also: incremental detection under each tile height,
graph plans re-captured after a change of shape, the single-frame options, the
autotuner's choice and its cache.
"""
import itertools
import os

import numpy as np
import pytest
import torch

from oracle import ref
from paper_1008_2192_amd import _lib, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"

SHAPES = [dict(tile_h=th, persistent=pe, fused=fu, grow_h=gh)
          for th, pe in itertools.product((16, 32, 64), (0, 1))
          for fu, gh in ((0, 0), (0, 8), (0, 16), (0, 32), (1, 0))]


def f32(x):
    return float(np.float32(x))


def fparams(f):
    return dict(gain=f32(f.gain), readnoise=f32(f.readnoise), sky=f32(f.sky),
                sigclip=f32(f.sigclip), sigfrac=f32(f.sigfrac), objlim=f32(f.objlim))


def batch_frames():
    c2 = synth.c2()
    c2.img = np.ascontiguousarray(c2.img[:230, :301])
    out = [synth.c1(), c2]
    for (H, W, seed) in [(33, 97, 31), (1, 40, 32), (40, 1, 33), (70, 130, 35), (97, 65, 38),
                         (150, 2100, 39), (129, 1000, 40), (64, 1984, 41)]:
        out.append(synth.c1_density_frame(H, W, seed, 1.0, 5.0))
    # 15% of the pixels hit: tiles overflow the work and contrast lists at every height
    out.append(synth.render(128, 192, 77, sky_e=100.0, gain=2.0, readnoise=5.0, n_stars=40,
                            star_fwhm=2.0, star_flux="lognormal", hit_coverage=0.15,
                            hit_len=(1, 8), hit_amp=(200.0, 5000.0)))
    return out


def make_items(frames, incremental=False):
    items = []
    for f in frames:
        img = torch.from_numpy(f.img).to(DEV)
        items.append(dict(img=img, out_clean=torch.full_like(img, -1.0),
                          out_mask=torch.full(img.shape, 7, dtype=torch.uint8, device=DEV),
                          niter=4, early_stop=False, incremental=incremental, **fparams(f)))
    return items


def snapshot(items):
    return [(it["out_clean"].clone(), it["out_mask"].clone()) for it in items]


def poison(items):
    for it in items:
        it["out_clean"].fill_(-1.0)
        it["out_mask"].fill_(7)


@pytest.fixture(scope="module")
def reference():
    frames = batch_frames()
    items = make_items(frames)
    plan = _lib.Plan(items, use_graph=False)
    assert plan.get_tuning() == _lib.DEFAULT_TUNING
    plan.run()
    stats = plan.stats()
    ref_out = snapshot(items)
    for f, (c, m), st in zip(frames, ref_out, stats):
        r = ref.lacosmic(f.img, niter=4, early_stop=False, **fparams(f))
        np.testing.assert_array_equal(m.cpu().numpy(), r["mask"], err_msg=str(f.img.shape))
        np.testing.assert_allclose(c.cpu().numpy().astype(np.float64), r["clean"], rtol=1e-5,
                                   atol=0, err_msg=str(f.img.shape))
        assert st["n_flagged"] == int(r["mask"].sum())
    plan.close()
    return frames, ref_out, stats


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "t{tile_h}p{persistent}f{fused}g{grow_h}"
                         .format(**s))
def test_every_shape_bit_identical(reference, shape):
    frames, ref_out, ref_stats = reference
    items = make_items(frames)
    plan = _lib.Plan(items, use_graph=False)
    plan.set_tuning(**shape)
    assert plan.get_tuning() == shape
    for rep in range(2):           # a second run on the same plan (tickets, stale stamps)
        poison(items)
        plan.run()
        stats = plan.stats()
        for f, it, (c, m), st, rst in zip(frames, items, ref_out, stats, ref_stats):
            assert torch.equal(it["out_mask"], m), (shape, f.img.shape, rep)
            assert torch.equal(it["out_clean"], c), (shape, f.img.shape, rep)
            assert st == rst, (shape, f.img.shape, rep)
    plan.close()


@pytest.mark.parametrize("tile_h", [16, 32, 64])
@pytest.mark.parametrize("fused", [0, 1])
def test_incremental_detection_under_each_shape(reference, tile_h, fused):
    frames, ref_out, _ = reference
    items = make_items(frames, incremental=True)
    plan = _lib.Plan(items, use_graph=False)
    plan.set_tuning(tile_h=tile_h, persistent=1, fused=fused)
    for rep in range(2):
        poison(items)
        plan.run()
        plan.stats()
        for f, it, (c, m) in zip(frames, items, ref_out):
            assert torch.equal(it["out_mask"], m), (tile_h, fused, f.img.shape, rep)
            assert torch.equal(it["out_clean"], c), (tile_h, fused, f.img.shape, rep)
    plan.close()


def test_graph_plan_recaptured_after_set_tuning(reference):
    frames, ref_out, _ = reference
    items = make_items(frames)
    plan = _lib.Plan(items, use_graph=True)
    for shape in (dict(tile_h=64, persistent=1, fused=1, grow_h=0),
                  dict(tile_h=16, persistent=0, fused=0, grow_h=16)):
        plan.set_tuning(**shape)
        for rep in range(3):
            poison(items)
            plan.run()
            plan.stats()
            _ = torch.randn(1000, device=DEV).sum().item()     # eager work between replays
            for it, (c, m) in zip(items, ref_out):
                assert torch.equal(it["out_mask"], m), (shape, rep)
                assert torch.equal(it["out_clean"], c), (shape, rep)
    plan.close()


def test_single_frame_options(reference):
    frames, ref_out, _ = reference
    try:
        for tile_h, fused, grow_h in ((16, 0, 16), (64, 1, 0), (32, 1, 0), (64, 0, 32)):
            _lib.set_single_tuning(tile_h, fused, grow_h)
            for f, (c, m) in zip(frames, ref_out):
                img = torch.from_numpy(f.img).to(DEV)
                gc, gm = _lib.lacosmic(img, niter=4, early_stop=False, **fparams(f))
                na_c, na_m = _lib.lacosmic_noalloc(img, niter=4, early_stop=False, **fparams(f))
                torch.cuda.synchronize()
                assert torch.equal(gm, m) and torch.equal(gc, c), (tile_h, fused, f.img.shape)
                assert torch.equal(na_m, m) and torch.equal(na_c, c), (tile_h, fused, f.img.shape)
            # the teacher-forced iteration keeps its G2 plane under any option
            f = frames[0]
            J = torch.from_numpy(f.img).to(DEV)
            M0 = torch.zeros(f.img.shape, dtype=torch.uint8, device=DEV)
            G2, M1, J2, n = _lib.debug_iterate(J, M0, **fparams(f))
            torch.cuda.synchronize()
            r = ref.iterate(f.img, np.zeros(f.img.shape, np.uint8), **fparams(f))
            np.testing.assert_array_equal(G2.cpu().numpy(), r["G2"])
            assert int(n.item()) == r["n"]
    finally:
        _lib.set_single_tuning(32, 0, 0)


def test_autotune_choice_and_cache(reference, tmp_path):
    frames, ref_out, _ = reference
    cache = tmp_path / "tune.txt"
    os.environ["CRB_TUNE_CACHE"] = str(cache)
    try:
        items = make_items(frames)
        plan = _lib.Plan(items, use_graph=False)
        res = plan.autotune(reps=2, use_cache=True)
        print(f"autotune: {res}", flush=True)
        assert res["ms"] > 0 and res["default_ms"] > 0 and res["ms"] <= res["default_ms"]
        assert plan.get_tuning() == res["tuning"]
        poison(items)
        plan.run()
        plan.stats()
        for it, (c, m) in zip(items, ref_out):
            assert torch.equal(it["out_mask"], m) and torch.equal(it["out_clean"], c)
        plan.close()
        text = cache.read_text()
        assert text.startswith("crb-tune 1 ") and "tile_h=" in text
        # a new plan over the same layout starts with the cached shapes, and autotune with
        # the cache applies them without timing
        plan2 = _lib.Plan(make_items(frames), use_graph=True)
        assert plan2.get_tuning() == res["tuning"]
        res2 = plan2.autotune(reps=2, use_cache=True)
        assert res2["tuning"] == res["tuning"] and res2["ms"] == -1.0
        plan2.close()
    finally:
        del os.environ["CRB_TUNE_CACHE"]


def test_autotune_refuses_in_place_frames():
    f = synth.c1()
    img = torch.from_numpy(f.img).to(DEV)
    items = [dict(img=img, out_clean=img,
                  out_mask=torch.empty(img.shape, dtype=torch.uint8, device=DEV),
                  niter=4, **fparams(f))]
    plan = _lib.Plan(items, use_graph=False)
    with pytest.raises(_lib.CrbError):
        plan.autotune(reps=1, use_cache=False)
    plan.close()


@pytest.mark.parametrize("shape", [dict(tile_h=32, persistent=0, fused=0, grow_h=0),
                                   dict(tile_h=64, persistent=0, fused=1, grow_h=0),
                                   dict(tile_h=16, persistent=1, fused=0, grow_h=16)],
                         ids=["default", "t64-fused", "t16-persistent"])
def test_one_frame_plans(reference, shape):
    """A plan of one frame launches it by value (as crb_lacosmic does) unless its
    detection is persistent; eager and graph runs, with the work counters switched on
    between them, reproduce the reference."""
    frames, ref_out, ref_stats = reference
    for i in (0, 1, 7):
        items = make_items([frames[i]])
        for use_graph in (False, True):
            plan = _lib.Plan(items, use_graph=use_graph)
            plan.set_tuning(**shape)
            for counting in (False, True):
                if counting and not use_graph:
                    plan.set_counting(True)
                poison(items)
                plan.run()
                st = plan.stats()
                c, m = ref_out[i]
                assert torch.equal(items[0]["out_mask"], m), (shape, i, use_graph)
                assert torch.equal(items[0]["out_clean"], c), (shape, i, use_graph)
                assert st[0] == ref_stats[i], (shape, i, use_graph)
            if not use_graph:
                counts = plan.work_counts()
                assert counts["work_pixels"] > 0, (shape, i)
            plan.close()
