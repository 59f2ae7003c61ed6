"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: masks and counts bit-exact; the cleaned image within 1e-5 relative (FP32
output against the binary64 oracle; the kernels' replacements are exact FP32
selections or the correctly rounded mean of two).  The oracle's decision statistics
are binary64; the detection decides from an FP32 estimate of S where its error bound
settles the comparison and in binary64 otherwise, so for a given input J_k the
detection is identical; the teacher-forced test feeds both sides the same FP32 J_k
each iteration.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import ref
from paper_1008_2192_amd import _lib, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def f32(x):
    return float(np.float32(x))


def fparams(f):
    """The FP32 parameter values the GPU receives, for the binary64 oracle."""
    return dict(gain=f32(f.gain), readnoise=f32(f.readnoise), sky=f32(f.sky),
                sigclip=f32(f.sigclip), sigfrac=f32(f.sigfrac), objlim=f32(f.objlim))


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small_frames():
    """Frames spanning several detection tiles with ragged tails, plus tiny ones."""
    out = [synth.c1()]
    c2 = synth.c2()
    c2.img = np.ascontiguousarray(c2.img[:230, :301])
    out.append(c2)
    for (H, W, seed) in [(33, 97, 31), (1, 40, 32), (40, 1, 33), (5, 5, 34), (70, 130, 35),
                         (2, 3, 36), (1, 1, 37), (97, 65, 38)]:
        out.append(synth.c1_density_frame(H, W, seed, 1.0, 5.0))
    return out


def test_fp64_sqrt_and_division_correctly_rounded():
    rng = np.random.default_rng(0)
    x = 10.0 ** rng.uniform(-6, 9, 200000)
    y = 10.0 ** rng.uniform(-4, 6, 200000)
    s, d = _lib.debug_fp64(torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(s.cpu().numpy(), np.sqrt(x))
    np.testing.assert_array_equal(d.cpu().numpy(), x / y)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_median_networks_match_oracle(r):
    rng = np.random.default_rng(r)
    shapes = [(1, 1), (1, 9), (9, 1), (3, 5), (37, 53), (64, 64), (130, 67)]
    for (H, W) in shapes:
        for kind in ("ties", "cont"):
            if kind == "ties":
                x = rng.integers(0, 5, (H, W)).astype(np.float32)
            else:
                x = rng.normal(100, 10, (H, W)).astype(np.float32)
            g = _lib.debug_median(torch.from_numpy(x).to(DEV), r)
            torch.cuda.synchronize()
            exp = ref.median_filter(x.astype(np.float64), r).astype(np.float32)
            np.testing.assert_array_equal(g.cpu().numpy(), exp, err_msg=f"{H}x{W} {kind}")


def dilate(mask, r):
    """In-frame (2r+1)^2 dilation, computed by shifting (no library call)."""
    H, W = mask.shape
    out = np.zeros_like(mask)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            ys, ye = max(0, -dy), min(H, H - dy)
            xs, xe = max(0, -dx), min(W, W - dx)
            if ys < ye and xs < xe:
                out[ys:ye, xs:xe] |= mask[ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def grow_from_codes(codes):
    """G1 and G2 of the method from a code plane (A, hi, lo bits)."""
    A, hi, lo = (codes & 1) > 0, (codes & 2) > 0, (codes & 4) > 0
    G1 = dilate(A, 1) & hi
    return G1, dilate(G1, 1) & lo


def check_codes(got, exp, near, tr, what):
    """Codes equal the full definition within distance 2 of S > sigclip and are 0 or
    the full definition elsewhere; G1 and G2 built from them equal the oracle's."""
    far = got[~near]
    log(f"{what}: {int((got[near] != exp[near]).sum())} code mismatches near "
        f"S > sigclip ({int(near.sum())} px), {int((far != 0).sum())} nonzero elsewhere, "
        f"{int((exp & 1).sum())} first-selected")
    np.testing.assert_array_equal(got[near], exp[near], err_msg=what)
    assert ((far == 0) | (far == exp[~near])).all(), what
    G1, G2 = grow_from_codes(got)
    np.testing.assert_array_equal(G1, tr["g1"] > 0, err_msg=what)
    np.testing.assert_array_equal(G2, tr["g2"] > 0, err_msg=what)


def expected_codes(tr, p):
    return (tr["first"] | ((tr["sprime"] > p["sigclip"]) << 1) |
            ((tr["sprime"] > p["sigfrac"] * p["sigclip"]) << 2)).astype(np.uint8)


@pytest.mark.parametrize("exact", [False, True], ids=["estimate", "binary64"])
def test_detection_codes_match_oracle(exact):
    """Both detection paths: decisions from the FP32 estimate of S where its bound
    settles them, and every work-set pixel re-evaluated in binary64 from J.  The last
    frame is quantised to steps of 8 ADU, so that windows hold many ties and the lower
    bound of med5(J) that marks the candidates often equals med5(J)."""
    ties = synth.c1(seed=11)
    ties.img = (np.round(ties.img / np.float32(8.0)) * np.float32(8.0)).astype(np.float32)
    for f in small_frames() + [ties]:
        p = fparams(f)
        tr = ref.iterate(f.img, np.zeros(f.img.shape, np.uint8), trace=True, **p)
        near = dilate(tr["s"] > p["sigclip"], 2)
        codes = _lib.debug_detect(torch.from_numpy(f.img).to(DEV), exact=exact, **p)
        torch.cuda.synchronize()
        check_codes(codes.cpu().numpy(), expected_codes(tr, p), near, tr,
                    f"detect {f.img.shape} exact={exact}")


@pytest.mark.parametrize("objlim", [0.02, 0.5, 1.0, 2.0, 3.0, 4.0, 6.0, 10.0, 30.0])
def test_contrast_decisions_across_objlim(objlim):
    """The contrast test decided by counting the med7 window against its switching
    value, at objlim values that move that value through the window: codes equal the
    oracle's near S > sigclip on a frame dense in hits and stars."""
    f = synth.c2()
    img = np.ascontiguousarray(f.img[:160, :200])
    p = fparams(f)
    p["objlim"] = f32(objlim)
    tr = ref.iterate(img, np.zeros(img.shape, np.uint8), trace=True, **p)
    near = dilate(tr["s"] > p["sigclip"], 2)
    exp = expected_codes(tr, p)
    codes = _lib.debug_detect(torch.from_numpy(img).to(DEV), **p)
    torch.cuda.synchronize()
    check_codes(codes.cpu().numpy(), exp, near, tr, f"objlim {objlim}")
    assert 0 < int((exp & 1).sum()) < int((exp & 2).sum()) or objlim in (0.02, 30.0)


# Frames whose statistics span many binades: gains, sky levels and signal scales
# far from the synthetic workloads, negative skies (the floor of m), a zero read noise.
SCALES = [(1.0, 5.0, 0.0, 1.0), (1e-3, 0.5, 0.0, 1e3), (1e3, 50.0, 0.0, 1e-3),
          (2.5, 0.0, -120.0, 1.0), (0.7, 3.0, 1e4, 30.0), (7.0, 8.0, 0.0, 1e-6)]


@pytest.mark.parametrize("case", range(len(SCALES)))
def test_s_estimate_error_bound(case):
    """|s - S| <= err at every pixel, S from the oracle's binary64 trace, and the
    bound is tight enough to settle S > sigclip from s at nearly every pixel."""
    gain, rn, sky, scale = SCALES[case]
    f = synth.c1_density_frame(97, 131, 500 + case, max(gain, 1.0), max(rn, 1.0))
    img = np.ascontiguousarray((f.img.astype(np.float64) * scale).astype(np.float32))
    p = dict(gain=f32(gain), readnoise=f32(rn), sky=f32(sky), sigclip=4.5, sigfrac=0.3,
             objlim=4.0)
    tr = ref.iterate(img, np.zeros(img.shape, np.uint8), trace=True, **p)
    s, err = _lib.debug_s_estimate(torch.from_numpy(img).to(DEV), **p)
    torch.cuda.synchronize()
    s = s.cpu().numpy().astype(np.float64)
    err = err.cpu().numpy().astype(np.float64)
    S = tr["s"]
    assert np.isfinite(err).all(), case
    gap = np.abs(s - S)
    undecided = np.abs(s - p["sigclip"]) <= err
    log(f"s estimate case {case}: max |s - S| / err = {float((gap / np.maximum(err, 1e-300)).max()):.3g}, "
        f"median err / (1 + S) = {float(np.median(err / (1 + S))):.3g}, "
        f"{int(undecided.sum())} px undecided at sigclip, {int((S > p['sigclip']).sum())} hot")
    assert (gap <= err).all(), case
    assert undecided.sum() <= 2, case
    # the dense bound the detection takes its candidates from: above S everywhere, and
    # its candidates hold every pixel of S > sigclip
    u = _lib.debug_s_bound(torch.from_numpy(img).to(DEV), **p)
    torch.cuda.synchronize()
    u = u.cpu().numpy().astype(np.float64)
    log(f"dense bound case {case}: min (u - S) / (1 + S) = {float(((u - S) / (1 + S)).min()):.3g}, "
        f"{int((u > p['sigclip']).sum())} candidates for {int((S > p['sigclip']).sum())} hot")
    assert (u >= S).all(), case
    assert (u > np.float64(np.float32(p["sigclip"]) * np.float32(1 - 2.0 ** -20)))[S > p["sigclip"]].all()
    codes = _lib.debug_detect(torch.from_numpy(img).to(DEV), **p)
    torch.cuda.synchronize()
    near = dilate(S > p["sigclip"], 2)
    check_codes(codes.cpu().numpy(), expected_codes(tr, p), near, tr, f"scales case {case}")


def test_single_output_med5_network_binary64():
    rng = np.random.default_rng(5)
    for (H, W) in [(1, 1), (1, 7), (7, 1), (5, 5), (33, 70)]:
        for kind in ("ties", "cont"):
            if kind == "ties":
                x = rng.integers(0, 4, (H, W)).astype(np.float64)
            else:
                x = rng.normal(0, 1, (H, W)) * 10.0 ** rng.integers(-3, 4, (H, W))
            g = _lib.debug_median5_f64(torch.from_numpy(x).to(DEV))
            torch.cuda.synchronize()
            np.testing.assert_array_equal(g.cpu().numpy(), ref.median_filter(x, 2),
                                          err_msg=f"{H}x{W} {kind}")


def test_work_counts_match_oracle_sets():
    """Plan work counters on one iteration: the work set holds D2(S > sigclip) &
    (S > sigfrac*sigclip) (from the estimate of S widened by its bound: a few more
    pixels at most), the contrast tests are exactly the pixels with S' > sigclip, and
    binary64 re-evaluations are rare."""
    frames = small_frames()[:2] + [synth.c1_density_frame(300, 400, 77, 2.5, 6.0)]
    items, exp_w, exp_c = [], 0, 0
    for f in frames:
        p = fparams(f)
        tr = ref.iterate(f.img, np.zeros(f.img.shape, np.uint8), trace=True, **p)
        lowlim = np.float64(np.float32(p["sigfrac"])) * np.float64(np.float32(p["sigclip"]))
        exp_w += int((dilate(tr["s"] > p["sigclip"], 2) & (tr["s"] > lowlim)).sum())
        exp_c += int((tr["sprime"] > p["sigclip"]).sum())
        img = torch.from_numpy(f.img).to(DEV)
        items.append(dict(img=img, out_clean=torch.empty_like(img),
                          out_mask=torch.empty(img.shape, dtype=torch.uint8, device=DEV),
                          niter=1, early_stop=False, **p))
    plan = _lib.Plan(items, use_graph=False)
    plan.set_counting(True)
    plan.run()
    got = plan.work_counts()
    plan.set_counting(False)                  # clears the counters and stops counting
    plan.run()
    assert plan.work_counts() == dict(work_pixels=0, contrast_tests=0, reevaluated=0,
                                      exact_med5=0)
    plan.close()
    log(f"work counts {got}, expected {exp_w} / {exp_c}")
    assert exp_w <= got["work_pixels"] <= exp_w + exp_w // 100 + 4
    assert got["contrast_tests"] == exp_c
    assert got["reevaluated"] <= got["work_pixels"] // 100 + 4
    # every work-set pixel has its med5(J) selected exactly
    assert got["work_pixels"] <= got["exact_med5"] <= sum(f.img.size for f in frames)


def test_iterations_teacher_forced():
    """Each iteration from the same FP32 J_k and M_{k-1} on both sides."""
    for f in small_frames()[:3] + small_frames()[6:]:
        p = fparams(f)
        J = f.img.astype(np.float32)
        M = np.zeros(J.shape, np.uint8)
        for k in range(1, 5):
            exp = ref.iterate(J.astype(np.float64), M, **p)
            G2, Mk, Jn, n = _lib.debug_iterate(torch.from_numpy(J).to(DEV),
                                               torch.from_numpy(M).to(DEV), **p)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(G2.cpu().numpy(), exp["G2"])
            np.testing.assert_array_equal(Mk.cpu().numpy(), exp["M"])
            assert int(n.item()) == exp["n"]
            np.testing.assert_array_equal(Jn.cpu().numpy(), exp["Jnext"].astype(np.float32))
            log(f"iterate {J.shape} k={k}: n={exp['n']} ok")
            J = exp["Jnext"].astype(np.float32)
            M = exp["M"]


def compare_end_to_end(f, clean, mask, r):
    gm = mask.cpu().numpy()
    gc = clean.cpu().numpy().astype(np.float64)
    nmis = int((gm != r["mask"]).sum())
    rel = np.abs(gc - r["clean"]) / np.maximum(np.abs(r["clean"]), np.finfo(np.float64).tiny)
    log(f"end-to-end {f.img.shape}: flagged {int(gm.sum())}, mask mismatches {nmis}, "
        f"max rel diff {rel.max():.3g}")
    assert nmis == 0
    assert rel.max() <= 1e-5
    assert (gc[r["clean"] == 0] == 0).all()


@pytest.mark.parametrize("early_stop", [True, False])
def test_end_to_end_small(early_stop):
    for f in small_frames():
        img = torch.from_numpy(f.img).to(DEV)
        clean, mask = _lib.lacosmic(img, niter=4, early_stop=early_stop, **fparams(f))
        torch.cuda.synchronize()
        r = ref.lacosmic(f.img, niter=4, early_stop=early_stop, **fparams(f))
        compare_end_to_end(f, clean, mask, r)


@pytest.mark.parametrize("tile_h", [16, 32, 64])
def test_crowded_tiles_overflow_lists(tile_h):
    """A frame with 15% of its pixels hit: tiles hold more work-set pixels than the
    block's list (8 rows' worth) and more contrast pixels than its contrast list, so
    the bitmap and in-lane fallbacks run; codes and four iterations equal the oracle's
    under each detection tile height."""
    f = synth.render(128, 192, 77, sky_e=100.0, gain=2.0, readnoise=5.0, n_stars=40,
                     star_fwhm=2.0, star_flux="lognormal", hit_coverage=0.15, hit_len=(1, 8),
                     hit_amp=(200.0, 5000.0))
    p = fparams(f)
    tr = ref.iterate(f.img, np.zeros(f.img.shape, np.uint8), trace=True, **p)
    near = dilate(tr["s"] > p["sigclip"], 2)
    work = near & (tr["s"] > np.float64(np.float32(p["sigfrac"])) * p["sigclip"])
    most = max(int(work[y:y + tile_h, x:x + 64].sum())
               for y in range(0, 128, tile_h) for x in range(0, 192, 64))
    assert most > 8 * tile_h, most          # the list overflows in some tile
    try:
        _lib.set_single_tuning(tile_h, 0, 0)
        img = torch.from_numpy(f.img).to(DEV)
        codes = _lib.debug_detect(img, **p)
        clean, mask = _lib.lacosmic(img, niter=4, early_stop=False, **p)
        torch.cuda.synchronize()
    finally:
        _lib.set_single_tuning(32, 0, 0)
    check_codes(codes.cpu().numpy(), expected_codes(tr, p), near, tr, f"crowded t{tile_h}")
    r = ref.lacosmic(f.img, niter=4, early_stop=False, **p)
    compare_end_to_end(f, clean, mask, r)


EXTREMES = [
    dict(sigclip=1.5),                       # many hot pixels: a dense work set
    dict(sigclip=50.0),                      # none
    dict(sigfrac=0.0), dict(sigfrac=1.0),
    dict(objlim=0.01), dict(objlim=1e4),
    dict(readnoise=0.0, sky=-300.0),         # m <= 0 everywhere: the 1e-4 noise floor
    dict(readnoise=0.0, sky=0.0),
    dict(gain=0.05), dict(gain=50.0),
    dict(niter=1), dict(niter=2), dict(niter=7),
]


@pytest.mark.parametrize("over", EXTREMES, ids=[",".join(f"{k}={v}" for k, v in o.items())
                                               for o in EXTREMES])
def test_parameter_extremes(over):
    frames = [synth.c1_density_frame(97, 130, 91, 2.0, 5.0)]
    neg = synth.c1_density_frame(70, 90, 92, 1.0, 4.0)
    neg.img = (neg.img - np.float32(100.0)).astype(np.float32)     # sky-subtracted frame
    frames.append(neg)
    for f in frames:
        p = fparams(f)
        niter = over.get("niter", 4)
        p.update({k: f32(v) for k, v in over.items() if k != "niter"})
        img = torch.from_numpy(f.img).to(DEV)
        clean, mask = _lib.lacosmic(img, niter=niter, early_stop=False, **p)
        torch.cuda.synchronize()
        r = ref.lacosmic(f.img, niter=niter, early_stop=False, **p)
        compare_end_to_end(f, clean, mask, r)


def test_niter_zero_constant_and_in_place():
    f = synth.c1()
    img = torch.from_numpy(f.img).to(DEV)
    clean, mask = _lib.lacosmic(img, niter=0, **fparams(f))
    torch.cuda.synchronize()
    assert torch.equal(clean, img) and int(mask.sum()) == 0
    for v in (24.3, 137.0):
        c = torch.full((50, 70), v, dtype=torch.float32, device=DEV)
        cl, m = _lib.lacosmic(c, 7.0, 5.0, sigfrac=0.3, objlim=4.0, niter=4)
        torch.cuda.synchronize()
        assert torch.equal(cl, c) and int(m.sum()) == 0
    work = img.clone()
    cl, m = _lib.lacosmic(work, out_clean=work, niter=4, **fparams(f))
    cl2, m2 = _lib.lacosmic(img, niter=4, **fparams(f))
    torch.cuda.synchronize()
    assert torch.equal(cl, cl2) and torch.equal(m, m2)


def make_items(frames, early_stop=True):
    items = []
    for f in frames:
        img = torch.from_numpy(f.img).to(DEV)
        items.append(dict(img=img, out_clean=torch.empty_like(img),
                          out_mask=torch.empty(img.shape, dtype=torch.uint8, device=DEV),
                          niter=f.niter, early_stop=early_stop, **fparams(f)))
    return items


def test_batched_matches_solo_and_oracle_counts():
    frames = small_frames()
    frames[2].gain, frames[2].readnoise = 3.25, 6.5
    frames[4].niter = 2
    items = make_items(frames)
    stats = _lib.lacosmic_batched(items)
    for f, it, st in zip(frames, items, stats):
        c, m = _lib.lacosmic(it["img"], niter=f.niter, **fparams(f))
        torch.cuda.synchronize()
        assert torch.equal(c, it["out_clean"]) and torch.equal(m, it["out_mask"])
        r = ref.lacosmic(f.img, niter=f.niter, **fparams(f))
        assert st["iters_run"] == r["iters"], (st, r["iters"])
        assert st["n_flagged"] == int(r["mask"].sum())


def edge_frames():
    """Frames wider than one grow strip (992 px) and taller than a row of detection tiles,
    with c2's dense, long hits: iterations 2-4 flag hundreds of new pixels, many of them
    next to pixels flagged before and on either side of strip and tile edges."""
    return [synth.render(H, W, seed, sky_e=50.0, gain=7.0, readnoise=5.0, n_stars=40,
                         star_fwhm=1.5, star_flux="lognormal", hit_coverage=0.02,
                         hit_len=(1, 20), hit_amp=(100.0, 10000.0), name=f"{H}x{W}")
            for (H, W, seed) in [(96, 2000, 61), (100, 1993, 62)]]


def test_later_iterations_near_strip_and_tile_edges():
    """After iteration 1 the grow runs only on strips within reach of A (8-row strips on
    the batched path) and the replacement only near new flags: whole 4-iteration runs,
    solo and batched, equal the oracle on frames where that matters at the edges."""
    frames = edge_frames()
    for f in frames:
        # from the oracle alone: later iterations add flags on tile edges
        J, M = f.img.astype(np.float64), np.zeros(f.img.shape, np.uint8)
        at_edges = 0
        for k in range(1, 5):
            r = ref.iterate(J, M, **fparams(f))
            ys, xs = np.nonzero((r["G2"] != 0) & (M == 0))
            if k >= 2:
                at_edges += int(((ys % 32 < 3) | (ys % 32 > 28) | (xs % 64 < 3) |
                                 (xs % 64 > 60)).sum())
            J, M = r["Jnext"], r["M"]
        assert at_edges > 100, (f.name, at_edges)
    items = make_items(frames, early_stop=False)
    _lib.lacosmic_batched(items)
    for f, it in zip(frames, items):
        log(f"edge frame {f.name}")
        r = ref.lacosmic(f.img, niter=4, early_stop=False, **fparams(f))
        c, m = _lib.lacosmic(it["img"], niter=4, early_stop=False, **fparams(f))
        torch.cuda.synchronize()
        compare_end_to_end(f, c, m, r)
        compare_end_to_end(f, it["out_clean"], it["out_mask"], r)


def test_plan_graph_replays_match_solo():
    frames = small_frames()[:4]
    items = make_items(frames, early_stop=False)
    plan = _lib.Plan(items, use_graph=True)
    for rep in range(3):
        for it in items:
            it["out_clean"].fill_(-1.0)
            it["out_mask"].fill_(7)
        plan.run()
        stats = plan.stats()
        _ = torch.randn(1000, device=DEV).sum().item()       # eager work between replays
        for f, it, st in zip(frames, items, stats):
            c, m = _lib.lacosmic(it["img"], niter=4, early_stop=False, **fparams(f))
            torch.cuda.synchronize()
            assert torch.equal(c, it["out_clean"]), rep
            assert torch.equal(m, it["out_mask"]), rep
            assert st["iters_run"] == 4
    plan.close()


def sampled_windows(H, W, rng, n=6, size=16):
    pts = [(0, 0), (H - size, W - size), (0, W - size), (H - size, 0)]
    while len(pts) < n:
        pts.append((int(rng.integers(0, H - size)), int(rng.integers(0, W - size))))
    return pts


def check_sampled(f, clean, mask, niter, size=16):
    """Oracle on crops with a halo of 8 px per iteration: the crop interior is exact."""
    rng = np.random.default_rng(f.seed)
    H, W = f.img.shape
    halo = 8 * niter
    gm = mask.cpu().numpy()
    gc = clean.cpu().numpy()
    for (y, x) in sampled_windows(H, W, rng, size=size):
        a0, a1 = max(0, y - halo), min(H, y + size + halo)
        b0, b1 = max(0, x - halo), min(W, x + size + halo)
        r = ref.lacosmic(np.ascontiguousarray(f.img[a0:a1, b0:b1]), niter=niter,
                         early_stop=False, **fparams(f))
        em = r["mask"][y - a0:y - a0 + size, x - b0:x - b0 + size]
        ec = r["clean"][y - a0:y - a0 + size, x - b0:x - b0 + size]
        np.testing.assert_array_equal(gm[y:y + size, x:x + size], em, err_msg=str((y, x)))
        np.testing.assert_allclose(gc[y:y + size, x:x + size].astype(np.float64), ec, rtol=1e-5,
                                   atol=0, err_msg=str((y, x)))


def test_full_size_4096_sampled():
    f = synth.c3()
    img = torch.from_numpy(f.img).to(DEV)
    clean, mask = _lib.lacosmic(img, niter=4, early_stop=False, **fparams(f))
    torch.cuda.synchronize()
    log(f"c3 4096x4096: flagged {int(mask.sum())} ({int(f.hits.sum())} hit pixels)")
    check_sampled(f, clean, mask, 4)


def test_mixed_batch_sampled():
    frames = [synth.c1_density_frame(800, 800, 4000, 3.5, 4.25),
              synth.c1_density_frame(2048, 4096, 4032, 6.75, 7.5),
              synth.c1_density_frame(1024, 1024, 4016, 1.25, 3.0)]
    items = make_items(frames, early_stop=False)
    plan = _lib.Plan(items, use_graph=True)
    plan.run()
    plan.stats()
    for f, it in zip(frames, items):
        check_sampled(f, it["out_clean"], it["out_mask"], 4)
    plan.close()


def test_calibration_copy_b32():
    """The counter-calibration copy (4-byte buffer loads) copies exactly, across its
    2^20-element chunks and a ragged tail."""
    for n in (1, 1000, (1 << 20) + 7, 3 * (1 << 20)):
        src = torch.arange(n, dtype=torch.float32, device=DEV) * 0.5
        dst = torch.full_like(src, -1.0)
        _lib.debug_copy_b32(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst), n
