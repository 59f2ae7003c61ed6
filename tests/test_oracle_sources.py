"""Pins of the oracle's SOURCES work function (the paper's example of a work
function returning structures instead of subimages, Section 7): closed forms on
constant and symmetric images, a brute force over shifted copies of tiny images
with many ties, the separation rule, strictness of the threshold, and invariance
under a partition into subimages whose border is the declared radius max(r, a)."""
import numpy as np
import pytest

from oracle import ref


def shifted(img, dy, dx, fill):
    """out[y, x] = img[y + dy, x + dx], `fill` outside the frame."""
    H, W = img.shape
    out = np.full((H, W), fill, dtype=np.float64)
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    if ys < ye and xs < xe:
        out[ys:ye, xs:xe] = img[ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def brute_sources(img, t, sky, r, a):
    """Whole-array formulation: a pixel is a peak when every offset within r passes
    (smaller value, or equal value at an offset that is later in raster order)."""
    v = img.astype(np.float64)
    peak = v > t
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dy == 0 and dx == 0:
                continue
            q = shifted(v, dy, dx, -np.inf)
            later = dy > 0 or (dy == 0 and dx > 0)
            peak &= (q < v) | ((q == v) if later else False)
    flux = np.zeros_like(v)
    sy = np.zeros_like(v)
    sx = np.zeros_like(v)
    npix = np.zeros(v.shape, np.int64)
    for dy in range(-a, a + 1):
        for dx in range(-a, a + 1):
            inside = shifted(np.ones_like(v), dy, dx, 0.0)
            d = (shifted(v, dy, dx, 0.0) - sky) * inside
            flux += d
            sy += dy * d
            sx += dx * d
            npix += inside.astype(np.int64)
    ys, xs = np.nonzero(peak)
    return [(int(y), int(x), float(v[y, x]), int(npix[y, x]), float(flux[y, x]),
             float(sy[y, x]), float(sx[y, x])) for y, x in zip(ys, xs)]


def as_tuples(rec):
    return [(int(s["y"]), int(s["x"]), float(s["peak"]), int(s["npix"]), float(s["flux"]),
             float(s["sy"]), float(s["sx"])) for s in rec]


@pytest.mark.parametrize("H,W,r,a", [(1, 1, 1, 0), (1, 9, 2, 3), (7, 1, 3, 1), (6, 7, 2, 2),
                                     (20, 13, 8, 8)])
def test_constant_frame_has_one_source_at_origin(H, W, r, a):
    c, sky = 7.0, 2.0
    rec = ref.sources(np.full((H, W), c, np.float32), 1.0, sky, r, a)
    assert len(rec) == 1 and rec["y"][0] == 0 and rec["x"][0] == 0
    ny, nx = min(a + 1, H), min(a + 1, W)           # in-frame part of the aperture
    assert rec["npix"][0] == ny * nx
    assert rec["flux"][0] == ny * nx * (c - sky)
    assert rec["sy"][0] == nx * (c - sky) * (ny - 1) * ny / 2
    assert rec["sx"][0] == ny * (c - sky) * (nx - 1) * nx / 2


@pytest.mark.parametrize("seed,r,a", [(1, 1, 0), (2, 1, 2), (3, 2, 1), (4, 3, 3), (5, 2, 4),
                                      (6, 4, 0)])
def test_brute_force_with_ties(seed, r, a):
    rng = np.random.default_rng(seed)
    H, W = rng.integers(1, 17, 2)
    img = rng.integers(0, 4, (H, W)).astype(np.float32)   # values 0..3: many ties
    got = as_tuples(ref.sources(img, 0.5, 1.0, r, a))
    assert got == brute_sources(img, 0.5, 1.0, r, a)


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_real_valued(seed):
    rng = np.random.default_rng(100 + seed)
    img = rng.normal(0, 1, (24, 31)).astype(np.float32)
    rec = ref.sources(img, 1.0, 0.25, 2, 2)
    exp = brute_sources(img, 1.0, 0.25, 2, 2)
    assert [(s[0], s[1], s[2], s[3]) for s in as_tuples(rec)] == [e[:4] for e in exp]
    for s, e in zip(as_tuples(rec), exp):          # sums in another order: within rounding
        assert s[4:] == pytest.approx(e[4:], rel=1e-12, abs=1e-12)


def test_symmetric_star():
    """A centred integer profile: one source at its centre, zero first moments, and
    the aperture sums the closed-form total of the profile inside the box."""
    prof = np.array([1, 4, 9, 4, 1], np.float64)
    img = np.zeros((21, 25), np.float32)
    img[8:13, 10:15] = 10.0 * np.outer(prof, prof)
    rec = ref.sources(img, 5.0, 0.0, 3, 2)
    assert len(rec) == 1
    s = rec[0]
    assert (s["y"], s["x"], s["peak"]) == (10, 12, 810.0)
    assert s["flux"] == 10.0 * prof.sum() ** 2 and s["npix"] == 25
    assert s["sy"] == 0.0 and s["sx"] == 0.0
    rec1 = ref.sources(img, 5.0, 0.0, 3, 1)            # inner 3x3 only
    assert rec1[0]["flux"] == 10.0 * prof[1:4].sum() ** 2


@pytest.mark.parametrize("r", [1, 2, 5])
def test_separation_rule(r):
    """Two peaks at Chebyshev distance d: both are sources iff d > r; otherwise only
    the brighter, and on a tie the earlier in raster order."""
    for d in range(1, r + 3):
        for bright_second in (False, True):
            img = np.zeros((30, 30), np.float32)
            img[10, 10] = 50.0
            img[10 + d, 10 + (d // 2)] = 60.0 if bright_second else 50.0
            rec = ref.sources(img, 1.0, 0.0, r, 0)
            pos = [(int(s["y"]), int(s["x"])) for s in rec]
            if d > r:
                assert pos == [(10, 10), (10 + d, 10 + d // 2)]
            elif bright_second:
                assert pos == [(10 + d, 10 + d // 2)]
            else:
                assert pos == [(10, 10)]


def test_threshold_is_strict_and_plateau_first_pixel():
    img = np.zeros((12, 12), np.float32)
    img[3, 3] = 5.0
    img[7:9, 6:8] = 9.0                                 # 2x2 plateau
    assert [(s["y"], s["x"]) for s in ref.sources(img, 5.0, 0.0, 2, 0)] == [(7, 6)]
    assert [(s["y"], s["x"]) for s in ref.sources(img, np.nextafter(np.float32(5.0), 0), 0.0,
                                                  2, 0)] == [(3, 3), (7, 6)]
    assert len(ref.sources(img, 9.0, 0.0, 2, 0)) == 0


def test_capacity_truncates_but_counts():
    img = np.zeros((10, 40), np.float32)
    img[5, 2::4] = 3.0                                  # 10 separated peaks
    full = ref.sources(img, 1.0, 0.0, 1, 1)
    assert len(full) == 10
    import ctypes
    out = np.zeros(3, ref.SOURCE_DTYPE)
    cnt = ctypes.c_longlong(0)
    rc = ref.lib().crb_ref_sources(img.ctypes.data, 10, 40, 1.0, 0.0, 1, 1, out.ctypes.data, 3,
                                   ctypes.byref(cnt))
    assert rc == 0 and cnt.value == 10
    assert np.array_equal(out, full[:3])


def partitioned_sources(img, t, sky, r, a, ny, nx, border):
    """Split the frame into ny x nx rectangles, extend each by `border` pixels on its
    shared edges, run the work function on each extended subimage on its own, keep
    the records whose peak lies in the rectangle, and shift them to frame coordinates."""
    H, W = img.shape
    out = []
    for i in range(ny):
        for j in range(nx):
            y0, y1 = H * i // ny, H * (i + 1) // ny
            x0, x1 = W * j // nx, W * (j + 1) // nx
            a0, a1 = max(0, y0 - border), min(H, y1 + border)
            b0, b1 = max(0, x0 - border), min(W, x1 + border)
            for s in ref.sources(img[a0:a1, b0:b1], t, sky, r, a):
                y, x = int(s["y"]) + a0, int(s["x"]) + b0
                if y0 <= y < y1 and x0 <= x < x1:
                    s = s.copy()
                    s["y"], s["x"] = y, x
                    out.append(s)
    rec = np.array(out, ref.SOURCE_DTYPE)
    return rec[np.lexsort((rec["x"], rec["y"]))] if len(rec) else rec


@pytest.mark.parametrize("ny,nx,r,a", [(2, 3, 2, 2), (4, 1, 3, 1), (3, 3, 1, 4), (1, 6, 2, 0)])
def test_partition_with_declared_radius_is_exact(ny, nx, r, a):
    rng = np.random.default_rng(ny * 10 + nx)
    img = rng.normal(10.0, 3.0, (64, 72)).astype(np.float32)
    img[rng.integers(0, 64, 40), rng.integers(0, 72, 40)] += 30.0
    full = ref.sources(img, 16.0, 10.0, r, a)
    assert len(full) > 10
    part = partitioned_sources(img, 16.0, 10.0, r, a, ny, nx, max(r, a))
    assert np.array_equal(part, full)


def test_partition_with_short_border_differs():
    """A peak just inside a rectangle whose brighter neighbour lies one pixel beyond
    a border of r - 1 is (wrongly) reported; the declared radius r removes it."""
    img = np.zeros((16, 16), np.float32)
    img[5, 7] = 20.0          # rectangle 0 (columns 0..7)
    img[5, 10] = 30.0         # rectangle 1 (columns 8..15), distance 3 = r
    full = ref.sources(img, 1.0, 0.0, 3, 0)
    assert [(s["y"], s["x"]) for s in full] == [(5, 10)]
    short = partitioned_sources(img, 1.0, 0.0, 3, 0, 1, 2, 2)
    assert [(s["y"], s["x"]) for s in short] == [(5, 7), (5, 10)]
    assert np.array_equal(partitioned_sources(img, 1.0, 0.0, 3, 0, 1, 2, 3), full)


def test_invalid_arguments():
    img = np.zeros((4, 4), np.float32)
    for r, a in [(0, 1), (9, 1), (1, -1), (1, 9)]:
        with pytest.raises(ValueError):
            ref.sources(img, 1.0, 0.0, r, a)
    with pytest.raises(ValueError):
        ref.sources(img, float("nan"), 0.0, 1, 1)
