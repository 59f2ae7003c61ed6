"""GPU tile farm with the SOURCES work function (the paper's example of actors that
return structures, Section 7): the records found on the GPU equal the oracle's,
field by field and bit for bit, for any tile shape, worker count and radius; the
list is complete and duplicate-free when truncated; POISSON on 2-D tiles still
matches the oracle."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_1008_2192_amd import _lib, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def gpu_sources(img, t, sky, r, a, **kw):
    lst = _lib.farm_sources(torch.from_numpy(np.ascontiguousarray(img)).to(DEV), t, sky, r, a,
                            **kw)
    torch.cuda.synchronize()
    return lst.numpy()


def oracle_sorted(img, t, sky, r, a):
    rec = ref.sources(img, t, sky, r, a)
    return rec.view(_lib.SOURCE_DTYPE)


def star_field(H, W, seed, n_peaks=60):
    rng = np.random.default_rng(seed)
    img = rng.normal(100.0, 5.0, (H, W)).astype(np.float32)
    if H * W >= 4:
        ys, xs = rng.integers(0, H, n_peaks), rng.integers(0, W, n_peaks)
        img[ys, xs] += rng.uniform(20, 400, n_peaks).astype(np.float32)
    return img


@pytest.mark.parametrize("H,W,r,a,th,tw,workers", [
    (97, 131, 2, 2, 32, 64, 64), (97, 131, 1, 3, 7, 13, 5), (97, 131, 3, 0, 1, 131, 1000),
    (256, 256, 8, 8, 16, 16, 2048), (1, 3000, 2, 4, 1, 256, 7), (600, 1, 3, 2, 64, 1, 3),
    (1, 1, 1, 1, 32, 64, 1), (33, 65, 5, 1, 33, 65, 1), (64, 64, 2, 2, 200, 40, 2)])
def test_sources_match_oracle(H, W, r, a, th, tw, workers):
    img = star_field(H, W, H * 7 + W)
    exp = oracle_sorted(img, 115.0, 100.0, r, a)
    got = gpu_sources(img, 115.0, 100.0, r, a, tile_h=th, tile_w=tw, workers=workers)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("seed,r,a", [(1, 1, 1), (2, 2, 0), (3, 3, 3)])
def test_sources_many_ties(seed, r, a):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 4, (77, 90)).astype(np.float32)
    exp = oracle_sorted(img, 0.5, 1.0, r, a)
    assert len(exp) > 10
    for th, tw in [(32, 64), (5, 9), (77, 1)]:
        got = gpu_sources(img, 0.5, 1.0, r, a, tile_h=th, tile_w=tw, workers=37)
        assert np.array_equal(got, exp)


def test_sources_constant_and_empty():
    img = np.full((50, 70), 3.0, np.float32)
    got = gpu_sources(img, 1.0, 0.5, 2, 2)
    assert np.array_equal(got, oracle_sorted(img, 1.0, 0.5, 2, 2))
    assert len(got) == 1 and (got["y"][0], got["x"][0]) == (0, 0)
    lst = _lib.farm_sources(torch.from_numpy(img).to(DEV), 3.0, 0.0, 2, 2, capacity=0)
    torch.cuda.synchronize()
    assert int(lst.count.item()) == 0


def test_sources_truncated_list_is_a_subset():
    img = star_field(300, 300, 11, n_peaks=400)
    exp = oracle_sorted(img, 115.0, 100.0, 2, 2)
    assert len(exp) > 100
    cap = len(exp) // 3
    lst = _lib.farm_sources(torch.from_numpy(img).to(DEV), 115.0, 100.0, 2, 2, capacity=cap,
                            tile_h=16, tile_w=16, workers=64)
    torch.cuda.synchronize()
    assert int(lst.count.item()) == len(exp)
    with pytest.raises(OverflowError):
        lst.numpy()
    part = lst.records[: cap * _lib.SOURCE_DTYPE.itemsize].cpu().numpy().view(_lib.SOURCE_DTYPE)
    keys = set(zip(part["y"].tolist(), part["x"].tolist()))
    assert len(keys) == cap
    by_pos = {(int(e["y"]), int(e["x"])): e for e in exp}
    for p in part:
        assert p.tobytes() == by_pos[(int(p["y"]), int(p["x"]))].tobytes()


def test_sources_repeat_calls_reuse_buffers():
    img = star_field(128, 200, 5)
    exp = oracle_sorted(img, 115.0, 100.0, 2, 2)
    x = torch.from_numpy(img).to(DEV)
    lst = _lib.farm_sources(x, 115.0, 100.0, 2, 2)
    for th in (32, 8):
        _lib.farm_sources(x, 115.0, 100.0, 2, 2, tile_h=th, out=lst)
        torch.cuda.synchronize()
        assert np.array_equal(lst.numpy(), exp)


def test_sources_on_crowded_field_full_size():
    """The 4096 x 4096 crowded field (20,000 stars, 1.5% cosmic-ray coverage): peaks
    5 sigma above the sky, 7 x 7 apertures, in the farm's default launch shape."""
    f = synth.c3()
    sky = 200.0 / 1.5
    t = sky + 5.0 * np.sqrt(200.0 + 16.0) / 1.5
    exp = oracle_sorted(f.img, t, sky, 2, 3)
    assert len(exp) > 20000
    got = gpu_sources(f.img, t, sky, 2, 3)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("th,tw,workers", [(7, 13, 9), (1, 1, 2048), (64, 64, 3)])
def test_poisson_on_2d_tiles(th, tw, workers):
    rng = np.random.default_rng(th * 100 + tw)
    x = rng.uniform(0, 40, (97, 131)).astype(np.float32)
    g = _lib.farm_image(_lib.CRB_WORK_POISSON, torch.from_numpy(x).to(DEV), seed=7,
                        workers=workers, tile_h=th, tile_w=tw)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g.cpu().numpy(), ref.poisson(x, 7))
