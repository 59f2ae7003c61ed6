"""GPU tests of the serving loop: every result is the same alone and in the mix,
admission respects the HBM budget and the slot limit, and a real-time trace drains."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_1008_2192_amd import _lib, serving, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def f32(x):
    return float(np.float32(x))


def mixed_frames():
    out = []
    for i, (H, W) in enumerate([(256, 256), (300, 517), (64, 1000), (800, 800), (129, 77),
                                (512, 1024), (33, 45), (700, 300)]):
        g = f32(1.0 + 0.8 * i)
        rn = f32(3.0 + 0.5 * i)
        out.append(synth.c1_density_frame(H, W, 900 + i, g, rn))
    return out


def solo(f):
    img = torch.from_numpy(f.img).to(DEV)
    c, m = _lib.lacosmic(img, f32(f.gain), f32(f.readnoise), niter=4)
    torch.cuda.synchronize()
    return c.cpu().numpy(), m.cpu().numpy()


def params(f):
    return dict(gain=f32(f.gain), readnoise=f32(f.readnoise), niter=4)


def test_results_identical_alone_and_in_the_mix():
    frames = mixed_frames()
    # a budget that holds about two large frames forces queueing and staggered rounds
    budget = 2 * _lib.workspace_bytes(800, 800) + 2 * 5 * 800 * 800 + (1 << 20)
    srv = serving.Server(budget, max_slots=3)
    ids = {srv.submit(f.img, **params(f)): i for i, f in enumerate(frames)}
    done = srv.drain()
    srv.close()
    assert len(done) == len(frames)
    for rid, lat, clean, mask in done:
        f = frames[ids[rid]]
        c, m = solo(f)
        np.testing.assert_array_equal(clean, c)
        np.testing.assert_array_equal(mask, m)
        assert lat > 0
    # alone in a fresh server
    f = frames[3]
    srv = serving.Server(1 << 34, max_slots=8)
    srv.submit(f.img, **params(f))
    (rid, lat, clean, mask), = srv.drain()
    srv.close()
    c, m = solo(f)
    np.testing.assert_array_equal(clean, c)
    np.testing.assert_array_equal(mask, m)


def test_matches_oracle_small():
    f = synth.c1()
    srv = serving.Server(1 << 32)
    srv.submit(f.img, **params(f))
    (rid, lat, clean, mask), = srv.drain()
    srv.close()
    r = ref.lacosmic(f.img, f32(f.gain), f32(f.readnoise), niter=4)
    np.testing.assert_array_equal(mask, r["mask"])
    np.testing.assert_allclose(clean.astype(np.float64), r["clean"], rtol=1e-5, atol=0)


def test_oversized_frame_refused_and_niter_zero():
    srv = serving.Server(1 << 20, max_slots=2)
    with pytest.raises(_lib.CrbError) as e:
        srv.submit(np.zeros((512, 512), np.float32), 1.0, 5.0)
    assert e.value.status == -5
    img = np.arange(100, dtype=np.float32).reshape(10, 10)
    srv.submit(img, 1.0, 5.0, niter=0)
    (rid, lat, clean, mask), = srv.drain()
    np.testing.assert_array_equal(clean, img)
    assert mask.sum() == 0
    srv.close()


def test_realtime_trace_drains():
    frames = mixed_frames()
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(1 / 200.0, 24))
    fr = [frames[i % len(frames)].img for i in range(24)]
    pr = [params(frames[i % len(frames)]) for i in range(24)]
    srv = serving.Server(1 << 34, max_slots=16)
    res = serving.replay(srv, arrivals, fr, pr, keep_results=True)
    srv.close()
    s = res.summary()
    print(s, flush=True)
    assert s["requests"] == 24 and len(res.results) == 24
    for j in (0, 3, 5):
        c, m = solo(frames[j % len(frames)])
        np.testing.assert_array_equal(res.results[j][0], c)
        np.testing.assert_array_equal(res.results[j][1], m)


def test_pinned_buffers_transfer_directly():
    frames = mixed_frames()[:4]
    srv = serving.Server(1 << 34, max_slots=4)
    ids = {srv.submit(torch.from_numpy(f.img).pin_memory(), **params(f)): i
           for i, f in enumerate(frames)}
    done = srv.drain()
    srv.close()
    assert len(done) == len(frames)
    for rid, lat, clean, mask in done:
        c, m = solo(frames[ids[rid]])
        np.testing.assert_array_equal(clean, c)
        np.testing.assert_array_equal(mask, m)


def test_device_resident_requests_identical_and_mixed_with_host_ones():
    """Requests whose image and outputs are device memory (the host link out of the way)
    give the same results as host requests and as solo runs, also when both kinds share
    rounds; mixing host and device buffers in one request is refused."""
    frames = mixed_frames()
    budget = 3 * _lib.workspace_bytes(800, 800) + 3 * 5 * 800 * 800 + (1 << 20)
    srv = serving.Server(budget, max_slots=4)
    ids = {}
    for i, f in enumerate(frames):
        src = torch.from_numpy(f.img).to(DEV) if i % 2 == 0 else f.img
        ids[srv.submit(src, **params(f))] = i
    torch.cuda.synchronize()
    done = srv.drain()
    assert len(done) == len(frames)
    for rid, lat, clean, mask in done:
        i = ids[rid]
        c, m = solo(frames[i])
        if i % 2 == 0:
            assert clean.is_cuda and mask.is_cuda
            clean, mask = clean.cpu().numpy(), mask.cpu().numpy()
        np.testing.assert_array_equal(clean, c)
        np.testing.assert_array_equal(mask, m)
    f = frames[0]
    img = torch.from_numpy(f.img).to(DEV)
    host_out = np.empty(f.img.shape, np.float32)
    dev_mask = torch.empty(f.img.shape, dtype=torch.uint8, device=DEV)
    import ctypes
    rid = ctypes.c_int64(0)
    st = _lib.lib().crb_server_submit(srv.handle, img.data_ptr(), f.img.shape[0], f.img.shape[1],
                                      f32(f.gain), f32(f.readnoise), 0.0, 4.5, 0.3, 4.0, 4,
                                      host_out.ctypes.data, dev_mask.data_ptr(), ctypes.byref(rid))
    assert st == -1
    srv.close()
