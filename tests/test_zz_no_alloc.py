"""The allocation-free entry point (crb_lacosmic_noalloc) against crb_lacosmic, through
the C ABI: two calls in a row on the shared device scratch, the second on a smaller
frame, each bit-identical to crb_lacosmic (masks and cleaned images), and the first
also checked against the FP64 oracle to the parity bar (masks bit-exact, cleaned image
within 1e-5 relative)."""
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
    return dict(gain=f32(f.gain), readnoise=f32(f.readnoise), sky=f32(f.sky),
                sigclip=f32(f.sigclip), sigfrac=f32(f.sigfrac), objlim=f32(f.objlim))


def run_both(f, early_stop):
    img = torch.from_numpy(f.img).to(DEV)
    p = fparams(f)
    # poison the outputs so that an unwritten pixel shows
    c_na = torch.full_like(img, -7.0)
    m_na = torch.full(img.shape, 9, dtype=torch.uint8, device=DEV)
    _lib.lacosmic_noalloc(img, niter=4, out_clean=c_na, out_mask=m_na, early_stop=early_stop,
                          **p)
    c_ref, m_ref = _lib.lacosmic(img, niter=4, early_stop=early_stop, **p)
    torch.cuda.synchronize()
    return c_na, m_na, c_ref, m_ref


@pytest.mark.parametrize("early_stop", [False, True])
def test_noalloc_matches_crb_lacosmic_twice_second_smaller(early_stop):
    first = synth.c2()
    first.img = np.ascontiguousarray(first.img[:400, :517])
    second = synth.c1_density_frame(97, 65, 38, 1.0, 5.0)
    for i, f in enumerate((first, second)):
        print(f"noalloc call {i}: {f.img.shape} early_stop={early_stop}", flush=True)
        c_na, m_na, c_ref, m_ref = run_both(f, early_stop)
        assert torch.equal(m_na, m_ref), f"mask differs on call {i}"
        assert torch.equal(c_na, c_ref), f"cleaned image differs on call {i}"
        if i == 0:
            r = ref.lacosmic(f.img, niter=4, early_stop=early_stop, **fparams(f))
            np.testing.assert_array_equal(m_na.cpu().numpy(), r["mask"])
            np.testing.assert_allclose(c_na.cpu().numpy().astype(np.float64), r["clean"],
                                       rtol=1e-5, atol=0)
        assert int(m_na.sum()) > 0, "the frame should have flagged pixels"


def test_noalloc_rejects_frames_beyond_the_scratch():
    img = torch.zeros((8, 8), dtype=torch.float32, device=DEV)
    big_h, big_w = 6000, 6000       # about 180 MB of workspace
    L = _lib.lib()
    st = L.crb_lacosmic_noalloc(img.data_ptr(), big_h, big_w, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4,
                                img.data_ptr() + (1 << 30), img.data_ptr() + (1 << 31))
    assert st == -4
    assert b"scratch" in L.crb_last_error()
