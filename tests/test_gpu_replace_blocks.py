"""The replacement reads a pixel's window as aligned 8-pixel row blocks only where J (the
caller's out_clean) starts on a 16-byte boundary and the mask (out_mask) on a 4-byte one,
and the blocks lie inside the frame; everywhere else it loads the 25 clamped positions one
by one.  Output buffers at every offset give the aligned run's masks and cleaned images
bit for bit, and the aligned run matches the FP64 oracle.  Widths that are and are not
multiples of 4 make the blocks start at every offset within a row; hits on the frame's
last rows and columns take the per-pixel path next to block pixels.
"""
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


def frames():
    out = [synth.c1_density_frame(130, 67, 51, 2.0, 5.0),
           synth.c1_density_frame(96, 256, 52, 4.0, 3.0)]
    # hits on the last rows and columns: per-pixel windows beside block windows
    f = synth.c1_density_frame(61, 75, 53, 1.5, 4.0)
    img = f.img.copy()
    img[-1, 10:14] += 4000.0
    img[30, -2:] += 3000.0
    img[-2:, -1] += 5000.0
    f.img = np.ascontiguousarray(img)
    out.append(f)
    return out


@pytest.fixture(scope="module")
def aligned_runs():
    runs = []
    for f in frames():
        img = torch.from_numpy(f.img).to(DEV)
        c, m = _lib.lacosmic(img, niter=4, early_stop=False, **fparams(f))
        torch.cuda.synchronize()
        r = ref.lacosmic(f.img, niter=4, early_stop=False, **fparams(f))
        np.testing.assert_array_equal(m.cpu().numpy(), r["mask"], err_msg=str(f.img.shape))
        np.testing.assert_allclose(c.cpu().numpy().astype(np.float64), r["clean"], rtol=1e-5,
                                   atol=0, err_msg=str(f.img.shape))
        runs.append((f, c.clone(), m.clone()))
    return runs


# (out_clean offset in floats, out_mask offset in bytes): 4 floats keep J on a 16-byte
# boundary at another base; the others take the per-pixel path
@pytest.mark.parametrize("j_off,m_off", [(4, 0), (1, 0), (2, 0), (3, 0), (0, 1), (0, 2),
                                         (4, 4), (1, 3)])
def test_outputs_at_any_offset(aligned_runs, j_off, m_off):
    for f, c_ref, m_ref in aligned_runs:
        H, W = f.img.shape
        img = torch.from_numpy(f.img).to(DEV)
        cbuf = torch.full((H * W + 8,), -1.0, dtype=torch.float32, device=DEV)
        mbuf = torch.full((H * W + 8,), 7, dtype=torch.uint8, device=DEV)
        out_c = cbuf[j_off:j_off + H * W].view(H, W)
        out_m = mbuf[m_off:m_off + H * W].view(H, W)
        assert out_c.data_ptr() % 16 == (0 if j_off % 4 == 0 else 4 * (j_off % 4))
        _lib.lacosmic(img, niter=4, early_stop=False, out_clean=out_c, out_mask=out_m,
                      **fparams(f))
        torch.cuda.synchronize()
        assert torch.equal(out_m, m_ref), (f.img.shape, j_off, m_off)
        assert torch.equal(out_c, c_ref), (f.img.shape, j_off, m_off)
        # nothing written outside the views
        assert bool((cbuf[:j_off] == -1.0).all()) and bool((cbuf[j_off + H * W:] == -1.0).all())
        assert bool((mbuf[:m_off] == 7).all()) and bool((mbuf[m_off + H * W:] == 7).all())
