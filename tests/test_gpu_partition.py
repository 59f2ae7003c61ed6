"""GPU partitioned runs (the paper's subimages with a border) against the oracle's
stitched subimage runs, and exactness once the border covers the dependency radius."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_1008_2192_amd import _lib, synth
from tests.test_oracle_pins import stitched

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("ny,nx,border", [(2, 2, 0), (1, 7, 6), (2, 3, 3), (3, 2, 32), (4, 1, 8)])
def test_partitioned_matches_oracle_subimages(ny, nx, border):
    f = synth.render(96, 112, 21, sky_e=100.0, gain=1.0, readnoise=5.0, n_stars=8,
                     star_fwhm=2.0, star_flux="lognormal", n_hits=40, hit_len=(1, 5),
                     hit_amp=(200.0, 5000.0))

    def fn(sub, _):
        r = ref.lacosmic(sub, 1.0, 5.0, niter=4)
        return dict(clean=r["clean"], mask=r["mask"])

    exp = stitched(f.img, ny, nx, border, fn)
    c, m = _lib.lacosmic_partitioned(torch.from_numpy(f.img).to(DEV), 1.0, 5.0, ny, nx, border)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(m.cpu().numpy(), exp["mask"])
    np.testing.assert_allclose(c.cpu().numpy().astype(np.float64), exp["clean"], rtol=1e-5, atol=0)


def test_border_32_equals_unpartitioned():
    f = synth.c2()
    img = torch.from_numpy(f.img).to(DEV)
    c0, m0 = _lib.lacosmic(img, f.gain, f.readnoise, niter=4)
    for ny, nx in [(2, 4), (6, 6), (1, 36)]:
        c, m = _lib.lacosmic_partitioned(img, f.gain, f.readnoise, ny, nx, 32)
        torch.cuda.synchronize()
        assert torch.equal(m, m0) and torch.equal(c, c0), (ny, nx)
