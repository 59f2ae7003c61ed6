"""Incremental detection (CRB_FLAG_INCREMENTAL / CRB_OPT_INCREMENTAL) gives results
bit-identical to the full re-run of every iteration, through every entry point that
offers it, while evaluating fewer work-set pixels."""
import numpy as np
import pytest
import torch

from paper_1008_2192_amd import _lib, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def f32(x):
    return float(np.float32(x))


def frames():
    out = [synth.c1(), synth.c1_density_frame(300, 417, 61, 2.5, 6.0),
           synth.c1_density_frame(33, 97, 62, 1.0, 5.0), synth.c1_density_frame(1, 70, 63, 1.0, 5.0)]
    c2 = synth.c2()
    c2.img = np.ascontiguousarray(c2.img[:260, :333])
    out.append(c2)
    return out


def items_for(fs, incremental, niter=4):
    items = []
    for f in fs:
        img = torch.from_numpy(f.img).to(DEV)
        items.append(dict(img=img, out_clean=torch.empty_like(img),
                          out_mask=torch.empty(img.shape, dtype=torch.uint8, device=DEV),
                          gain=f32(f.gain), readnoise=f32(f.readnoise), sky=f32(f.sky),
                          sigclip=f32(f.sigclip), sigfrac=f32(f.sigfrac), objlim=f32(f.objlim),
                          niter=niter, early_stop=False, incremental=incremental))
    return items


@pytest.mark.parametrize("niter", [4, 7])
@pytest.mark.parametrize("use_graph", [False, True])
def test_plan_incremental_identical(niter, use_graph):
    fs = frames()
    full, inc = items_for(fs, False, niter), items_for(fs, True, niter)
    pf = _lib.Plan(full, use_graph=False)
    pi = _lib.Plan(inc, use_graph=use_graph)
    pf.set_counting(True)
    pi.set_counting(True)
    pf.run()
    pi.run()
    wf, wi = pf.work_counts(), pi.work_counts()
    sf, si = pf.stats(), pi.stats()
    pi.run()            # a second run (a graph replay when captured) starts afresh
    torch.cuda.synchronize()
    si2 = pi.stats()
    pf.close()
    pi.close()
    for a, b in zip(full, inc):
        assert torch.equal(a["out_mask"], b["out_mask"])
        assert torch.equal(a["out_clean"].view(torch.int32), b["out_clean"].view(torch.int32))
    assert sf == si == si2
    print(f"work pixels full {wf['work_pixels']}, incremental {wi['work_pixels']}", flush=True)
    assert wi["work_pixels"] < wf["work_pixels"]


def test_single_frame_and_partitioned_incremental_identical():
    f = synth.c2()
    img = torch.from_numpy(np.ascontiguousarray(f.img[:300, :400])).to(DEV)
    p = dict(gain=f32(f.gain), readnoise=f32(f.readnoise), sky=f32(f.sky),
             sigclip=f32(f.sigclip), sigfrac=f32(f.sigfrac), objlim=f32(f.objlim))
    c0, m0 = _lib.lacosmic(img, niter=5, early_stop=False, **p)
    c1, m1 = _lib.lacosmic(img, niter=5, early_stop=False, incremental=True, **p)
    pc0, pm0 = _lib.lacosmic_partitioned(img, ny=2, nx=3, border=40, niter=5, **p)
    pc1, pm1 = _lib.lacosmic_partitioned(img, ny=2, nx=3, border=40, niter=5, incremental=True,
                                         **p)
    _lib.lacosmic(img, niter=1, incremental=False, **p)     # leave the option off
    torch.cuda.synchronize()
    assert torch.equal(m0, m1) and torch.equal(c0.view(torch.int32), c1.view(torch.int32))
    assert torch.equal(pm0, pm1) and torch.equal(pc0.view(torch.int32), pc1.view(torch.int32))
