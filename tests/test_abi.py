"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
symbol include/crb.h declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crb.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(crb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1008_2192_amd import _lib
    return _lib.lib()


def test_header_symbols_exported(L):
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    from paper_1008_2192_amd import _lib
    assert sorted(_lib.EXPORTS) == names


def test_frame_struct_layout():
    from paper_1008_2192_amd import _lib
    assert ctypes.sizeof(_lib.Frame) == 80
    assert _lib.Frame.n_flagged.offset == 72


def test_invalid_arguments_rejected_on_host(L):
    from paper_1008_2192_amd import _lib
    p = ctypes.c_void_p(16)        # never dereferenced: validation fails first
    q = ctypes.c_void_p(1 << 40)
    m = ctypes.c_void_p(1 << 41)
    cases = [
        (0, 10, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4, -1),      # H < 1
        (10, 0, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4, -1),      # W < 1
        (65536, 65536, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4, -4),  # too many pixels
        (10, 10, 0.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4, -1),     # gain
        (10, 10, 1.0, -1.0, 0.0, 4.5, 0.3, 4.0, 4, -1),    # read noise
        (10, 10, 1.0, 5.0, 0.0, 0.0, 0.3, 4.0, 4, -1),     # sigclip
        (10, 10, 1.0, 5.0, 0.0, 4.5, 1.5, 4.0, 4, -1),     # sigfrac
        (10, 10, 1.0, 5.0, 0.0, 4.5, 0.3, 0.0, 4, -1),     # objlim
        (10, 10, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, -1, -1),    # niter
        (10, 10, float("nan"), 5.0, 0.0, 4.5, 0.3, 4.0, 4, -1),
        (10, 10, 1.0, 5.0, float("inf"), 4.5, 0.3, 4.0, 4, -1),
    ]
    for H, W, g, rn, sky, sc, sf, ol, ni, expect in cases:
        st = L.crb_lacosmic(p, H, W, g, rn, sky, sc, sf, ol, ni, q, m)
        assert st == expect, (H, W, g, rn, sky, sc, sf, ol, ni, st)
        assert L.crb_last_error()
    # null pointers and overlapping buffers
    assert L.crb_lacosmic(None, 4, 4, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4, q, m) == -1
    assert L.crb_lacosmic(p, 4, 4, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4, ctypes.c_void_p(20), m) == -1
    assert L.crb_lacosmic(p, 4, 4, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4, q, ctypes.c_void_p(24)) == -1
    assert L.crb_set_option(99, 1) == -1
    assert L.crb_set_option(_lib.CRB_OPT_EARLY_STOP, 2) == -1
    assert L.crb_workspace_bytes(0, 5) == 0
    assert L.crb_workspace_bytes(100, 100) >= 100 * 100 * 5


def test_batched_rejects_bad_frames(L):
    from paper_1008_2192_amd import _lib
    arr = (_lib.Frame * 2)()
    for i in range(2):
        arr[i] = _lib.Frame(16 + i * 4096, (1 << 40) + i * 4096, (1 << 41) + i * 4096, 8, 8, 1.0,
                            5.0, 0.0, 4.5, 0.3, 4.0, 4, 0, 0, 0, 0)
    arr[1].sigfrac = 2.0
    assert L.crb_lacosmic_batched(arr, 2, None) == -1
    assert b"frame 1" in L.crb_last_error()
    arr[1].sigfrac = 0.3
    arr[1].out_clean = arr[0].out_clean            # two frames writing one buffer
    assert L.crb_lacosmic_batched(arr, 2, None) == -1
    assert L.crb_lacosmic_batched(arr, 0, None) == -1


def test_server_argument_validation(L):
    out = ctypes.c_void_p()
    assert L.crb_server_create(0, 4, ctypes.byref(out)) == -1
    assert L.crb_server_create(1 << 30, 0, ctypes.byref(out)) == -1
    rid = ctypes.c_int64()
    assert L.crb_server_submit(None, ctypes.c_void_p(16), 4, 4, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4,
                               ctypes.c_void_p(32), ctypes.c_void_p(48), ctypes.byref(rid)) == -1
    n = ctypes.c_int32()
    assert L.crb_server_poll(None, None, None, 0, ctypes.byref(n)) == -1
    assert L.crb_server_pending(None) == 0


def test_work_struct_layouts():
    from paper_1008_2192_amd import _lib
    assert ctypes.sizeof(_lib.Work) == 32
    assert _lib.Work.seed.offset == 8 and _lib.Work.aperture_radius.offset == 28
    assert _lib.SOURCE_DTYPE.itemsize == 40 and _lib.SOURCE_DTYPE.fields["flux"][1] == 16


def test_work_radius_declarations(L):
    from paper_1008_2192_amd import _lib
    assert _lib.work_radius(_lib.CRB_WORK_LACOSMIC, niter=4) == 32
    assert _lib.work_radius(_lib.CRB_WORK_LACOSMIC, niter=1) == 8
    assert _lib.work_radius(_lib.CRB_WORK_POISSON) == 0
    assert _lib.work_radius(_lib.CRB_WORK_WAITER) == 0
    assert _lib.work_radius(_lib.CRB_WORK_SOURCES, r=2, a=5) == 5
    assert _lib.work_radius(_lib.CRB_WORK_SOURCES, r=3, a=0) == 3
    for kw in [dict(kind=_lib.CRB_WORK_SOURCES, r=0), dict(kind=_lib.CRB_WORK_SOURCES, r=9),
               dict(kind=_lib.CRB_WORK_SOURCES, r=2, a=-1),
               dict(kind=_lib.CRB_WORK_SOURCES, r=2, threshold=float("inf")),
               dict(kind=_lib.CRB_WORK_LACOSMIC, niter=-1), dict(kind=9)]:
        w = _lib.make_work(**kw)
        assert L.crb_work_radius(ctypes.byref(w)) == -1, kw
        assert L.crb_last_error()
    assert L.crb_work_radius(None) == -1


def test_farm_argument_validation(L):
    from paper_1008_2192_amd import _lib
    src = _lib.make_work(_lib.CRB_WORK_SOURCES, threshold=1.0, r=2, a=2)
    poi = _lib.make_work(_lib.CRB_WORK_POISSON, seed=1)
    lac = _lib.make_work(_lib.CRB_WORK_LACOSMIC, niter=4)
    x = ctypes.c_void_p(1 << 40)          # never dereferenced: validation fails first
    img = ctypes.c_void_p(1 << 41)
    lst = ctypes.c_void_p(1 << 42)
    cnt = ctypes.c_void_p(1 << 43)
    run = L.crb_farm_run
    b = ctypes.byref
    assert run(b(lac), x, 8, 8, 4, 8, 8, img, None, 0, None) == -1
    assert run(None, x, 8, 8, 4, 8, 8, img, None, 0, None) == -1
    assert run(b(poi), None, 8, 8, 4, 8, 8, img, None, 0, None) == -1
    assert run(b(poi), x, 0, 8, 4, 8, 8, img, None, 0, None) == -1
    assert run(b(poi), x, 65536, 65536, 4, 8, 8, img, None, 0, None) == -4
    assert run(b(poi), x, 8, 8, 0, 8, 8, img, None, 0, None) == -1
    assert run(b(poi), x, 8, 8, (1 << 22) + 1, 8, 8, img, None, 0, None) == -1
    assert run(b(poi), x, 8, 8, 4, 0, 8, img, None, 0, None) == -1
    assert run(b(poi), x, 8, 8, 4, 8, 8, None, None, 0, None) == -1
    assert run(b(poi), x, 8, 8, 4, 8, 8, img, lst, 4, cnt) == -1
    assert run(b(poi), x, 8, 8, 4, 8, 8, ctypes.c_void_p((1 << 40) + 4), None, 0, None) == -1
    assert run(b(src), x, 8, 8, 4, 8, 8, img, lst, 4, cnt) == -1       # list kind, image out
    assert run(b(src), x, 8, 8, 4, 8, 8, None, lst, 4, None) == -1     # no count
    assert run(b(src), x, 8, 8, 4, 8, 8, None, lst, 4, ctypes.c_void_p((1 << 43) + 4)) == -1
    assert run(b(src), x, 8, 8, 4, 8, 8, None, None, 4, cnt) == -1     # capacity, no list
    assert run(b(src), x, 8, 8, 4, 8, 8, None, lst, -1, cnt) == -1
    assert run(b(src), x, 8, 8, 4, 8, 8, None, x, 4, cnt) == -1        # list overlaps frame
    assert L.crb_work_run(_lib.CRB_WORK_SOURCES, x, 8, 8, 0, 4, 1, img) == -1
    assert L.crb_lacosmic_partitioned(x, 64, 64, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4, 2, 2, -2,
                                      img, lst) == -1


def test_counting_and_debug_entry_validation(L):
    c = (ctypes.c_int64 * 4)()
    assert L.crb_plan_set_counting(None, 1) == -1
    assert L.crb_plan_work_counts(None, c) == -1
    assert L.crb_debug_median5_f64(None, 4, 4, ctypes.c_void_p(1 << 40)) == -1
    assert L.crb_debug_median5_f64(ctypes.c_void_p(1 << 41), 0, 4, ctypes.c_void_p(1 << 40)) == -1
    assert L.crb_debug_median5_f64(ctypes.c_void_p(1 << 40), 4, 4, ctypes.c_void_p((1 << 40) + 8)) == -1
    from paper_1008_2192_amd import _lib
    fr = _lib.Frame()
    fr.H, fr.W, fr.gain, fr.readnoise, fr.sigclip, fr.sigfrac, fr.objlim, fr.niter = \
        8, 8, 1.0, 5.0, 4.5, 0.3, 4.0, 1
    a, b = ctypes.c_void_p(1 << 40), ctypes.c_void_p(1 << 41)
    assert L.crb_debug_detect_exact(None, ctypes.byref(fr), a) == -1
    assert L.crb_debug_s_estimate(a, ctypes.byref(fr), None, b) == -1
    assert L.crb_debug_s_estimate(a, ctypes.byref(fr), b, ctypes.c_void_p((1 << 41) + 4)) == -1
    assert L.crb_debug_s_bound(a, ctypes.byref(fr), None) == -1
    assert L.crb_debug_s_bound(a, ctypes.byref(fr), ctypes.c_void_p((1 << 40) + 4)) == -1
    fr.gain = 0.0
    assert L.crb_debug_s_estimate(a, ctypes.byref(fr), b, ctypes.c_void_p(1 << 42)) == -1
    assert L.crb_debug_s_bound(a, ctypes.byref(fr), b) == -1
    assert L.crb_set_option(_lib.CRB_OPT_INCREMENTAL, 2) == -1
    assert L.crb_set_option(_lib.CRB_OPT_INCREMENTAL, 0) == 0


def prototypes():
    """{name: [parameter type strings]} of the functions include/crb.h declares."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    text = re.sub(r"#[^\n]*", "", text)
    out = {}
    for m in re.finditer(r"\b(crb_[a-z0-9_]+)\s*\(([^;{)]*)\)\s*;", text):
        params = [re.sub(r"\s+", " ", p).strip() for p in m.group(2).split(",")]
        out[m.group(1)] = [re.sub(r"\s*\b[a-zA-Z_][a-zA-Z0-9_]*$", "", p).replace(" *", "*")
                           for p in params if p and p != "void"]
    return out


def test_boundary_signatures():
    """The calls the boundary is specified by keep their argument lists: crb_lacosmic
    with the (img, H, W, gain, readnoise, sky, sigclip, sigfrac, objlim, niter,
    out_clean, out_mask) signature, the batched variant over crb_frame records on a
    stream, the stream, error and workspace queries, and the teacher-forced iteration
    with H and W as arguments."""
    P = prototypes()
    f32, i32 = "float", "int32_t"
    assert P["crb_lacosmic"] == ["const float*", i32, i32, f32, f32, f32, f32, f32, f32, i32,
                                 "float*", "uint8_t*"]
    assert P["crb_lacosmic_noalloc"] == P["crb_lacosmic"]
    assert P["crb_lacosmic_batched"] == ["crb_frame*", i32, "void*"]
    assert P["crb_set_stream"] == ["void*"]
    assert P["crb_last_error"] == []
    assert P["crb_workspace_bytes"] == [i32, i32]
    assert P["crb_debug_iterate"] == ["const float*", "const uint8_t*", i32, i32,
                                      "const crb_frame*", "uint8_t*", "uint8_t*", "float*",
                                      "int64_t*"]


def test_noalloc_rejects_oversized_frames_on_host(L):
    """A frame whose workspace exceeds the fixed scratch is refused before any device
    work (the pointers are never dereferenced)."""
    p, q, m = ctypes.c_void_p(16), ctypes.c_void_p(1 << 40), ctypes.c_void_p(1 << 41)
    assert L.crb_workspace_bytes(6000, 6000) > (96 << 20)
    assert L.crb_lacosmic_noalloc(p, 6000, 6000, 1.0, 5.0, 0.0, 4.5, 0.3, 4.0, 4, q, m) == -4
    assert b"scratch" in L.crb_last_error()
    assert L.crb_workspace_bytes(4096, 4096) <= (96 << 20)
