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
