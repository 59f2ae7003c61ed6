"""ctypes wrapper around the FP64 L.A.Cosmic oracle (``crb_ref.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.
Arrays are numpy, on the host; the C library is built by ``build()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crb_ref.c")
_LIB = os.path.join(_HERE, "libcrb_ref.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: binary64 arithmetic, no contraction, no fast-math."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("gain", ctypes.c_double), ("readnoise", ctypes.c_double),
                ("sky", ctypes.c_double), ("sigclip", ctypes.c_double),
                ("sigfrac", ctypes.c_double), ("objlim", ctypes.c_double)]


class Trace(ctypes.Structure):
    _fields_ = [("lplus", ctypes.c_void_p), ("noise", ctypes.c_void_p), ("s", ctypes.c_void_p),
                ("sprime", ctypes.c_void_p), ("fhat", ctypes.c_void_p),
                ("first", ctypes.c_void_p), ("g1", ctypes.c_void_p), ("g2", ctypes.c_void_p)]


_lib = None
_lib_path = None


def use_library(path=None):
    """Load the oracle from another build of the same source (the default build when
    path is None); the mutation tests compile deliberately broken copies this way."""
    global _lib, _lib_path
    _lib = None
    _lib_path = path


def lib():
    global _lib
    if _lib is None:
        path = _lib_path or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(path)
        dp = ctypes.c_void_p
        L.crb_ref_median_filter.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.crb_ref_lplus.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        L.crb_ref_iterate.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Params),
                                      dp, dp, dp, ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(Trace)]
        L.crb_ref_lacosmic.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Params),
                                       ctypes.c_int, ctypes.c_int, dp, dp,
                                       ctypes.POINTER(ctypes.c_int), dp]
        L.crb_ref_philox4x32_10.argtypes = [dp, dp, dp]
        L.crb_ref_philox4x32_10.restype = None
        L.crb_ref_expneg.argtypes = [ctypes.c_double]
        L.crb_ref_expneg.restype = ctypes.c_double
        L.crb_ref_poisson.argtypes = [dp, ctypes.c_longlong, ctypes.c_ulonglong, dp]
        L.crb_ref_sources.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_int, ctypes.c_int, dp,
                                      ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]
        for f in (L.crb_ref_median_filter, L.crb_ref_lplus, L.crb_ref_iterate,
                  L.crb_ref_lacosmic, L.crb_ref_poisson, L.crb_ref_sources):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def make_params(gain, readnoise, sky=0.0, sigclip=4.5, sigfrac=0.3, objlim=4.0) -> Params:
    return Params(float(gain), float(readnoise), float(sky), float(sigclip), float(sigfrac),
                  float(objlim))


def median_filter(x: np.ndarray, r: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    rc = lib().crb_ref_median_filter(_ptr(x), x.shape[0], x.shape[1], r, _ptr(out))
    if rc:
        raise ValueError(f"crb_ref_median_filter failed ({rc})")
    return out


def lplus(J: np.ndarray) -> np.ndarray:
    J = np.ascontiguousarray(J, dtype=np.float64)
    out = np.empty_like(J)
    rc = lib().crb_ref_lplus(_ptr(J), J.shape[0], J.shape[1], _ptr(out))
    if rc:
        raise ValueError(f"crb_ref_lplus failed ({rc})")
    return out


def iterate(J: np.ndarray, Mprev: np.ndarray, gain, readnoise, sky=0.0, sigclip=4.5,
            sigfrac=0.3, objlim=4.0, trace: bool = False) -> dict:
    """One iteration; returns dict with G2, M, Jnext, n (and the trace planes)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    H, W = J.shape
    Mprev = np.ascontiguousarray(Mprev, dtype=np.uint8)
    assert Mprev.shape == J.shape
    G2 = np.empty((H, W), np.uint8)
    M = np.empty((H, W), np.uint8)
    Jn = np.empty((H, W), np.float64)
    nn = ctypes.c_longlong(0)
    res = dict(G2=G2, M=M, Jnext=Jn)
    tr = None
    if trace:
        planes = {k: np.empty((H, W), np.float64) for k in ("lplus", "noise", "s", "sprime", "fhat")}
        bits = {k: np.empty((H, W), np.uint8) for k in ("first", "g1", "g2")}
        tr = Trace(*[_ptr(planes[k]) for k in ("lplus", "noise", "s", "sprime", "fhat")],
                   *[_ptr(bits[k]) for k in ("first", "g1", "g2")])
        res.update(planes)
        res.update(bits)
    p = make_params(gain, readnoise, sky, sigclip, sigfrac, objlim)
    rc = lib().crb_ref_iterate(_ptr(J), _ptr(Mprev), H, W, ctypes.byref(p), _ptr(G2), _ptr(M),
                               _ptr(Jn), ctypes.byref(nn), ctypes.byref(tr) if tr else None)
    if rc:
        raise ValueError(f"crb_ref_iterate failed ({rc})")
    res["n"] = int(nn.value)
    return res


def lacosmic(img: np.ndarray, gain, readnoise, sky=0.0, sigclip=4.5, sigfrac=0.3, objlim=4.0,
             niter=4, early_stop=True) -> dict:
    """Full run on an FP32 frame; returns dict(clean=float64, mask=uint8, iters, counts)."""
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W = img.shape
    clean = np.empty((H, W), np.float64)
    mask = np.empty((H, W), np.uint8)
    iters = ctypes.c_int(0)
    counts = np.zeros(max(niter, 1), np.int64)
    p = make_params(gain, readnoise, sky, sigclip, sigfrac, objlim)
    rc = lib().crb_ref_lacosmic(_ptr(img), H, W, ctypes.byref(p), int(niter), int(bool(early_stop)),
                                _ptr(clean), _ptr(mask), ctypes.byref(iters), _ptr(counts))
    if rc:
        raise ValueError(f"crb_ref_lacosmic failed ({rc})")
    return dict(clean=clean, mask=mask, iters=int(iters.value), counts=counts[:iters.value].copy())


def lacosmic_frame(frame, niter: Optional[int] = None, early_stop=True) -> dict:
    """Run on a ``synth.Frame``."""
    return lacosmic(frame.img, frame.gain, frame.readnoise, frame.sky, frame.sigclip,
                    frame.sigfrac, frame.objlim,
                    frame.niter if niter is None else niter, early_stop)


def philox4x32_10(ctr, key) -> list:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().crb_ref_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(v) for v in out]


def expneg(x: float) -> float:
    return float(lib().crb_ref_expneg(float(x)))


def poisson(means: np.ndarray, seed: int) -> np.ndarray:
    """The POISSON work function: one deviate per pixel (float32 counts)."""
    m = np.ascontiguousarray(means, dtype=np.float32)
    out = np.empty_like(m)
    rc = lib().crb_ref_poisson(_ptr(m), m.size, int(seed), _ptr(out))
    if rc:
        raise ValueError("crb_ref_poisson failed")
    return out


# One record of the SOURCES work function (crb_ref_source, 40 bytes).
SOURCE_DTYPE = np.dtype([("y", np.int32), ("x", np.int32), ("peak", np.float32),
                         ("npix", np.int32), ("flux", np.float64), ("sy", np.float64),
                         ("sx", np.float64)])


def sources(img: np.ndarray, threshold: float, sky: float = 0.0, r: int = 2,
            a: int = 2) -> np.ndarray:
    """The SOURCES work function on a whole frame: a structured array (SOURCE_DTYPE)
    of the local peaks above threshold, in raster order, with their aperture sums."""
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W = img.shape
    L = lib()
    cnt = ctypes.c_longlong(0)
    rc = L.crb_ref_sources(_ptr(img), H, W, float(threshold), float(sky), int(r), int(a),
                           None, 0, ctypes.byref(cnt))
    if rc:
        raise ValueError(f"crb_ref_sources failed ({rc})")
    out = np.zeros(max(cnt.value, 1), SOURCE_DTYPE)
    rc = L.crb_ref_sources(_ptr(img), H, W, float(threshold), float(sky), int(r), int(a),
                           _ptr(out), out.size, ctypes.byref(cnt))
    if rc:
        raise ValueError(f"crb_ref_sources failed ({rc})")
    return out[:cnt.value].copy()
