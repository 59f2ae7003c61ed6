"""ctypes binding of libcrb (include/crb.h): argument marshalling only.

Every step of the method runs in the HIP library; PyTorch supplies device memory
and streams.  Import fails loudly when libcrb.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrb.so")

CRB_FLAG_NO_EARLY_STOP = 1
CRB_FLAG_INCREMENTAL = 2
CRB_OPT_EARLY_STOP = 1
CRB_OPT_INCREMENTAL = 2
CRB_OPT_TILE_H = 3
CRB_OPT_FUSED = 4
CRB_OPT_GROW_H = 5
STATUS = {0: "CRB_OK", -1: "CRB_EINVAL", -2: "CRB_ENOMEM", -3: "CRB_EDEVICE",
          -4: "CRB_ETOOBIG", -5: "CRB_EBUSY"}

EXPORTS = ["crb_lacosmic", "crb_lacosmic_noalloc", "crb_lacosmic_batched", "crb_lacosmic_partitioned", "crb_plan_create", "crb_plan_run",
           "crb_plan_stats", "crb_plan_destroy", "crb_plan_set_timing", "crb_plan_kernel_times", "crb_set_stream", "crb_set_option",
           "crb_last_error", "crb_workspace_bytes", "crb_release_workspace",
           "crb_server_create", "crb_server_submit", "crb_server_poll", "crb_server_pending",
           "crb_server_destroy", "crb_debug_iterate", "crb_debug_detect", "crb_debug_median",
           "crb_debug_fp64", "crb_work_run", "crb_work_radius", "crb_farm_run",
           "crb_plan_set_counting", "crb_plan_work_counts", "crb_debug_median5_f64",
           "crb_debug_detect_exact", "crb_debug_s_estimate", "crb_plan_set_tuning",
           "crb_plan_get_tuning", "crb_plan_autotune", "crb_debug_copy_b32", "crb_debug_s_bound"]
CRB_WORK_LACOSMIC = 0
CRB_WORK_POISSON = 1
CRB_WORK_WAITER = 2
CRB_WORK_SOURCES = 3

# One record of the SOURCES work function (crb_source, 40 bytes).
SOURCE_DTYPE = np.dtype([("y", np.int32), ("x", np.int32), ("peak", np.float32),
                         ("npix", np.int32), ("flux", np.float64), ("sy", np.float64),
                         ("sx", np.float64)])


class CrbError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class Work(ctypes.Structure):
    """Mirror of ``crb_work``."""
    _fields_ = [("kind", ctypes.c_int32), ("niter", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("threshold", ctypes.c_float), ("sky", ctypes.c_float),
                ("peak_radius", ctypes.c_int32), ("aperture_radius", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    """Mirror of ``crb_tuning`` (a plan's launch shapes)."""
    _fields_ = [("tile_h", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("grow_h", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return dict(tile_h=self.tile_h, persistent=self.persistent, fused=self.fused,
                    grow_h=self.grow_h)


DEFAULT_TUNING = dict(tile_h=32, persistent=0, fused=0, grow_h=0)


class Frame(ctypes.Structure):
    """Mirror of ``crb_frame``."""
    _fields_ = [("img", ctypes.c_void_p), ("out_clean", ctypes.c_void_p),
                ("out_mask", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("gain", ctypes.c_float), ("readnoise", ctypes.c_float), ("sky", ctypes.c_float),
                ("sigclip", ctypes.c_float), ("sigfrac", ctypes.c_float),
                ("objlim", ctypes.c_float), ("niter", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("iters_run", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_flagged", ctypes.c_int64)]


_lib = None


def lib():
    """Load libcrb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libcrb.so not found at {LIB_PATH}: build it first "
                           f"(python -m paper_1008_2192_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.crb_lacosmic.argtypes = [vp, i32, i32, f32, f32, f32, f32, f32, f32, i32, vp, vp]
    L.crb_lacosmic_noalloc.argtypes = L.crb_lacosmic.argtypes
    L.crb_lacosmic_batched.argtypes = [ctypes.POINTER(Frame), i32, vp]
    L.crb_lacosmic_partitioned.argtypes = [vp, i32, i32, f32, f32, f32, f32, f32, f32, i32,
                                           i32, i32, i32, vp, vp]
    L.crb_plan_create.argtypes = [ctypes.POINTER(Frame), i32, vp, i32, ctypes.POINTER(vp)]
    L.crb_plan_run.argtypes = [vp]
    L.crb_plan_stats.argtypes = [vp, ctypes.POINTER(Frame), i32]
    L.crb_plan_destroy.argtypes = [vp]
    L.crb_plan_destroy.restype = None
    L.crb_plan_set_timing.argtypes = [vp, i32]
    L.crb_plan_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(i64)]
    L.crb_plan_set_counting.argtypes = [vp, i32]
    L.crb_plan_work_counts.argtypes = [vp, ctypes.POINTER(i64)]
    L.crb_debug_median5_f64.argtypes = [vp, i32, i32, vp]
    L.crb_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.crb_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.crb_plan_autotune.argtypes = [vp, i32, i32, ctypes.POINTER(Tuning),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    L.crb_set_stream.argtypes = [vp]
    L.crb_set_option.argtypes = [i32, i64]
    L.crb_last_error.argtypes = []
    L.crb_last_error.restype = ctypes.c_char_p
    L.crb_workspace_bytes.argtypes = [i32, i32]
    L.crb_workspace_bytes.restype = ctypes.c_size_t
    L.crb_release_workspace.argtypes = [vp]
    L.crb_server_create.argtypes = [ctypes.c_size_t, i32, ctypes.POINTER(vp)]
    L.crb_server_submit.argtypes = [vp, vp, i32, i32, f32, f32, f32, f32, f32, f32, i32, vp, vp,
                                    ctypes.POINTER(i64)]
    L.crb_server_poll.argtypes = [vp, vp, vp, i32, ctypes.POINTER(i32)]
    L.crb_server_pending.argtypes = [vp]
    L.crb_server_pending.restype = i32
    L.crb_server_destroy.argtypes = [vp]
    L.crb_server_destroy.restype = None
    L.crb_debug_iterate.argtypes = [vp, vp, i32, i32, ctypes.POINTER(Frame), vp, vp, vp, vp]
    L.crb_debug_detect.argtypes = [vp, ctypes.POINTER(Frame), vp]
    L.crb_debug_detect_exact.argtypes = [vp, ctypes.POINTER(Frame), vp]
    L.crb_debug_s_estimate.argtypes = [vp, ctypes.POINTER(Frame), vp, vp]
    L.crb_debug_s_bound.argtypes = [vp, ctypes.POINTER(Frame), vp]
    L.crb_debug_median.argtypes = [vp, i32, i32, i32, vp]
    L.crb_debug_fp64.argtypes = [vp, vp, i32, vp, vp]
    L.crb_debug_copy_b32.argtypes = [vp, vp, i64]
    L.crb_work_run.argtypes = [i32, vp, i32, i32, ctypes.c_uint64, i32, i32, vp]
    L.crb_work_radius.argtypes = [ctypes.POINTER(Work)]
    L.crb_work_radius.restype = i32
    L.crb_farm_run.argtypes = [ctypes.POINTER(Work), vp, i32, i32, i32, i32, i32, vp, vp, i64, vp]
    for name in ("crb_lacosmic", "crb_lacosmic_noalloc", "crb_lacosmic_batched", "crb_lacosmic_partitioned",
                 "crb_plan_create", "crb_plan_run",
                 "crb_plan_stats", "crb_plan_set_timing", "crb_plan_kernel_times", "crb_set_stream", "crb_set_option", "crb_release_workspace",
                 "crb_server_create", "crb_server_submit", "crb_server_poll",
                 "crb_debug_iterate", "crb_debug_detect", "crb_debug_median", "crb_debug_fp64",
                 "crb_work_run", "crb_farm_run", "crb_plan_set_counting", "crb_plan_work_counts",
                 "crb_debug_median5_f64", "crb_debug_detect_exact", "crb_debug_s_estimate",
                 "crb_plan_set_tuning", "crb_plan_get_tuning", "crb_plan_autotune",
                 "crb_debug_copy_b32", "crb_debug_s_bound"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(fn: str, status: int) -> None:
    if status != 0:
        msg = lib().crb_last_error()
        raise CrbError(fn, status, msg.decode() if msg else "")


def _stream(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev2d(t: torch.Tensor, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 2-D {dtype} tensor")
    return t


def set_stream(stream: Optional[torch.cuda.Stream] = None) -> None:
    check("crb_set_stream", lib().crb_set_stream(ctypes.c_void_p(_stream(stream))))


def set_single_tuning(tile_h: int = 32, fused: int = 0, grow_h: int = 0) -> None:
    """Launch shapes of the single-frame entry points (CRB_OPT_TILE_H, CRB_OPT_FUSED,
    CRB_OPT_GROW_H); every shape gives identical results."""
    L = lib()
    check("crb_set_option", L.crb_set_option(CRB_OPT_TILE_H, tile_h))
    check("crb_set_option", L.crb_set_option(CRB_OPT_FUSED, fused))
    check("crb_set_option", L.crb_set_option(CRB_OPT_GROW_H, grow_h))


def lacosmic(img: torch.Tensor, gain: float, readnoise: float, sky: float = 0.0,
             sigclip: float = 4.5, sigfrac: float = 0.3, objlim: float = 4.0, niter: int = 4,
             out_clean: Optional[torch.Tensor] = None, out_mask: Optional[torch.Tensor] = None,
             early_stop: bool = True, incremental: bool = False,
             stream: Optional[torch.cuda.Stream] = None):
    """crb_lacosmic on device tensors; returns (clean float32, mask uint8).
    incremental: CRB_OPT_INCREMENTAL (identical results, less detection work)."""
    _dev2d(img, torch.float32, "img")
    H, W = img.shape
    if out_clean is None:
        out_clean = torch.empty_like(img)
    if out_mask is None:
        out_mask = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    _dev2d(out_clean, torch.float32, "out_clean")
    _dev2d(out_mask, torch.uint8, "out_mask")
    L = lib()
    set_stream(stream)
    check("crb_set_option", L.crb_set_option(CRB_OPT_EARLY_STOP, 1 if early_stop else 0))
    check("crb_set_option", L.crb_set_option(CRB_OPT_INCREMENTAL, 1 if incremental else 0))
    check("crb_lacosmic", L.crb_lacosmic(img.data_ptr(), H, W, gain, readnoise, sky, sigclip,
                                         sigfrac, objlim, niter, out_clean.data_ptr(),
                                         out_mask.data_ptr()))
    return out_clean, out_mask


def lacosmic_noalloc(img: torch.Tensor, gain: float, readnoise: float, sky: float = 0.0,
                     sigclip: float = 4.5, sigfrac: float = 0.3, objlim: float = 4.0,
                     niter: int = 4, out_clean: Optional[torch.Tensor] = None,
                     out_mask: Optional[torch.Tensor] = None, early_stop: bool = True,
                     stream: Optional[torch.cuda.Stream] = None):
    """crb_lacosmic_noalloc: crb_lacosmic with the library's fixed device scratch as its
    workspace (no device allocation by the library); returns (clean, mask)."""
    _dev2d(img, torch.float32, "img")
    H, W = img.shape
    if out_clean is None:
        out_clean = torch.empty_like(img)
    if out_mask is None:
        out_mask = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    _dev2d(out_clean, torch.float32, "out_clean")
    _dev2d(out_mask, torch.uint8, "out_mask")
    L = lib()
    set_stream(stream)
    check("crb_set_option", L.crb_set_option(CRB_OPT_EARLY_STOP, 1 if early_stop else 0))
    check("crb_set_option", L.crb_set_option(CRB_OPT_INCREMENTAL, 0))
    check("crb_lacosmic_noalloc", L.crb_lacosmic_noalloc(
        img.data_ptr(), H, W, gain, readnoise, sky, sigclip, sigfrac, objlim, niter,
        out_clean.data_ptr(), out_mask.data_ptr()))
    return out_clean, out_mask


def lacosmic_partitioned(img: torch.Tensor, gain: float, readnoise: float, ny: int, nx: int,
                         border: int, sky: float = 0.0, sigclip: float = 4.5,
                         sigfrac: float = 0.3, objlim: float = 4.0, niter: int = 4,
                         incremental: bool = False,
                         stream: Optional[torch.cuda.Stream] = None):
    """crb_lacosmic_partitioned: independent subimages with a border, stitched."""
    _dev2d(img, torch.float32, "img")
    H, W = img.shape
    out_clean = torch.empty_like(img)
    out_mask = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    set_stream(stream)
    check("crb_set_option", lib().crb_set_option(CRB_OPT_INCREMENTAL, 1 if incremental else 0))
    check("crb_lacosmic_partitioned", lib().crb_lacosmic_partitioned(
        img.data_ptr(), H, W, gain, readnoise, sky, sigclip, sigfrac, objlim, niter, ny, nx,
        border, out_clean.data_ptr(), out_mask.data_ptr()))
    return out_clean, out_mask


def make_frames(items: Sequence[dict]) -> "ctypes.Array[Frame]":
    """items: dicts with img, out_clean, out_mask tensors and the parameters
    (early_stop, default True; incremental, default False)."""
    arr = (Frame * len(items))()
    for i, it in enumerate(items):
        img = _dev2d(it["img"], torch.float32, "img")
        oc = _dev2d(it["out_clean"], torch.float32, "out_clean")
        om = _dev2d(it["out_mask"], torch.uint8, "out_mask")
        H, W = img.shape
        arr[i] = Frame(img.data_ptr(), oc.data_ptr(), om.data_ptr(), H, W, it["gain"],
                       it["readnoise"], it.get("sky", 0.0), it.get("sigclip", 4.5),
                       it.get("sigfrac", 0.3), it.get("objlim", 4.0), it.get("niter", 4),
                       (CRB_FLAG_NO_EARLY_STOP if not it.get("early_stop", True) else 0) |
                       (CRB_FLAG_INCREMENTAL if it.get("incremental", False) else 0), 0, 0, 0)
    return arr


def lacosmic_batched(items: Sequence[dict], stream: Optional[torch.cuda.Stream] = None
                     ) -> List[dict]:
    """crb_lacosmic_batched; returns per-frame dict(iters_run, n_flagged)."""
    arr = make_frames(items)
    check("crb_lacosmic_batched",
          lib().crb_lacosmic_batched(arr, len(items), ctypes.c_void_p(_stream(stream))))
    return [dict(iters_run=f.iters_run, n_flagged=f.n_flagged) for f in arr]


class Plan:
    """A batch plan (crb_plan_*), optionally graph-captured.  By default it runs on a
    stream of its own, ordered after the caller's current stream at each run and
    before it afterwards; with on_current_stream it runs on the stream that is current
    at creation, with no cross-stream waits (a graph plan needs that stream to be one
    other than the null stream, on which no graph can be captured)."""

    def __init__(self, items: Sequence[dict], use_graph: bool = True,
                 on_current_stream: bool = False):
        self.items = list(items)
        self.frames = make_frames(self.items)
        self.handle = ctypes.c_void_p()
        if on_current_stream and use_graph and torch.cuda.current_stream().cuda_stream == 0:
            raise ValueError("a graph plan cannot be captured on the null stream")
        self.stream = torch.cuda.current_stream() if on_current_stream else torch.cuda.Stream()
        self._own = not on_current_stream
        check("crb_plan_create", lib().crb_plan_create(
            self.frames, len(self.items), ctypes.c_void_p(self.stream.cuda_stream),
            1 if use_graph else 0, ctypes.byref(self.handle)))

    def run(self) -> None:
        if not self._own:
            check("crb_plan_run", lib().crb_plan_run(self.handle))
            return
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        check("crb_plan_run", lib().crb_plan_run(self.handle))
        cur.wait_stream(self.stream)

    def stats(self) -> List[dict]:
        check("crb_plan_stats", lib().crb_plan_stats(self.handle, self.frames, len(self.items)))
        return [dict(iters_run=f.iters_run, n_flagged=f.n_flagged) for f in self.frames]

    def set_tuning(self, tile_h: int = 32, persistent: int = 0, fused: int = 0,
                   grow_h: int = 0) -> None:
        """crb_plan_set_tuning: the launch shapes of later runs (identical results)."""
        t = Tuning(tile_h, persistent, fused, grow_h)
        check("crb_plan_set_tuning", lib().crb_plan_set_tuning(self.handle, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        check("crb_plan_get_tuning", lib().crb_plan_get_tuning(self.handle, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, reps: int = 3, use_cache: bool = True) -> dict:
        """crb_plan_autotune: time the launch shapes, apply the fastest; returns
        dict(tuning, ms, default_ms) (ms are -1 when the tune cache supplied it)."""
        t = Tuning()
        ms, dms = ctypes.c_double(), ctypes.c_double()
        check("crb_plan_autotune", lib().crb_plan_autotune(
            self.handle, reps, 1 if use_cache else 0, ctypes.byref(t), ctypes.byref(ms),
            ctypes.byref(dms)))
        return dict(tuning=t.as_dict(), ms=ms.value, default_ms=dms.value)

    def set_timing(self, enable: bool) -> None:
        check("crb_plan_set_timing", lib().crb_plan_set_timing(self.handle, 1 if enable else 0))

    KINDS = ("init", "detect", "grow", "replace")

    def kernel_times(self) -> dict:
        """{kind: (total ms, launches)} since timing was enabled."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        check("crb_plan_kernel_times", lib().crb_plan_kernel_times(self.handle, ms, n))
        return {k: (ms[i], int(n[i])) for i, k in enumerate(self.KINDS)}

    def set_counting(self, enable: bool) -> None:
        check("crb_plan_set_counting", lib().crb_plan_set_counting(self.handle,
                                                                   1 if enable else 0))

    def work_counts(self) -> dict:
        """Detection work since counting was enabled: work-set pixels (med5 of S and
        the threshold bits), contrast tests (S'/F^ > objlim), binary64 re-evaluations
        (work-set pixels the FP32 estimate of S could not decide) and pixels whose
        med5(J) was selected exactly (those near a pixel where S may exceed sigclip)."""
        c = (ctypes.c_int64 * 4)()
        check("crb_plan_work_counts", lib().crb_plan_work_counts(self.handle, c))
        return dict(work_pixels=int(c[0]), contrast_tests=int(c[1]), reevaluated=int(c[2]),
                    exact_med5=int(c[3]))

    def close(self) -> None:
        if self.handle:
            lib().crb_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _params_frame(H: int, W: int, gain, readnoise, sky=0.0, sigclip=4.5, sigfrac=0.3,
                  objlim=4.0) -> Frame:
    return Frame(None, None, None, H, W, gain, readnoise, sky, sigclip, sigfrac, objlim, 1, 0,
                 0, 0, 0)


def debug_iterate(J: torch.Tensor, M_prev: torch.Tensor, gain, readnoise, sky=0.0,
                  sigclip=4.5, sigfrac=0.3, objlim=4.0,
                  stream: Optional[torch.cuda.Stream] = None):
    """One iteration on (J_k, M_{k-1}); returns (G2, M_k, J_{k+1}, n_k tensor)."""
    _dev2d(J, torch.float32, "J")
    _dev2d(M_prev, torch.uint8, "M_prev")
    H, W = J.shape
    G2 = torch.empty((H, W), dtype=torch.uint8, device=J.device)
    M = torch.empty_like(G2)
    Jn = torch.empty_like(J)
    n = torch.zeros(1, dtype=torch.int64, device=J.device)
    p = _params_frame(H, W, gain, readnoise, sky, sigclip, sigfrac, objlim)
    set_stream(stream)
    check("crb_debug_iterate", lib().crb_debug_iterate(J.data_ptr(), M_prev.data_ptr(), H, W,
                                                       ctypes.byref(p), G2.data_ptr(),
                                                       M.data_ptr(), Jn.data_ptr(),
                                                       n.data_ptr()))
    return G2, M, Jn, n


def debug_detect(J: torch.Tensor, gain, readnoise, sky=0.0, sigclip=4.5, sigfrac=0.3,
                 objlim=4.0, exact: bool = False,
                 stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Detection codes (crb_debug_detect; crb_debug_detect_exact with exact=True)."""
    _dev2d(J, torch.float32, "J")
    H, W = J.shape
    codes = torch.empty((H, W), dtype=torch.uint8, device=J.device)
    p = _params_frame(H, W, gain, readnoise, sky, sigclip, sigfrac, objlim)
    set_stream(stream)
    name = "crb_debug_detect_exact" if exact else "crb_debug_detect"
    check(name, getattr(lib(), name)(J.data_ptr(), ctypes.byref(p), codes.data_ptr()))
    return codes


def debug_s_estimate(J: torch.Tensor, gain, readnoise, sky=0.0, sigclip=4.5, sigfrac=0.3,
                     objlim=4.0, stream: Optional[torch.cuda.Stream] = None):
    """The detection's FP32 estimate of S and its error bound (crb_debug_s_estimate)."""
    _dev2d(J, torch.float32, "J")
    H, W = J.shape
    s = torch.empty((H, W), dtype=torch.float32, device=J.device)
    err = torch.empty_like(s)
    p = _params_frame(H, W, gain, readnoise, sky, sigclip, sigfrac, objlim)
    set_stream(stream)
    check("crb_debug_s_estimate", lib().crb_debug_s_estimate(J.data_ptr(), ctypes.byref(p),
                                                             s.data_ptr(), err.data_ptr()))
    return s, err


def debug_s_bound(J: torch.Tensor, gain, readnoise, sky=0.0, sigclip=4.5, sigfrac=0.3,
                  objlim=4.0, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """The detection's dense upper bound of S (crb_debug_s_bound)."""
    _dev2d(J, torch.float32, "J")
    H, W = J.shape
    u = torch.empty((H, W), dtype=torch.float32, device=J.device)
    p = _params_frame(H, W, gain, readnoise, sky, sigclip, sigfrac, objlim)
    set_stream(stream)
    check("crb_debug_s_bound", lib().crb_debug_s_bound(J.data_ptr(), ctypes.byref(p),
                                                       u.data_ptr()))
    return u


def debug_median(x: torch.Tensor, r: int, stream: Optional[torch.cuda.Stream] = None
                 ) -> torch.Tensor:
    _dev2d(x, torch.float32, "x")
    out = torch.empty_like(x)
    set_stream(stream)
    check("crb_debug_median", lib().crb_debug_median(x.data_ptr(), x.shape[0], x.shape[1], r,
                                                     out.data_ptr()))
    return out


def debug_median5_f64(x: torch.Tensor, stream: Optional[torch.cuda.Stream] = None
                      ) -> torch.Tensor:
    _dev2d(x, torch.float64, "x")
    out = torch.empty_like(x)
    set_stream(stream)
    check("crb_debug_median5_f64", lib().crb_debug_median5_f64(x.data_ptr(), x.shape[0],
                                                               x.shape[1], out.data_ptr()))
    return out


def debug_fp64(x: torch.Tensor, y: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
    if x.dtype != torch.float64 or y.dtype != torch.float64 or not x.is_cuda or not y.is_cuda:
        raise ValueError("x, y must be float64 CUDA tensors")
    x, y = x.contiguous(), y.contiguous()
    if x.numel() != y.numel():
        raise ValueError("x and y differ in size")
    s = torch.empty_like(x)
    d = torch.empty_like(x)
    set_stream(stream)
    check("crb_debug_fp64", lib().crb_debug_fp64(x.data_ptr(), y.data_ptr(), x.numel(),
                                                 s.data_ptr(), d.data_ptr()))
    return s, d


def debug_copy_b32(src: torch.Tensor, dst: torch.Tensor,
                   stream: Optional[torch.cuda.Stream] = None) -> None:
    """crb_debug_copy_b32: dst = src (float32, contiguous, same size) by 4-byte buffer
    loads and stores (HBM counter calibration)."""
    if src.dtype != torch.float32 or dst.dtype != torch.float32 or not src.is_cuda or \
            not dst.is_cuda or not src.is_contiguous() or not dst.is_contiguous() or \
            src.numel() != dst.numel():
        raise ValueError("src and dst must be contiguous float32 CUDA tensors of one size")
    set_stream(stream)
    check("crb_debug_copy_b32", lib().crb_debug_copy_b32(src.data_ptr(), dst.data_ptr(),
                                                         src.numel()))


def workspace_bytes(H: int, W: int) -> int:
    return int(lib().crb_workspace_bytes(H, W))


def work_run(kind: int, x: torch.Tensor, seed: int = 0, workers: int = 1024,
             band_rows: int = 1, out: Optional[torch.Tensor] = None,
             stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """crb_work_run: the POISSON or WAITER work function on a persistent tile farm."""
    _dev2d(x, torch.float32, "x")
    if out is None:
        out = torch.empty_like(x)
    set_stream(stream)
    check("crb_work_run", lib().crb_work_run(kind, x.data_ptr(), x.shape[0], x.shape[1],
                                             int(seed) & (2 ** 64 - 1), workers, band_rows,
                                             out.data_ptr()))
    return out


def make_work(kind: int, seed: int = 0, threshold: float = 0.0, sky: float = 0.0, r: int = 1,
              a: int = 0, niter: int = 0) -> Work:
    return Work(int(kind), int(niter), int(seed) & (2 ** 64 - 1), float(threshold), float(sky),
                int(r), int(a))


def work_radius(kind: int, **kw) -> int:
    """crb_work_radius: the dependency radius a work function declares."""
    w = make_work(kind, **kw)
    rad = lib().crb_work_radius(ctypes.byref(w))
    if rad < 0:
        check("crb_work_radius", -1)
    return int(rad)


def farm_image(kind: int, x: torch.Tensor, seed: int = 0, workers: int = 1024, tile_h: int = 1,
               tile_w: Optional[int] = None, out: Optional[torch.Tensor] = None,
               stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """crb_farm_run for an image work function (POISSON, WAITER) on tile_h x tile_w
    rectangles (tile_w defaults to the full width)."""
    _dev2d(x, torch.float32, "x")
    H, W = x.shape
    if out is None:
        out = torch.empty_like(x)
    w = make_work(kind, seed=seed)
    set_stream(stream)
    check("crb_farm_run", lib().crb_farm_run(ctypes.byref(w), x.data_ptr(), H, W, workers,
                                             tile_h, W if tile_w is None else tile_w,
                                             out.data_ptr(), None, 0, None))
    return out


class SourceList:
    """Device-side result of the SOURCES work function: `records` (uint8 tensor of
    capacity x 40 bytes) and `count` (int64 tensor of one element)."""

    def __init__(self, records: torch.Tensor, count: torch.Tensor, capacity: int):
        self.records, self.count, self.capacity = records, count, capacity

    def numpy(self) -> np.ndarray:
        """The records as a structured array (SOURCE_DTYPE) sorted by (y, x); raises
        if the list was truncated."""
        n = int(self.count.item())
        if n > self.capacity:
            raise OverflowError(f"{n} sources found, capacity {self.capacity}")
        rec = self.records[: n * SOURCE_DTYPE.itemsize].cpu().numpy().view(SOURCE_DTYPE)
        return rec[np.lexsort((rec["x"], rec["y"]))]


def farm_sources(x: torch.Tensor, threshold: float, sky: float = 0.0, r: int = 2, a: int = 2,
                 workers: int = 4096, tile_h: int = 32, tile_w: int = 64,
                 capacity: int = 1 << 20, out: Optional[SourceList] = None,
                 stream: Optional[torch.cuda.Stream] = None) -> SourceList:
    """crb_farm_run with the SOURCES work function: peaks above threshold with their
    aperture sums, by `workers` actors (waves); asynchronous (read the result with
    .numpy())."""
    _dev2d(x, torch.float32, "x")
    H, W = x.shape
    if out is None:
        out = SourceList(torch.empty(max(capacity, 1) * SOURCE_DTYPE.itemsize, dtype=torch.uint8,
                                     device=x.device),
                         torch.empty(1, dtype=torch.int64, device=x.device), capacity)
    w = make_work(CRB_WORK_SOURCES, threshold=threshold, sky=sky, r=r, a=a)
    set_stream(stream)
    check("crb_farm_run", lib().crb_farm_run(ctypes.byref(w), x.data_ptr(), H, W, workers,
                                             tile_h, tile_w, None, out.records.data_ptr(),
                                             out.capacity, out.count.data_ptr()))
    return out
