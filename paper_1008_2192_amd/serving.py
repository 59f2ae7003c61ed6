"""Serving: a thin Python driver over the C serving loop (crb_server_*).

The C library does admission by HBM budget, keeps each admitted frame's state on
the device and runs iteration-level rounds over all admitted frames; this module
only marshals host arrays, replays an arrival trace in real time and summarises
latencies.  A Server is used from one thread.
"""
from __future__ import annotations

import ctypes
import dataclasses
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib


class Server:
    def __init__(self, hbm_budget: int, max_slots: int = 64):
        self.handle = ctypes.c_void_p()
        L = _lib.lib()
        _lib.check("crb_server_create", L.crb_server_create(int(hbm_budget), int(max_slots),
                                                            ctypes.byref(self.handle)))
        self._outs: Dict[int, Tuple[np.ndarray, np.ndarray, np.ndarray]] = {}
        self._ids = (ctypes.c_int64 * 256)()
        self._lat = (ctypes.c_double * 256)()

    def submit(self, img, gain: float, readnoise: float, sky: float = 0.0,
               sigclip: float = 4.5, sigfrac: float = 0.3, objlim: float = 4.0,
               niter: int = 4) -> int:
        """img: a numpy array, a pinned CPU torch tensor (then the outputs are pinned
        tensors too and the server transfers without staging copies), or a CUDA tensor on
        the server's device, ready to be read (then the outputs are CUDA tensors and every
        transfer stays on the device)."""
        import torch
        if isinstance(img, torch.Tensor):
            if img.dtype != torch.float32 or img.dim() != 2 or not img.is_contiguous():
                raise ValueError("img must be a contiguous 2-D float32 tensor")
            H, W = img.shape
            if img.is_cuda:
                clean = torch.empty((H, W), dtype=torch.float32, device=img.device)
                mask = torch.empty((H, W), dtype=torch.uint8, device=img.device)
            else:
                pinned = img.is_pinned()
                clean = torch.empty((H, W), dtype=torch.float32, pin_memory=pinned)
                mask = torch.empty((H, W), dtype=torch.uint8, pin_memory=pinned)
            p_img, p_clean, p_mask = img.data_ptr(), clean.data_ptr(), mask.data_ptr()
        else:
            img = np.ascontiguousarray(img, dtype=np.float32)
            H, W = img.shape
            clean = np.empty((H, W), np.float32)
            mask = np.empty((H, W), np.uint8)
            p_img, p_clean, p_mask = img.ctypes.data, clean.ctypes.data, mask.ctypes.data
        rid = ctypes.c_int64(0)
        _lib.check("crb_server_submit", _lib.lib().crb_server_submit(
            self.handle, p_img, H, W, gain, readnoise, sky, sigclip, sigfrac, objlim,
            niter, p_clean, p_mask, ctypes.byref(rid)))
        self._outs[rid.value] = (img, clean, mask)    # keep buffers alive until done
        return rid.value

    def poll(self) -> List[Tuple[int, float, np.ndarray, np.ndarray]]:
        """Completed requests: (id, latency s, clean, mask)."""
        n = ctypes.c_int32(0)
        _lib.check("crb_server_poll", _lib.lib().crb_server_poll(
            self.handle, self._ids, self._lat, 256, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            rid = int(self._ids[i])
            _, clean, mask = self._outs.pop(rid)
            if not isinstance(clean, np.ndarray) and not clean.is_cuda:
                clean, mask = clean.numpy(), mask.numpy()
            out.append((rid, float(self._lat[i]), clean, mask))
        return out

    def pending(self) -> int:
        return int(_lib.lib().crb_server_pending(self.handle))

    def drain(self, timeout_s: float = 120.0):
        res = []
        t0 = time.perf_counter()
        while self.pending():
            res += self.poll()
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError("server did not drain")
        return res

    def close(self) -> None:
        if self.handle:
            _lib.lib().crb_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class TraceResult:
    n: int
    wall_s: float
    pixels: int
    latencies: np.ndarray           # seconds, in completion order
    results: Dict[int, Tuple[np.ndarray, np.ndarray]]

    def summary(self) -> dict:
        lat = np.sort(self.latencies)
        return {"requests": self.n, "wall_s": round(self.wall_s, 3),
                "frames_per_s": round(self.n / self.wall_s, 2),
                "mpix_per_s": round(self.pixels / self.wall_s / 1e6, 1),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "max_ms": round(float(lat[-1]) * 1e3, 3)}


def replay(server: Server, arrivals: Sequence[float], frames: Sequence, params: Sequence[dict],
           keep_results: bool = False, time_limit_s: float = 600.0) -> TraceResult:
    """Submit frame i at arrivals[i] seconds after the start (real time), polling the
    server in between; returns when every request has completed."""
    order = np.argsort(np.asarray(arrivals), kind="stable")
    t0 = time.perf_counter()
    i = 0
    n = len(order)
    lat = []
    results = {}
    idmap = {}
    px = 0
    while i < n or server.pending():
        now = time.perf_counter() - t0
        while i < n and arrivals[order[i]] <= now:
            j = int(order[i])
            rid = server.submit(frames[j], **params[j])
            idmap[rid] = j
            px += frames[j].shape[0] * frames[j].shape[1]
            i += 1
        for rid, l, clean, mask in server.poll():
            lat.append(l)
            if keep_results:
                results[idmap[rid]] = (clean, mask)
        if now > time_limit_s:
            raise TimeoutError("trace replay exceeded its time limit")
    wall = time.perf_counter() - t0
    return TraceResult(n, wall, px, np.asarray(lat), results)
