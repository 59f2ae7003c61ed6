"""Seeded synthetic CCD frames for L.A.Cosmic workloads.

This module only draws inputs: it holds none of the cosmic-ray detection or
cleaning arithmetic, and it is the one piece shared by the FP64 oracle tests
and the GPU path.  Every frame is a function of its seed (numpy PCG64).

The frames stand in for the HST WFPC2 frame the paper processes (Section 5:
an 800x800 WF3 frame, gain 7, read noise 5), which is not available here.
Each frame is built as

    electrons = sky + sum(stars) + sum(galaxies)
    noisy     = Poisson(electrons) + Normal(0, read_noise)
    adu       = noisy / gain  +  cosmic-ray hits (amplitude / gain)

Stars are pixel-integrated Gaussians (differences of erf), galaxies are 2-D
exponential discs rendered with 3x3 sub-sampling, and cosmic-ray hits are
rasterised line segments of constant amplitude, 1 or 2 pixels wide.

Workloads (sizes and parameters, see ``workload``):
  c1  one 256x256 frame, sky 100 e-, gain 1, read noise 5, 30 stars, 50 hits
  c2  one 800x800 frame shaped like a WFPC2 frame, 2% of pixels hit
  c3  one 4096x4096 crowded field, power-law star fluxes, 1.5% hit
  c4  64 frames of four sizes with per-frame gain and read noise
  c5  a Poisson request stream over the c4 sizes (serving)
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Tuple

import numpy as np
from scipy.special import erf

FWHM_TO_SIGMA = 1.0 / 2.3548200450309493


@dataclasses.dataclass
class Frame:
    """One synthetic frame plus the parameters it is cleaned with."""

    img: np.ndarray           # float32 (H, W), ADU
    gain: float               # electrons per ADU
    readnoise: float          # electrons
    sky: float = 0.0          # sky already subtracted from img, ADU (0: not subtracted)
    sigclip: float = 4.5
    sigfrac: float = 0.3
    objlim: float = 4.0
    niter: int = 4
    truth: Optional[np.ndarray] = None    # noiseless electrons/gain (float64), no hits
    hits: Optional[np.ndarray] = None     # bool (H, W): pixels touched by a hit
    seed: int = 0
    name: str = ""

    @property
    def shape(self) -> Tuple[int, int]:
        return self.img.shape

    def params(self) -> dict:
        return dict(gain=self.gain, readnoise=self.readnoise, sky=self.sky,
                    sigclip=self.sigclip, sigfrac=self.sigfrac, objlim=self.objlim,
                    niter=self.niter)

    def sha256(self) -> str:
        return hashlib.sha256(np.ascontiguousarray(self.img).tobytes()).hexdigest()


# ----------------------------------------------------------------------------
# rendering helpers
# ----------------------------------------------------------------------------

def _add_gaussian_stars(e: np.ndarray, rng: np.random.Generator, n: int, fwhm: float,
                        fluxes: np.ndarray) -> None:
    H, W = e.shape
    sig = fwhm * FWHM_TO_SIGMA
    xc = rng.uniform(0.0, W, n)
    yc = rng.uniform(0.0, H, n)
    rad = int(math.ceil(5.0 * sig)) + 1
    off = np.arange(-rad, rad + 1)
    s2 = math.sqrt(2.0) * sig
    for i in range(n):
        ix, iy = int(round(xc[i])), int(round(yc[i]))
        xs = ix + off
        ys = iy + off
        # fraction of the Gaussian falling in each pixel [x-0.5, x+0.5)
        fx = 0.5 * (erf((xs + 0.5 - xc[i]) / s2) - erf((xs - 0.5 - xc[i]) / s2))
        fy = 0.5 * (erf((ys + 0.5 - yc[i]) / s2) - erf((ys - 0.5 - yc[i]) / s2))
        mx = (xs >= 0) & (xs < W)
        my = (ys >= 0) & (ys < H)
        if not mx.any() or not my.any():
            continue
        stamp = fluxes[i] * np.outer(fy[my], fx[mx])
        e[ys[my][0]:ys[my][-1] + 1, xs[mx][0]:xs[mx][-1] + 1] += stamp


def _add_exponential_galaxies(e: np.ndarray, rng: np.random.Generator, n: int,
                              flux_median: float, flux_sigma_ln: float) -> None:
    H, W = e.shape
    xc = rng.uniform(0.0, W, n)
    yc = rng.uniform(0.0, H, n)
    h = rng.uniform(2.0, 6.0, n)
    q = rng.uniform(0.3, 1.0, n)
    pa = rng.uniform(0.0, math.pi, n)
    flux = flux_median * np.exp(flux_sigma_ln * rng.standard_normal(n))
    sub = (np.arange(3) - 1.0) / 3.0          # 3x3 sub-pixel centres
    for i in range(n):
        rad = int(math.ceil(8.0 * h[i]))
        ix, iy = int(round(xc[i])), int(round(yc[i]))
        xs = ix + np.arange(-rad, rad + 1)
        ys = iy + np.arange(-rad, rad + 1)
        gx = (xs[None, :, None, None] + sub[None, None, None, :]) - xc[i]
        gy = (ys[:, None, None, None] + sub[None, None, :, None]) - yc[i]
        c, s = math.cos(pa[i]), math.sin(pa[i])
        u = c * gx + s * gy
        v = (-s * gx + c * gy) / q[i]
        prof = np.exp(-np.sqrt(u * u + v * v) / h[i]).sum(axis=(2, 3))
        prof *= flux[i] / prof.sum()
        mx = (xs >= 0) & (xs < W)
        my = (ys >= 0) & (ys < H)
        if not mx.any() or not my.any():
            continue
        e[ys[my][0]:ys[my][-1] + 1, xs[mx][0]:xs[mx][-1] + 1] += prof[np.ix_(my, mx)]


def _raster_hits(rng: np.random.Generator, H: int, W: int, n: int, lmin: int, lmax: int,
                 amp_lo: float, amp_hi: float):
    """Rasterise n hits; returns (flat pixel index, amplitude in e-) per hit pixel."""
    x0 = rng.uniform(0.0, W, n)
    y0 = rng.uniform(0.0, H, n)
    L = rng.integers(lmin, lmax + 1, n)
    w = rng.integers(1, 3, n)
    th = rng.uniform(0.0, math.pi, n)
    A = rng.uniform(amp_lo, amp_hi, n)
    idx_all = []
    amp_all = []
    for i in range(n):
        t = np.arange(L[i])
        c, s = math.cos(th[i]), math.sin(th[i])
        px = np.rint(x0[i] + t * c)
        py = np.rint(y0[i] + t * s)
        if w[i] == 2:
            px = np.concatenate([px, np.rint(x0[i] + t * c - s)])
            py = np.concatenate([py, np.rint(y0[i] + t * s + c)])
        ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)
        flat = np.unique(py[ok].astype(np.int64) * W + px[ok].astype(np.int64))
        idx_all.append(flat)
        amp_all.append(np.full(flat.size, A[i]))
    if not idx_all:
        return np.zeros(0, np.int64), np.zeros(0)
    return np.concatenate(idx_all), np.concatenate(amp_all)


def render(H: int, W: int, seed: int, *, sky_e: float, gain: float, readnoise: float,
           n_stars: int, star_fwhm: float, star_flux: str, star_flux_median: float = 5000.0,
           star_flux_sigma_ln: float = 1.0, n_galaxies: int = 0,
           gal_flux_median: float = 2.0e4, n_hits: int = 0, hit_coverage: float = 0.0,
           hit_len: Tuple[int, int] = (1, 5), hit_amp: Tuple[float, float] = (200.0, 5000.0),
           name: str = "") -> Frame:
    """Render one frame.  ``star_flux`` is 'lognormal' or 'powerlaw'."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e = np.full((H, W), float(sky_e))
    if n_stars:
        if star_flux == "lognormal":
            flux = star_flux_median * np.exp(star_flux_sigma_ln * rng.standard_normal(n_stars))
        elif star_flux == "powerlaw":
            # cumulative N(>F) proportional to F^-1.5, truncated to [200, 2e5] e-
            fmin, fmax = 200.0, 2.0e5
            umin = (fmax / fmin) ** -1.5
            u = rng.uniform(umin, 1.0, n_stars)
            flux = fmin * u ** (-1.0 / 1.5)
        else:
            raise ValueError(star_flux)
        _add_gaussian_stars(e, rng, n_stars, star_fwhm, flux)
    if n_galaxies:
        _add_exponential_galaxies(e, rng, n_galaxies, gal_flux_median, 1.0)
    truth = e / gain
    noisy = rng.poisson(e).astype(np.float64) + rng.normal(0.0, readnoise, e.shape)
    adu = noisy / gain
    hits = np.zeros(H * W, dtype=bool)
    add = np.zeros(H * W)
    if n_hits:
        idx, amp = _raster_hits(rng, H, W, n_hits, hit_len[0], hit_len[1], *hit_amp)
        np.add.at(add, idx, amp)
        hits[idx] = True
    if hit_coverage > 0.0:
        target = hit_coverage * H * W
        mean_px = 0.75 * (hit_len[0] + hit_len[1])   # ~ pixels per hit (w averages 1.5)
        while hits.sum() < target:
            need = target - hits.sum()
            n = max(16, int(need / mean_px * 1.05))
            idx, amp = _raster_hits(rng, H, W, n, hit_len[0], hit_len[1], *hit_amp)
            np.add.at(add, idx, amp)
            hits[idx] = True
    adu = adu + (add / gain).reshape(H, W)
    return Frame(img=adu.astype(np.float32), gain=float(gain), readnoise=float(readnoise),
                 truth=truth, hits=hits.reshape(H, W), seed=seed, name=name)


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

C4_SIZES = ((800, 800), (1024, 1024), (2048, 4096), (4096, 2048))   # (H, W)


def c1(seed: int = 1) -> Frame:
    """256x256: sky 100 e-, gain 1, rn 5, 30 stars (FWHM 2, lognormal median 5000 e-),
    50 hits 1-5 px long, 1-2 px wide, amplitude U(200, 5000) e-."""
    return render(256, 256, seed, sky_e=100.0, gain=1.0, readnoise=5.0, n_stars=30,
                  star_fwhm=2.0, star_flux="lognormal", n_hits=50, hit_len=(1, 5),
                  hit_amp=(200.0, 5000.0), name="c1-256x256")


def c2(seed: int = 2) -> Frame:
    """800x800 WFPC2-like: sky 50 e-, gain 7, rn 5, 400 stars FWHM 1.5, 300 exponential
    galaxies (scale 2-6 px), hits covering 2% of pixels, 1-20 px, U(100, 10000) e-."""
    return render(800, 800, seed, sky_e=50.0, gain=7.0, readnoise=5.0, n_stars=400,
                  star_fwhm=1.5, star_flux="lognormal", n_galaxies=300,
                  gal_flux_median=2.0e4, hit_coverage=0.02, hit_len=(1, 20),
                  hit_amp=(100.0, 10000.0), name="c2-800x800")


def c3(seed: int = 3, size: int = 4096) -> Frame:
    """4096x4096 crowded field: sky 200 e-, gain 1.5, rn 4, 20000 stars FWHM 2.5 with
    power-law fluxes (slope -1.5), hits covering 1.5% of pixels (c2's lengths/amplitudes).
    ``size`` shrinks the frame keeping densities (for tests)."""
    n_stars = int(round(20000 * (size * size) / (4096 * 4096)))
    return render(size, size, seed, sky_e=200.0, gain=1.5, readnoise=4.0, n_stars=n_stars,
                  star_fwhm=2.5, star_flux="powerlaw", hit_coverage=0.015, hit_len=(1, 20),
                  hit_amp=(100.0, 10000.0), name=f"c3-{size}x{size}")


def c1_density_frame(H: int, W: int, seed: int, gain: float, readnoise: float,
                     name: str = "") -> Frame:
    """A frame of any size with c1's star and hit densities (30 stars and 50 hits per
    65,536 px), sky 100 e-; used by the mixed-size batch and the request stream."""
    scale = (H * W) / 65536.0
    return render(H, W, seed, sky_e=100.0, gain=gain, readnoise=readnoise,
                  n_stars=int(round(30 * scale)), star_fwhm=2.0, star_flux="lognormal",
                  n_hits=int(round(50 * scale)), hit_len=(1, 5), hit_amp=(200.0, 5000.0),
                  name=name or f"{H}x{W}")


def c4_frame(i: int, sizes=C4_SIZES, per_size: int = 16, base_seed: int = 4000) -> Frame:
    """Frame i of the mixed-size batch: size sizes[i // per_size], seed base_seed + i,
    gain U(1,8) and read noise U(3,8) e- from a generator keyed by the seed."""
    H, W = sizes[i // per_size]
    seed = base_seed + i
    prng = np.random.Generator(np.random.PCG64(seed + 10_000_000))
    g = float(np.float32(prng.uniform(1.0, 8.0)))
    rn = float(np.float32(prng.uniform(3.0, 8.0)))
    return c1_density_frame(H, W, seed, g, rn, name=f"c4[{i}]-{H}x{W}")


def c4(sizes=C4_SIZES, per_size: int = 16, base_seed: int = 4000) -> List[Frame]:
    """64 frames: 16 each of 800x800, 1024x1024, 2048x4096, 4096x2048 (H x W); per-frame
    gain U(1,8) and read noise U(3,8) e-, frame i seeded with 4000+i."""
    return [c4_frame(i, sizes, per_size, base_seed) for i in range(len(sizes) * per_size)]


@dataclasses.dataclass
class Request:
    t_arrival: float     # seconds since stream start
    H: int
    W: int
    seed: int
    gain: float
    readnoise: float


def c5_stream(rate: float = 40.0, duration: float = 60.0, seed: int = 5,
              sizes=C4_SIZES, base_seed: int = 5000) -> List[Request]:
    """Poisson arrivals at ``rate`` frames/s over ``duration`` s; request j has its own
    seed 5000+j, a size drawn uniformly from ``sizes``, gain U(1,8), read noise U(3,8)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    j = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        H, W = sizes[int(rng.integers(0, len(sizes)))]
        g = float(np.float32(rng.uniform(1.0, 8.0)))
        rn = float(np.float32(rng.uniform(3.0, 8.0)))
        out.append(Request(t, H, W, base_seed + j, g, rn))
        j += 1
    return out


def request_frame(r: Request) -> Frame:
    return c1_density_frame(r.H, r.W, r.seed, r.gain, r.readnoise, name=f"req{r.seed}")


def constant(H: int, W: int, value: float, gain: float = 1.0, readnoise: float = 5.0) -> Frame:
    """A frame whose every pixel has one value (the paper's constant test images
    hold 24.3 and 137)."""
    return Frame(img=np.full((H, W), value, dtype=np.float32), gain=gain, readnoise=readnoise)


def workload(name: str) -> List[Frame]:
    name = name.lower()
    if name == "c1":
        return [c1()]
    if name == "c2":
        return [c2()]
    if name == "c3":
        return [c3()]
    if name == "c4":
        return c4()
    raise ValueError(name)
