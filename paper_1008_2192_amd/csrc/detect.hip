// Detection kernel of libcrb for gfx950 (MI355X): the first stage of an L.A.Cosmic
// iteration (Mighell, Section 5) -- L+ (2x-subsampled clipped Laplacian, rebinned),
// N from med5(J), S = L+/(2N), S' = S - med5(S), F^ from med3(J) - med7(med3(J)),
// the first selection and the two threshold bits the grow reads -- on 32 x 64 LDS
// tiles with the halo each quantity needs, plus the parity-test kernels of its median
// networks.
//
// Numerics: medians are exact selections by min/max networks on FP32 (J, med3) or
// binary64 (S).  The statistics are binary64, evaluated in the same operation order
// as the plain definition (no contraction: built with -ffp-contract=off), so a
// decision on a given J is independent of the tiling and of the launch shape.
#include "kernels.h"
#include "device_common.h"

#include <math.h>

namespace crb {

#include "medtile.inc"

// 3x3 medians of a run of N horizontally adjacent outputs from three rows of N+2
// inputs.  Each column of three is sorted once (shared by up to three windows);
// the median of a 3x3 window with sorted columns is the median of
// (max of the column minima, median of the column medians, min of the column maxima).
template <int N>
__device__ __forceinline__ void med3_run(const float (&a)[N + 2], const float (&b)[N + 2],
                                         const float (&c)[N + 2], float (&o)[N]) {
    float lo[N + 2], mi[N + 2], hi[N + 2];
#pragma unroll
    for (int j = 0; j < N + 2; ++j) {
        lo[j] = min3f(a[j], b[j], c[j]);
        mi[j] = med3f(a[j], b[j], c[j]);
        hi[j] = max3f(a[j], b[j], c[j]);
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
        o[j] = med3f(max3f(lo[j], lo[j + 1], lo[j + 2]), med3f(mi[j], mi[j + 1], mi[j + 2]),
                     min3f(hi[j], hi[j + 1], hi[j + 2]));
}

// The four sub-pixels of the 2x block of a pixel of value c each have two
// neighbours inside the block (value c) and two outside (u above or d below,
// l left or r right).  Clipped Laplacian 4c - u - d - l - r of each, in that order,
// then the 2x2 mean, matching the literal 2x-grid computation term for term.
__device__ __forceinline__ double lplus(double c, double u, double d, double l, double r) {
    double s00 = 4.0 * c - u - c - l - c;
    double s01 = 4.0 * c - u - c - c - r;
    double s10 = 4.0 * c - c - d - l - c;
    double s11 = 4.0 * c - c - d - c - r;
    s00 = s00 > 0.0 ? s00 : 0.0;
    s01 = s01 > 0.0 ? s01 : 0.0;
    s10 = s10 > 0.0 ? s10 : 0.0;
    s11 = s11 > 0.0 ? s11 : 0.0;
    return (s00 + s01 + s10 + s11) / 4.0;
}

// ---------------------------------------------------------------------------
// detection
// ---------------------------------------------------------------------------

// Work shapes inside a detection block: med3 in runs of kRun3 outputs; med5(J) with
// L+, N, S in 2 x 5 thread tiles over the whole tile and its 2-pixel apron.  The
// remaining statistics are evaluated only where a code bit can matter (below).
constexpr int kRun3 = 14;

template <int TY, int TX>
struct DetectLayout {
    // logical extents of the LDS planes and their row pitches; the pitches spread the
    // stage-1 and stage-2 scalar accesses over the LDS banks
    static constexpr int JH = TY + 8, JW = TX + 8, JWP = TX + 11;   // J, apron 4
    static constexpr int MH = TY + 6, MW = TX + 6, MWP = TX + 12;   // med3(J), apron 3
    static constexpr int SH = TY + 4, SW = TX + 4, SWP = TX + 6;    // S (binary64), apron 2
    static constexpr int HW = (SW + 31) / 32;   // words per row of the S > sigclip bitmap
    static constexpr int QW = TX / 32;          // words per row of the work bitmap
    // after stage 2 the J buffer holds the code tile, the work bitmap and its prefix
    static constexpr int kCodeWords = TY * TX / 4;
    static constexpr int kWorkWords = TY * QW;
    static_assert(TX % 32 == 0 && kWorkWords == 64, "one wave builds the work bitmap");
    static_assert(QW + 1 <= HW, "dilation reads two bitmap words per work word");
    static_assert(JH * JWP >= kCodeWords + 2 * kWorkWords + 1, "J buffer reuse");
};

// Which pixels need S', F^ and the threshold bits.  With H = {S > sigclip} (S' > t
// implies S > t for t >= 0: med5(S) >= 0 because S >= 0, and rounding is monotone):
//   first(p) can be 1 only on H;
//   G1(p) needs an A pixel within distance 1, so hi(p) matters only on D1(H);
//   G2(p) needs a G1 pixel within distance 1, so lo(p) matters only on D2(H);
// and lo(p) = hi(p) = 0 wherever S(p) <= sigfrac * sigclip (sigfrac <= 1).  The
// block therefore evaluates med5(S) and the bits on Q = D2(H) & {S > sigfrac*sigclip}
// (the work set), med7(med3) and the contrast test on Q & {S' > sigclip}, and writes
// code 0 elsewhere; the codes agree with the full definition wherever the grow reads
// them through its two dilations.
template <int TY, int TX>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
void k_detect(const DevFrame *__restrict__ frames, const TileRef *__restrict__ tiles,
              DevFrame single, int kiter) {
    using L = DetectLayout<TY, TX>;
    __shared__ __align__(16) float sJ[L::JH * L::JWP];     // J, later codes + work bitmap
    __shared__ __align__(16) float sM3[L::MH * L::MWP];
    __shared__ __align__(16) double sS[L::SH * L::SWP];
    __shared__ float sM5[TY * TX];                          // med5(J) at the outputs
    __shared__ uint32_t sHot[L::SH * L::HW];                // S > sigclip, apron 2, in-frame
    __shared__ unsigned int sContrast;                      // contrast tests (work counting)
    uint8_t *const sCode = reinterpret_cast<uint8_t *>(sJ);
    uint32_t *const sQ = reinterpret_cast<uint32_t *>(sJ) + L::kCodeWords;
    uint32_t *const sQpre = sQ + L::kWorkWords;

    DevFrame f;
    int y0, x0;
    if (tiles) {
        const TileRef t = tiles[blockIdx.x];
        f = frames[t.frame];
        y0 = t.y0;
        x0 = t.x0;
    } else {
        f = single;
        y0 = blockIdx.y * TY;
        x0 = blockIdx.x * TX;
    }
    const int k = kiter ? kiter : f.k;
    if (frame_skips(f, k))
        return;
    const int H = f.H, W = f.W, tid = threadIdx.x;
    // iteration 1 reads the input frame and initialises J with the tile's own pixels
    const float *__restrict__ J = (k == 1) ? f.img : f.J;
    const double sigclip = f.sigclip;
    const double lowlim = (double)f.sigfrac * (double)f.sigclip;

    for (int i = tid; i < L::SH * L::HW; i += kThreads)
        sHot[i] = 0u;
    if (tid == 0)
        sContrast = 0u;
    // J over [y0-4, y0+TY+4) x [x0-4, x0+TX+4), clamped reads: all of a thread's
    // loads are issued before the first LDS store, so their latencies overlap
    {
        constexpr int NJ = L::JH * L::JW, NB = (NJ + kThreads - 1) / kThreads;
        float v[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int i = tid + b * kThreads;
            if (i < NJ) {
                const int r = i / L::JW, c = i - r * L::JW;
                v[b] = J[(size_t)clampi(y0 - 4 + r, H) * W + clampi(x0 - 4 + c, W)];
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int i = tid + b * kThreads;
            if (i < NJ) {
                const int r = i / L::JW, c = i - r * L::JW;
                sJ[r * L::JWP + c] = v[b];
            }
        }
    }
    __syncthreads();
    if (k == 1 && f.img != f.J) {
        for (int i = tid; i < TY * TX; i += kThreads) {
            const int r = i / TX, c = i - r * TX;
            if (y0 + r < H && x0 + c < W)
                f.J[(size_t)(y0 + r) * W + x0 + c] = sJ[(r + 4) * L::JWP + c + 4];
        }
    }

    // med3(J) over [y0-3, y0+TY+3) x [x0-3, x0+TX+3)
    {
        constexpr int NRX = (L::MW + kRun3 - 1) / kRun3;
        for (int t = tid; t < L::MH * NRX; t += kThreads) {
            const int r = t / NRX;
            const int cx = min((t - r * NRX) * kRun3, L::MW - kRun3);
            float a[kRun3 + 2], b[kRun3 + 2], c[kRun3 + 2], o[kRun3];
#pragma unroll
            for (int j = 0; j < kRun3 + 2; ++j) {
                a[j] = sJ[r * L::JWP + cx + j];
                b[j] = sJ[(r + 1) * L::JWP + cx + j];
                c[j] = sJ[(r + 2) * L::JWP + cx + j];
            }
            med3_run<kRun3>(a, b, c, o);
#pragma unroll
            for (int j = 0; j < kRun3; ++j)
                sM3[r * L::MWP + cx + j] = o[j];
        }
    }

    // med5(J), L+, N and S over [y0-2, y0+TY+2) x [x0-2, x0+TX+2); marks H
    {
        constexpr int TTY = 2, TTX = 5, PW = TTX + 4;
        constexpr int NTY = (L::SH + TTY - 1) / TTY, NTX = (L::SW + TTX - 1) / TTX;
        const double gain = f.gain, sky = f.sky, rn = f.readnoise;
        const double rn2 = rn * rn;
        for (int t = tid; t < NTY * NTX; t += kThreads) {
            const int ty = t / NTX;
            const int r = min(ty * TTY, L::SH - TTY);
            const int c = min((t - ty * NTX) * TTX, L::SW - TTX);
            float v[(TTY + 4) * PW], m5[TTY * TTX];
#pragma unroll
            for (int i = 0; i < TTY + 4; ++i)
#pragma unroll
                for (int j = 0; j < PW; ++j)
                    v[i * PW + j] = sJ[(r + i) * L::JWP + c + j];
            med5_t2x5(v, m5);
#pragma unroll
            for (int i = 0; i < TTY; ++i) {
#pragma unroll
                for (int j = 0; j < TTX; ++j) {
                    const int pc = (i + 2) * PW + (j + 2);
                    const double lp = lplus(v[pc], v[pc - PW], v[pc + PW], v[pc - 1], v[pc + 1]);
                    double m = (double)m5[i * TTX + j] + sky;
                    if (m <= 0.0)
                        m = 1e-4;
                    const double N = sqrt(gain * m + rn2) / gain;
                    const double S = lp / (2.0 * N);
                    sS[(r + i) * L::SWP + c + j] = S;
                    const int cy = r + i - 2, cxx = c + j - 2;
                    if (cy >= 0 && cy < TY && cxx >= 0 && cxx < TX)
                        sM5[cy * TX + cxx] = m5[i * TTX + j];
                    const int gy = y0 + cy, gx = x0 + cxx;
                    if (S > sigclip && gy >= 0 && gy < H && gx >= 0 && gx < W)
                        atomicOr(&sHot[(r + i) * L::HW + ((c + j) >> 5)], 1u << ((c + j) & 31));
                }
            }
        }
    }
    __syncthreads();

    // Region cells outside the image must hold the value of their clamped cell:
    // the windows of the work set read med3 and S at clamped neighbour positions.
    if (y0 < 3 || x0 < 3 || y0 + TY + 3 > H || x0 + TX + 3 > W) {
        for (int i = tid; i < L::MH * L::MW; i += kThreads) {
            const int r = i / L::MW, c = i - r * L::MW;
            const int gy = y0 - 3 + r, gx = x0 - 3 + c;
            if (gy < 0 || gy >= H || gx < 0 || gx >= W)
                sM3[r * L::MWP + c] =
                    sM3[(clampi(gy, H) - (y0 - 3)) * L::MWP + (clampi(gx, W) - (x0 - 3))];
        }
        for (int i = tid; i < L::SH * L::SW; i += kThreads) {
            const int r = i / L::SW, c = i - r * L::SW;
            const int gy = y0 - 2 + r, gx = x0 - 2 + c;
            if (gy < 0 || gy >= H || gx < 0 || gx >= W)
                sS[r * L::SWP + c] =
                    sS[(clampi(gy, H) - (y0 - 2)) * L::SWP + (clampi(gx, W) - (x0 - 2))];
        }
    }
    // the J buffer is free: clear the code tile
    for (int i = tid; i < L::kCodeWords; i += kThreads)
        reinterpret_cast<uint32_t *>(sJ)[i] = 0u;
    // work bitmap Q = D2(H) & {S > sigfrac*sigclip} on the tile's in-frame pixels, one
    // 32-pixel word per lane of the first wave, and its prefix sum of pixel counts
    if (tid < L::kWorkWords) {
        const int r = tid / L::QW, w = tid - r * L::QW;
        unsigned long long x = 0ull;
#pragma unroll
        for (int dr = 0; dr < 5; ++dr) {
            const uint32_t *row = &sHot[(r + dr) * L::HW + w];
            x |= (unsigned long long)row[0] | ((unsigned long long)row[1] << 32);
        }
        // bit b of the dilation covers region columns 32w+b .. 32w+b+4, centred on
        // the tile column 32w+b
        uint32_t q = (uint32_t)(x | (x >> 1) | (x >> 2) | (x >> 3) | (x >> 4));
        const int vc = W - x0 - 32 * w;
        if (y0 + r >= H || vc <= 0)
            q = 0u;
        else if (vc < 32)
            q &= (1u << vc) - 1u;
        for (uint32_t m = q; m; m &= m - 1u) {
            const int b = __ffs(m) - 1;
            if (!(sS[(r + 2) * L::SWP + 32 * w + b + 2] > lowlim))
                q &= ~(1u << b);
        }
        sQ[tid] = q;
        int v = __popc(q);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int u = __shfl_up(v, off);
            if (tid >= off)
                v += u;
        }
        sQpre[tid + 1] = (uint32_t)v;
        if (tid == 0)
            sQpre[0] = 0u;
    }
    __syncthreads();

    // the work set, compacted: thread t takes the t-th, (t+256)-th, ... pixel of Q
    {
        const int total = (int)sQpre[L::kWorkWords];
        const double objlim = f.objlim;
        const double gain = f.gain, sky = f.sky, rn = f.readnoise;
        const double rn2 = rn * rn;
        unsigned int ncontrast = 0u;
        for (int qi = tid; qi < total; qi += kThreads) {
            int lo = 0, hi = L::kWorkWords - 1;    // last word whose prefix is <= qi
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((int)sQpre[mid] <= qi)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            uint32_t bits = sQ[lo];
            for (int n = qi - (int)sQpre[lo]; n > 0; --n)
                bits &= bits - 1u;
            const int r = lo / L::QW, c = (lo - r * L::QW) * 32 + (__ffs(bits) - 1);
            double v[25], ms[1];
#pragma unroll
            for (int i = 0; i < 5; ++i)
#pragma unroll
                for (int j = 0; j < 5; ++j)
                    v[i * 5 + j] = sS[(r + i) * L::SWP + c + j];
            med5_t1x1(v, ms);
            const double sp = v[12] - ms[0];
            const bool hbit = sp > sigclip;
            const bool lbit = sp > lowlim;
            bool first = false;
            if (hbit) {
                // N as in the S stage, from the stored med5(J)
                double m = (double)sM5[r * TX + c] + sky;
                if (m <= 0.0)
                    m = 1e-4;
                const double N = sqrt(gain * m + rn2) / gain;
                float w7[49], m7[1];
#pragma unroll
                for (int i = 0; i < 7; ++i)
#pragma unroll
                    for (int j = 0; j < 7; ++j)
                        w7[i * 7 + j] = sM3[(r + i) * L::MWP + c + j];
                med7_t1x1(w7, m7);
                double fh = ((double)w7[24] - (double)m7[0]) / N;
                if (fh < 0.01)
                    fh = 0.01;
                first = sp / fh > objlim;
                ++ncontrast;
            }
            sCode[r * TX + c] = (uint8_t)((first ? 1 : 0) | (hbit ? 2 : 0) | (lbit ? 4 : 0));
        }
        if ((f.flags & kCountWork) && ncontrast)
            atomicAdd(&sContrast, ncontrast);
        __syncthreads();

        // codes of the tile, 8 per thread
        uint8_t *__restrict__ codes = f.codes;
        for (int i = tid; i < TY * TX / 8; i += kThreads) {
            const int r = i / (TX / 8), c = (i - r * (TX / 8)) * 8;
            const int gy = y0 + r, gx = x0 + c;
            if (gy >= H || gx >= W)
                continue;
            uint8_t *dst = codes + (size_t)gy * W + gx;
            const uint2 word = *reinterpret_cast<const uint2 *>(&sCode[r * TX + c]);
            if (gx + 8 <= W && ((uintptr_t)dst & 7u) == 0u) {
                *reinterpret_cast<uint2 *>(dst) = word;
            } else {
                const int nb = min(8, W - gx);
                for (int b = 0; b < nb; ++b)
                    dst[b] = sCode[r * TX + c + b];
            }
        }
        if ((f.flags & kCountWork) && tid == 0 && f.work) {
            if (total)
                atomicAdd(&f.work[0], (unsigned long long)total);
            if (sContrast)
                atomicAdd(&f.work[1], (unsigned long long)sContrast);
        }
    }
}

// ---------------------------------------------------------------------------
// parity-test kernels: the median networks alone
// ---------------------------------------------------------------------------

template <int R>
__global__ __launch_bounds__(kThreads) void k_debug_median(const float *__restrict__ in, int H,
                                                           int W, float *__restrict__ out) {
    constexpr int TY = (R == 2) ? 2 : 1, TX = (R == 1) ? kRun3 : (R == 2 ? 5 : 1);
    constexpr int PH = TY + 2 * R, PW = TX + 2 * R;
    const int ntx = (W + TX - 1) / TX, nty = (H + TY - 1) / TY;
    const int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= ntx * nty)
        return;
    const int y0 = (t / ntx) * TY, x0 = (t % ntx) * TX;
    float v[PH * PW], o[TY * TX];
#pragma unroll
    for (int i = 0; i < PH; ++i)
#pragma unroll
        for (int j = 0; j < PW; ++j)
            v[i * PW + j] = in[(size_t)clampi(y0 - R + i, H) * W + clampi(x0 - R + j, W)];
    if constexpr (R == 1) {
        float a[kRun3 + 2], b[kRun3 + 2], c[kRun3 + 2];
#pragma unroll
        for (int j = 0; j < kRun3 + 2; ++j) {
            a[j] = v[j];
            b[j] = v[PW + j];
            c[j] = v[2 * PW + j];
        }
        med3_run<kRun3>(a, b, c, o);
    } else if constexpr (R == 2) {
        med5_t2x5(v, o);
    } else {
        med7_t1x1(v, o);
    }
#pragma unroll
    for (int i = 0; i < TY; ++i)
#pragma unroll
        for (int j = 0; j < TX; ++j)
            if (y0 + i < H && x0 + j < W)
                out[(size_t)(y0 + i) * W + x0 + j] = o[i * TX + j];
}

// 5x5 clamped median of binary64 values by the single-output network the detection
// kernel applies to S.
__global__ __launch_bounds__(kThreads) void k_debug_median5_f64(const double *__restrict__ in,
                                                                int H, int W,
                                                                double *__restrict__ out) {
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t >= (long long)H * W)
        return;
    const int y = (int)(t / W), x = (int)(t - (long long)y * W);
    double v[25], o[1];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j)
            v[i * 5 + j] = in[(size_t)clampi(y - 2 + i, H) * W + clampi(x - 2 + j, W)];
    med5_t1x1(v, o);
    out[t] = o[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_detect(const DevFrame *d_frames, const TileRef *d_tiles, int ntiles,
                         const DevFrame &single, int k, hipStream_t s) {
    if (d_tiles) {
        if (ntiles <= 0)
            return hipSuccess;
        k_detect<kDetectTY, kDetectTX><<<ntiles, kThreads, 0, s>>>(d_frames, d_tiles, single, k);
    } else {
        dim3 grid((single.W + kDetectTX - 1) / kDetectTX, (single.H + kDetectTY - 1) / kDetectTY);
        k_detect<kDetectTY, kDetectTX><<<grid, kThreads, 0, s>>>(nullptr, nullptr, single, k);
    }
    return hipGetLastError();
}

hipError_t launch_debug_median5_f64(const double *in, int H, int W, double *out,
                                   hipStream_t s) {
    const size_t n = (size_t)H * (size_t)W;
    k_debug_median5_f64<<<(unsigned int)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(in, H,
                                                                                         W, out);
    return hipGetLastError();
}

hipError_t launch_debug_median(const float *in, int H, int W, int r, float *out, hipStream_t s) {
    const int ty = (r == 2) ? 2 : 1, tx = (r == 1) ? kRun3 : (r == 2 ? 5 : 1);
    const size_t n = (size_t)((H + ty - 1) / ty) * (size_t)((W + tx - 1) / tx);
    const unsigned int grid = (unsigned int)((n + kThreads - 1) / kThreads);
    if (r == 1)
        k_debug_median<1><<<grid, kThreads, 0, s>>>(in, H, W, out);
    else if (r == 2)
        k_debug_median<2><<<grid, kThreads, 0, s>>>(in, H, W, out);
    else
        k_debug_median<3><<<grid, kThreads, 0, s>>>(in, H, W, out);
    return hipGetLastError();
}

}  // namespace crb
