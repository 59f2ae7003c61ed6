// HIP kernels of libcrb for gfx950 (MI355X): one L.A.Cosmic iteration as three
// launches -- detection, grow/count, replacement -- plus init and stats helpers.
//
// Method (Mighell, Section 5; equations of the iteration as listed in crb.h):
//   detection  : L+ (2x-subsampled clipped Laplacian, rebinned), N from med5(J),
//                S = L+/(2N), S' = S - med5(S), F^ from med3(J) - med7(med3(J)),
//                first selection and the two threshold bits used by the grow;
//   grow/count : two 3x3 dilations gated at sigclip and sigfrac*sigclip, the
//                new-flag count n_k and the cumulative mask;
//   replacement: median of the unflagged clamped 5x5 neighbours of each flagged
//                pixel.
// The paper's subimages with a 6-pixel overlap (Section 6.2) become LDS tiles with
// the halo each stage needs: 4 pixels of J for detection (med7 of med3, and med5
// of S built from a 2-pixel apron of S), 2 pixels of codes for the grow.
//
// Numerics: medians are exact selections by min/max networks on FP32 (J, med3) or
// binary64 (S).  The statistics are binary64, evaluated in the same operation order
// as the plain definition (no contraction: built with -ffp-contract=off), so a
// decision on a given J is independent of the tiling and of the launch shape.
#include "kernels.h"

#include <math.h>

namespace crb {

__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }

#include "medtile.inc"

__device__ __forceinline__ int clampi(int i, int n) { return min(max(i, 0), n - 1); }
__device__ __forceinline__ float med3f(float a, float b, float c) {
    return __builtin_amdgcn_fmed3f(a, b, c);
}
__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }
__device__ __forceinline__ float max3f(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }

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

// Iteration k of frame f is skipped when k exceeds its niter, or (early stop) when
// the previous iteration selected no new pixel: that iteration reproduced its input,
// so every later one would too.
__device__ __forceinline__ bool frame_skips(const DevFrame &f, int k) {
    if (k < 1 || k > f.niter)
        return true;
    if (k == 1 || (f.flags & kNoEarlyStop))
        return false;
    return f.nnew[k - 2] == 0ull;
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
// grow + count + cumulative mask + flagged list
// ---------------------------------------------------------------------------
//
// Word-parallel: a lane holds the codes of 16 horizontally adjacent pixels in four
// dwords (byte j of dword d = pixel 4d + j), so a 3-wide dilation is byte shifts
// inside the lane plus the edge bytes of the neighbouring lanes.  A wave covers 62
// such groups (992 pixels) of a strip of kGrowTY rows; lanes 0 and 63 hold the
// groups just outside the strip, whose inner edge bytes the dilation needs.  Rows
// stream through a delay line: codes of row y give the horizontal dilation of the
// first selection at y, then G1 at y-1 (vertical OR of three rows, gated by
// S' > sigclip), then G2 at y-2 (gated by S' > sigfrac*sigclip).  No LDS and no
// block barrier.  The flagged list is written row by row across the wave, so
// consecutive entries are neighbours in a row.

constexpr uint32_t kByteLsb = 0x01010101u;

struct Px16 {
    uint32_t d[4];
};

__device__ __forceinline__ uint32_t shfl_prev(uint32_t v) {   // value of lane-1
    return (uint32_t)__shfl_up((int)v, 1);
}
__device__ __forceinline__ uint32_t shfl_next(uint32_t v) {   // value of lane+1
    return (uint32_t)__shfl_down((int)v, 1);
}
// 3-wide horizontal OR of byte flags (one flag in bit 0 of each byte)
__device__ __forceinline__ Px16 hdilate(const Px16 &v) {
    const uint32_t left = shfl_prev(v.d[3]) >> 24;          // pixel just left of this lane
    const uint32_t right = shfl_next(v.d[0]) << 24;         // pixel just right of this lane
    Px16 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t lo = q == 0 ? left : (v.d[q - 1] >> 24);
        const uint32_t hi = q == 3 ? right : (v.d[q + 1] << 24);
        o.d[q] = v.d[q] | (v.d[q] << 8) | (v.d[q] >> 8) | lo | hi;
    }
    return o;
}

// 16 bytes of row y starting at pixel x (x multiple of 16); bytes outside read 0
__device__ __forceinline__ Px16 load16(const uint8_t *__restrict__ p, int y, int x, int H, int W,
                                       bool aligned) {
    Px16 v = {{0u, 0u, 0u, 0u}};
    if (y < 0 || y >= H || x + 16 <= 0 || x >= W)
        return v;
    const uint8_t *row = p + (size_t)y * W;
    if (aligned && x >= 0) {
        const uint4 q = *reinterpret_cast<const uint4 *>(row + x);
        v.d[0] = q.x; v.d[1] = q.y; v.d[2] = q.z; v.d[3] = q.w;
        return v;
    }
#pragma unroll
    for (int b = 0; b < 16; ++b)
        if (x + b >= 0 && x + b < W)
            v.d[b >> 2] |= (uint32_t)row[x + b] << (8 * (b & 3));
    return v;
}

__device__ __forceinline__ void store16(uint8_t *__restrict__ p, int y, int x, int W,
                                        bool aligned, const Px16 &v) {
    uint8_t *row = p + (size_t)y * W;
    if (aligned) {
        *reinterpret_cast<uint4 *>(row + x) = make_uint4(v.d[0], v.d[1], v.d[2], v.d[3]);
        return;
    }
#pragma unroll
    for (int b = 0; b < 16; ++b)
        if (x + b < W)
            row[x + b] = (uint8_t)(v.d[b >> 2] >> (8 * (b & 3)));
}

// bits 0, 8, 16, 24 of v -> bits 0..3 (the four products land on bits 21..24 without carries)
__device__ __forceinline__ uint32_t squeeze4(uint32_t v) { return ((v * 0x00204081u) >> 21) & 0xFu; }

__device__ __forceinline__ unsigned int wave_sum(unsigned int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += (unsigned int)__shfl_xor((int)v, o);
    return v;
}

__device__ __forceinline__ unsigned int wave_incl_scan(unsigned int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned int u = (unsigned int)__shfl_up((int)v, o);
        if (lane >= o)
            v += u;
    }
    return v;
}

template <int TYG>
__global__ __launch_bounds__(kThreads) void k_grow(const DevFrame *__restrict__ frames,
                                                   const TileRef *__restrict__ tiles,
                                                   DevFrame single, int kiter, int ntiles) {
    const int lane = threadIdx.x & 63;
    const int wt = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);   // wave tile index
    if (wt >= ntiles)
        return;
    DevFrame f;
    int y0, x0;
    if (tiles) {
        const TileRef t = tiles[wt];
        f = frames[t.frame];
        y0 = t.y0;
        x0 = t.x0;
    } else {
        f = single;
        const int ntx = (f.W + kGrowTX - 1) / kGrowTX;
        y0 = (wt / ntx) * TYG;
        x0 = (wt % ntx) * kGrowTX;
    }
    const int k = kiter ? kiter : f.k;
    if (frame_skips(f, k))
        return;
    const int H = f.H, W = f.W;
    const bool aligned = (W & 15) == 0;
    const bool fresh = k == 1 && (f.flags & kFreshMask);   // mask not yet initialised
    const int px = x0 - 16 + 16 * lane;                // first pixel of this lane's group
    const bool owner = lane >= 1 && lane <= kGrowTX / 16 && px < W;

    Px16 hA0 = {}, hA1 = {};          // dilated first selection, rows y-2, y-1
    Px16 hi1 = {};                    // [S' > sigclip] at row y-1
    Px16 lo1 = {}, lo2 = {};          // [S' > low] at rows y-1, y-2
    Px16 hG0 = {}, hG1 = {};          // dilated G1 at rows y-3, y-2
    uint32_t mbits[TYG / 2];          // mask bits of the strip, 16 per row
    unsigned int nnew = 0, nm = 0;
#pragma unroll
    for (int t = 0; t < TYG + 4; ++t) {
        const int y = y0 - 2 + t;
        const Px16 c = load16(f.codes, y, px, H, W, aligned);
        Px16 a, hi2, lo0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a.d[q] = c.d[q] & kByteLsb;
            hi2.d[q] = (c.d[q] >> 1) & kByteLsb;
            lo0.d[q] = (c.d[q] >> 2) & kByteLsb;
        }
        const Px16 hA2 = hdilate(a);
        Px16 g1;                                      // G1 at row y-1 (zero outside the image)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            g1.d[q] = (hA0.d[q] | hA1.d[q] | hA2.d[q]) & hi1.d[q];
        const Px16 hG2 = hdilate(g1);
        if (t >= 4) {
            const int r = t - 4;                     // output row y0 + r == y - 2
            Px16 g2;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                g2.d[q] = (hG0.d[q] | hG1.d[q] | hG2.d[q]) & lo2.d[q];
            uint32_t m16 = 0;
            if (owner && y - 2 < H) {
                const Px16 mp = fresh ? Px16{} : load16(f.mask, y - 2, px, H, W, aligned);
                Px16 m;
                uint32_t anynew = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t nw = g2.d[q] & ~mp.d[q];
                    m.d[q] = mp.d[q] | g2.d[q];
                    anynew |= nw;
                    nnew += (unsigned int)__popc(nw);
                    m16 |= squeeze4(m.d[q]) << (4 * q);
                }
                if (anynew || fresh)
                    store16(f.mask, y - 2, px, W, aligned, m);
                if (f.g2)
                    store16(f.g2, y - 2, px, W, aligned, g2);
                nm += (unsigned int)__popc(m16);
            }
            if (r & 1)
                mbits[r >> 1] |= m16 << 16;
            else
                mbits[r >> 1] = m16;
        }
        hA0 = hA1; hA1 = hA2;
        lo2 = lo1; lo1 = lo0;
        hi1 = hi2;
        hG0 = hG1; hG1 = hG2;
    }
    // one atomic per wave for the count and one for the list space
    const unsigned int tn = wave_sum(nnew);
    const unsigned int total = wave_sum(nm);
    unsigned int base = 0;
    if (lane == 0) {
        if (tn)
            atomicAdd(&f.nnew[k - 1], (unsigned long long)tn);
        if (total)
            base = atomicAdd(&f.listlen[k - 1], total);
    }
    base = (unsigned int)__shfl((int)base, 0);
    if (!total)
        return;
    // entries row by row across the wave, each lane's pixels in order
#pragma unroll
    for (int r = 0; r < TYG; ++r) {
        uint32_t m16 = (mbits[r >> 1] >> (16 * (r & 1))) & 0xFFFFu;
        if (__ballot(m16 != 0) == 0ull)
            continue;
        const unsigned int cnt = (unsigned int)__popc(m16);
        const unsigned int incl = wave_incl_scan(cnt, lane);
        unsigned int off = base + incl - cnt;
        while (m16) {
            const int b = __ffs(m16) - 1;
            f.list[off++] = (uint32_t)(y0 + r) * (uint32_t)W + (uint32_t)(px + b);
            m16 &= m16 - 1;
        }
        base += (unsigned int)__shfl((int)incl, 63);
    }
}

// ---------------------------------------------------------------------------
// replacement
// ---------------------------------------------------------------------------

// Unflagged pixels are never written and flagged ones are never read as values, so
// the update in place is race-free within the launch.
__device__ __forceinline__ void replace_one(const DevFrame &f, uint32_t p) {
    const int W = f.W, H = f.H;
    const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * (uint32_t)W);
    float v[25];
    int cnt = 0;
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy) {
        const size_t row = (size_t)clampi(y + dy, H) * W;
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            const size_t q = row + clampi(x + dx, W);
            const bool m = f.mask[q] != 0;
            v[(dy + 2) * 5 + dx + 2] = m ? INFINITY : f.J[q];
            cnt += m ? 0 : 1;
        }
    }
    if (cnt == 0)
        return;
    sort25(v);
    const int ia = (cnt - 1) >> 1, ib = cnt >> 1;
    float a = v[0], b = v[0];
#pragma unroll
    for (int j = 1; j < 25; ++j) {
        a = (j == ia) ? v[j] : a;
        b = (j == ib) ? v[j] : b;
    }
    f.J[p] = (ia == ib) ? a : (float)(((double)a + (double)b) * 0.5);
}

__global__ __launch_bounds__(kThreads) void k_list_prefix(const DevFrame *__restrict__ frames,
                                                          int nframes, int kiter,
                                                          unsigned int *__restrict__ prefix) {
    __shared__ unsigned int sPart[kThreads];
    __shared__ unsigned int sCarry;
    if (threadIdx.x == 0)
        sCarry = 0;
    __syncthreads();
    for (int base = 0; base < nframes; base += kThreads) {
        const int i = base + threadIdx.x;
        unsigned int len = 0;
        if (i < nframes) {
            const DevFrame &f = frames[i];
            const int k = kiter ? kiter : f.k;
            len = frame_skips(f, k) ? 0u : f.listlen[k - 1];
        }
        sPart[threadIdx.x] = len;
        __syncthreads();
        for (int o = 1; o < kThreads; o <<= 1) {      // inclusive scan
            const unsigned int v = threadIdx.x >= o ? sPart[threadIdx.x - o] : 0u;
            __syncthreads();
            sPart[threadIdx.x] += v;
            __syncthreads();
        }
        if (i < nframes)
            prefix[i] = sCarry + sPart[threadIdx.x] - len;
        __syncthreads();
        if (threadIdx.x == kThreads - 1)
            sCarry += sPart[kThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        prefix[nframes] = sCarry;
}

__global__ __launch_bounds__(kThreads) void k_replace(const DevFrame *__restrict__ frames,
                                                      int nframes,
                                                      const unsigned int *__restrict__ prefix,
                                                      DevFrame single, int kiter) {
    const unsigned int stride = gridDim.x * kThreads;
    unsigned int i = blockIdx.x * kThreads + threadIdx.x;
    if (!frames) {
        const int k = kiter ? kiter : single.k;
        if (frame_skips(single, k))
            return;
        const unsigned int n = single.listlen[k - 1];
        for (; i < n; i += stride)
            replace_one(single, single.list[i]);
        return;
    }
    const unsigned int total = prefix[nframes];
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD one
    // contiguous slice of the list (neighbouring pixels share cache lines in its L2).
    unsigned int end = total, step = stride;
    if ((gridDim.x & 7) == 0) {
        const unsigned int slice = (total + 7) >> 3;
        const unsigned int first = (blockIdx.x & 7) * slice;
        end = min(total, first + slice);
        i = first + (blockIdx.x >> 3) * kThreads + threadIdx.x;
        step = (gridDim.x >> 3) * kThreads;
    }
    for (; i < end; i += step) {
        int lo = 0, hi = nframes - 1;                  // last frame with prefix <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
        const DevFrame &f = frames[lo];
        replace_one(f, f.list[i - prefix[lo]]);
    }
}

// ---------------------------------------------------------------------------
// init and stats
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_init(const DevFrame *__restrict__ frames,
                                                   int nframes, DevFrame single) {
    const int nf = frames ? nframes : 1;
    const size_t gid = (size_t)blockIdx.x * kThreads + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (int fi = 0; fi < nf; ++fi) {
        const DevFrame f = frames ? frames[fi] : single;
        if (f.niter == 0) {
            const size_t n = (size_t)f.H * (size_t)f.W;
            for (size_t i = gid; i < n; i += stride) {
                if (f.img != f.J)
                    f.J[i] = f.img[i];
                f.mask[i] = 0;
            }
        }
        // counters restart at a frame's first iteration (f.k is 0 outside serving)
        if (f.nnew && f.k <= 1 && gid < (size_t)kMaxIter) {
            f.nnew[gid] = 0ull;
            f.listlen[gid] = 0u;
        }
    }
}

__global__ void k_stats(const DevFrame *__restrict__ frames, int nframes,
                        long long *__restrict__ stats) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nframes)
        return;
    const DevFrame f = frames[i];
    long long total = 0;
    int iters = 0;
    for (int k = 1; k <= f.niter; ++k) {
        iters = k;
        const unsigned long long n = f.nnew[k - 1];
        total += (long long)n;
        if (n == 0ull && !(f.flags & kNoEarlyStop))
            break;
    }
    stats[2 * i] = iters;
    stats[2 * i + 1] = total;
}

__global__ void k_round_stats(const DevFrame *__restrict__ frames, int nframes,
                              long long *__restrict__ stats) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nframes)
        return;
    const DevFrame f = frames[i];
    long long total = 0;
    for (int k = 1; k <= f.k; ++k)
        total += (long long)f.nnew[k - 1];
    stats[2 * i] = (long long)f.nnew[f.k - 1];
    stats[2 * i + 1] = total;
}

// ---------------------------------------------------------------------------
// subimage partition (the paper's 2-D split with a border, Section 6.2)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_extract(const float *__restrict__ img, int W,
                                                      const SubRect *__restrict__ subs) {
    const SubRect r = subs[blockIdx.y];
    const size_t n = (size_t)r.h * r.w;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kThreads) {
        const int y = (int)(i / r.w), x = (int)(i - (size_t)y * r.w);
        r.sub_img[i] = img[(size_t)(r.a0 + y) * W + r.b0 + x];
    }
}

__global__ __launch_bounds__(kThreads) void k_stitch(float *__restrict__ out_clean,
                                                     uint8_t *__restrict__ out_mask, int W,
                                                     const SubRect *__restrict__ subs) {
    const SubRect r = subs[blockIdx.y];
    const int ih = r.y1 - r.y0, iw = r.x1 - r.x0;
    const size_t n = (size_t)ih * iw;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kThreads) {
        const int y = r.y0 + (int)(i / iw), x = r.x0 + (int)(i % iw);
        const size_t q = (size_t)(y - r.a0) * r.w + (x - r.b0);
        out_clean[(size_t)y * W + x] = r.sub_clean[q];
        out_mask[(size_t)y * W + x] = r.sub_mask[q];
    }
}

// ---------------------------------------------------------------------------
// parity-test kernels: the median networks alone, binary64 sqrt and division
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

__global__ void k_debug_fp64(const double *__restrict__ x, const double *__restrict__ y, int n,
                             double *__restrict__ os, double *__restrict__ od) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        os[i] = sqrt(x[i]);
        od[i] = x[i] / y[i];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static unsigned int grid_for(size_t items, unsigned int cap) {
    size_t g = (items + kThreads - 1) / kThreads;
    if (g < 1)
        g = 1;
    return (unsigned int)(g < cap ? g : cap);
}

hipError_t launch_init(const DevFrame *d_frames, int nframes, const DevFrame &single,
                       size_t max_pixels, hipStream_t s) {
    const unsigned int grid = grid_for(max_pixels > (size_t)kMaxIter ? max_pixels : kMaxIter, 4096);
    k_init<<<grid, kThreads, 0, s>>>(d_frames, nframes, single);
    return hipGetLastError();
}

hipError_t launch_list_prefix(const DevFrame *d_frames, int nframes, int k,
                              unsigned int *d_prefix, hipStream_t s) {
    k_list_prefix<<<1, kThreads, 0, s>>>(d_frames, nframes, k, d_prefix);
    return hipGetLastError();
}

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

hipError_t launch_grow(const DevFrame *d_frames, const TileRef *d_tiles, int ntiles,
                       const DevFrame &single, int k, hipStream_t s) {
    constexpr int wpb = kThreads / 64;
    if (d_tiles) {
        if (ntiles <= 0)
            return hipSuccess;
        k_grow<kGrowTY><<<(ntiles + wpb - 1) / wpb, kThreads, 0, s>>>(d_frames, d_tiles, single,
                                                                       k, ntiles);
        return hipGetLastError();
    }
    // a single frame: short strips when the frame is small, so more waves share it
    const bool small = (size_t)single.H * single.W < ((size_t)1 << 22);
    const int ty = small ? kGrowTYSmall : kGrowTY;
    ntiles = ((single.W + kGrowTX - 1) / kGrowTX) * ((single.H + ty - 1) / ty);
    if (small)
        k_grow<kGrowTYSmall><<<(ntiles + wpb - 1) / wpb, kThreads, 0, s>>>(nullptr, nullptr,
                                                                            single, k, ntiles);
    else
        k_grow<kGrowTY><<<(ntiles + wpb - 1) / wpb, kThreads, 0, s>>>(nullptr, nullptr, single,
                                                                       k, ntiles);
    return hipGetLastError();
}

hipError_t launch_replace(const DevFrame *d_frames, int nframes, const unsigned int *d_prefix,
                          const DevFrame &single, int k, int grid, hipStream_t s) {
    k_replace<<<grid < 1 ? 1 : grid, kThreads, 0, s>>>(d_frames, nframes, d_prefix, single, k);
    return hipGetLastError();
}

hipError_t launch_stats(const DevFrame *d_frames, int nframes, long long *d_stats,
                        hipStream_t s) {
    k_stats<<<(nframes + 63) / 64, 64, 0, s>>>(d_frames, nframes, d_stats);
    return hipGetLastError();
}

hipError_t launch_round_stats(const DevFrame *d_frames, int nframes, long long *d_stats,
                              hipStream_t s) {
    k_round_stats<<<(nframes + 63) / 64, 64, 0, s>>>(d_frames, nframes, d_stats);
    return hipGetLastError();
}

hipError_t launch_extract(const float *img, int W, const SubRect *d_subs, int nsub,
                          size_t max_pixels, hipStream_t s) {
    dim3 grid(grid_for(max_pixels, 1024), nsub);
    k_extract<<<grid, kThreads, 0, s>>>(img, W, d_subs);
    return hipGetLastError();
}

hipError_t launch_stitch(float *out_clean, uint8_t *out_mask, int W, const SubRect *d_subs,
                         int nsub, size_t max_pixels, hipStream_t s) {
    dim3 grid(grid_for(max_pixels, 1024), nsub);
    k_stitch<<<grid, kThreads, 0, s>>>(out_clean, out_mask, W, d_subs);
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

hipError_t launch_debug_fp64(const double *x, const double *y, int n, double *out_sqrt,
                             double *out_div, hipStream_t s) {
    k_debug_fp64<<<(n + kThreads - 1) / kThreads, kThreads, 0, s>>>(x, y, n, out_sqrt, out_div);
    return hipGetLastError();
}

}  // namespace crb
