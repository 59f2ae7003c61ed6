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

// 3x3 medians of a run of 8 horizontally adjacent outputs from three rows of 10
// inputs.  Each column of three is sorted once (shared by up to three windows);
// the median of a 3x3 window with sorted columns is the median of
// (max of the column minima, median of the column medians, min of the column maxima).
__device__ __forceinline__ void med3_run8(const float (&a)[10], const float (&b)[10],
                                          const float (&c)[10], float (&o)[8]) {
    float lo[10], mi[10], hi[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        lo[j] = min3f(a[j], b[j], c[j]);
        mi[j] = med3f(a[j], b[j], c[j]);
        hi[j] = max3f(a[j], b[j], c[j]);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
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

template <int TY, int TX>
struct DetectLayout {
    static constexpr int JH = TY + 8, JW = TX + 8;              // J, apron 4
    static constexpr int MH = TY + 6, MW = TX + 6;              // med3(J), apron 3
    static constexpr int MWP = (MW + 3) & ~3;                   // 16-byte rows
    static constexpr int SH = TY + 4, SW = TX + 4;              // S (binary64), apron 2
};

template <int TY, int TX>
__global__ __launch_bounds__(kThreads) void k_detect(const DevFrame *__restrict__ frames,
                                                     const TileRef *__restrict__ tiles,
                                                     DevFrame single, int kiter) {
    using L = DetectLayout<TY, TX>;
    static_assert(TY % 2 == 0 && TX % 4 == 0, "detection tile must hold 2x4 thread tiles");
    __shared__ float sJ[L::JH * L::JW];
    __shared__ __align__(16) float sM3[L::MH * L::MWP];
    __shared__ __align__(16) double sS[L::SH * L::SW];
    __shared__ double sN[TY * TX];

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
    const float *__restrict__ J = f.J;

    // J over [y0-4, y0+TY+4) x [x0-4, x0+TX+4), clamped reads
    for (int i = tid; i < L::JH * L::JW; i += kThreads) {
        const int r = i / L::JW, c = i - r * L::JW;
        sJ[i] = J[(size_t)clampi(y0 - 4 + r, H) * W + clampi(x0 - 4 + c, W)];
    }
    __syncthreads();

    // med3(J) over [y0-3, y0+TY+3) x [x0-3, x0+TX+3): runs of 8 per thread
    {
        constexpr int NRX = (L::MW + 7) / 8;
        for (int t = tid; t < L::MH * NRX; t += kThreads) {
            const int r = t / NRX;
            const int cx = min((t - r * NRX) * 8, L::MW - 8);
            float a[10], b[10], c[10], o[8];
#pragma unroll
            for (int j = 0; j < 10; ++j) {
                a[j] = sJ[r * L::JW + cx + j];
                b[j] = sJ[(r + 1) * L::JW + cx + j];
                c[j] = sJ[(r + 2) * L::JW + cx + j];
            }
            med3_run8(a, b, c, o);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                sM3[r * L::MWP + cx + j] = o[j];
        }
    }

    // med5(J), L+, N and S over [y0-2, y0+TY+2) x [x0-2, x0+TX+2): 2x4 thread tiles
    {
        constexpr int NTY = (L::SH + 1) / 2, NTX = (L::SW + 3) / 4;
        constexpr int PW = 8;
        const double gain = f.gain, sky = f.sky, rn = f.readnoise;
        const double rn2 = rn * rn;
        for (int t = tid; t < NTY * NTX; t += kThreads) {
            const int ty = t / NTX;
            const int r = min(ty * 2, L::SH - 2);
            const int c = min((t - ty * NTX) * 4, L::SW - 4);
            float v[6 * PW], m5[8];
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = 0; j < PW; ++j)
                    v[i * PW + j] = sJ[(r + i) * L::JW + c + j];
            med5_t2x4(v, m5);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int pc = (i + 2) * PW + (j + 2);
                    const double lp = lplus(v[pc], v[pc - PW], v[pc + PW], v[pc - 1], v[pc + 1]);
                    double m = (double)m5[i * 4 + j] + sky;
                    if (m <= 0.0)
                        m = 1e-4;
                    const double N = sqrt(gain * m + rn2) / gain;
                    sS[(r + i) * L::SW + c + j] = lp / (2.0 * N);
                    const int cy = r + i - 2, cxx = c + j - 2;
                    if (cy >= 0 && cy < TY && cxx >= 0 && cxx < TX)
                        sN[cy * TX + cxx] = N;
                }
            }
        }
    }
    __syncthreads();

    // Region cells outside the image must hold the value of their clamped cell:
    // the nested filters read med3 and S at clamped neighbour positions.
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
                sS[i] = sS[(clampi(gy, H) - (y0 - 2)) * L::SW + (clampi(gx, W) - (x0 - 2))];
        }
        __syncthreads();
    }

    // med7(med3), med5(S), S', F^ and the threshold bits for the TY x TX outputs
    {
        constexpr int NTX = TX / 4;
        const double sigclip = f.sigclip, objlim = f.objlim;
        const double lowlim = (double)f.sigfrac * (double)f.sigclip;
        uint8_t *__restrict__ codes = f.codes;
        for (int t = tid; t < (TY / 2) * NTX; t += kThreads) {
            const int ty = t / NTX;
            const int r = ty * 2, c = (t - ty * NTX) * 4;
            float m7[8];
            {
                float v[8 * 10];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float4 q0 = *reinterpret_cast<const float4 *>(&sM3[(r + i) * L::MWP + c]);
                    const float4 q1 = *reinterpret_cast<const float4 *>(&sM3[(r + i) * L::MWP + c + 4]);
                    const float2 q2 = *reinterpret_cast<const float2 *>(&sM3[(r + i) * L::MWP + c + 8]);
                    v[i * 10 + 0] = q0.x; v[i * 10 + 1] = q0.y; v[i * 10 + 2] = q0.z; v[i * 10 + 3] = q0.w;
                    v[i * 10 + 4] = q1.x; v[i * 10 + 5] = q1.y; v[i * 10 + 6] = q1.z; v[i * 10 + 7] = q1.w;
                    v[i * 10 + 8] = q2.x; v[i * 10 + 9] = q2.y;
                }
                med7_t2x4(v, m7);
            }
            double ms[8];
            {
                double v[6 * 8];
#pragma unroll
                for (int i = 0; i < 6; ++i)
#pragma unroll
                    for (int j = 0; j < 8; j += 2) {
                        const double2 q = *reinterpret_cast<const double2 *>(&sS[(r + i) * L::SW + c + j]);
                        v[i * 8 + j] = q.x;
                        v[i * 8 + j + 1] = q.y;
                    }
                med5_t2x4(v, ms);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int gy = y0 + r + i;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int gx = x0 + c + j;
                    if (gy < H && gx < W) {
                        const double S = sS[(r + i + 2) * L::SW + c + j + 2];
                        const double N = sN[(r + i) * TX + c + j];
                        const double m3 = sM3[(r + i + 3) * L::MWP + c + j + 3];
                        const double sp = S - ms[i * 4 + j];
                        double fh = (m3 - (double)m7[i * 4 + j]) / N;
                        if (fh < 0.01)
                            fh = 0.01;
                        const bool hi = sp > sigclip;
                        const bool first = hi && (sp / fh > objlim);
                        const bool lo = sp > lowlim;
                        codes[(size_t)gy * W + gx] =
                            (uint8_t)((first ? 1 : 0) | (hi ? 2 : 0) | (lo ? 4 : 0));
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// grow + count + cumulative mask + flagged list
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_grow(const DevFrame *__restrict__ frames,
                                                   const TileRef *__restrict__ tiles,
                                                   DevFrame single, int kiter) {
    constexpr int CW = kGrowTX + 4, CH = kGrowTY + 4;   // codes, apron 2
    constexpr int GW = kGrowTX + 2, GH = kGrowTY + 2;   // G1, apron 1
    constexpr int NW = kThreads / 64;                   // waves
    constexpr int NP = kGrowTY / NW;                    // rows per wave
    __shared__ uint8_t sC[CH * CW];
    __shared__ uint8_t sG1[GH * GW];
    __shared__ unsigned int sCntNew[NW * NP], sCntM[NW * NP], sOff[NW * NP];
    __shared__ unsigned int sBase;

    DevFrame f;
    int y0, x0;
    if (tiles) {
        const TileRef t = tiles[blockIdx.x];
        f = frames[t.frame];
        y0 = t.y0;
        x0 = t.x0;
    } else {
        f = single;
        y0 = blockIdx.y * kGrowTY;
        x0 = blockIdx.x * kGrowTX;
    }
    const int k = kiter ? kiter : f.k;
    if (frame_skips(f, k))
        return;
    const int H = f.H, W = f.W, tid = threadIdx.x;

    for (int i = tid; i < CH * CW; i += kThreads) {
        const int r = i / CW, c = i - r * CW;
        const int gy = y0 - 2 + r, gx = x0 - 2 + c;
        sC[i] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? f.codes[(size_t)gy * W + gx] : 0;
    }
    __syncthreads();
    // G1 = dilate(first) and [S' > sigclip]; cells outside the image stay 0
    for (int i = tid; i < GH * GW; i += kThreads) {
        const int r = i / GW, c = i - r * GW;
        uint8_t any = 0;
#pragma unroll
        for (int dr = 0; dr < 3; ++dr)
#pragma unroll
            for (int dc = 0; dc < 3; ++dc)
                any |= sC[(r + dr) * CW + c + dc];
        sG1[i] = (uint8_t)((any & 1) & (sC[(r + 1) * CW + c + 1] >> 1));
    }
    __syncthreads();

    const int lane = tid & 63, w = tid >> 6;
    const int gx = x0 + lane;
    unsigned long long balM[NP];
    bool mine[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int row = w * NP + p;
        const int gy = y0 + row;
        const bool in = gy < H && gx < W;
        bool g2 = false, mprev = false;
        if (in) {
            uint8_t any = 0;
#pragma unroll
            for (int dr = 0; dr < 3; ++dr)
#pragma unroll
                for (int dc = 0; dc < 3; ++dc)
                    any |= sG1[(row + dr) * GW + lane + dc];
            g2 = any && ((sC[(row + 2) * CW + lane + 2] >> 2) & 1);
            const size_t q = (size_t)gy * W + gx;
            mprev = f.mask[q] != 0;
            if (g2 && !mprev)
                f.mask[q] = 1;
            if (f.g2)
                f.g2[q] = g2 ? 1 : 0;
        }
        const bool nw = g2 && !mprev;
        mine[p] = in && (g2 || mprev);
        const unsigned long long bn = __ballot(nw);
        balM[p] = __ballot(mine[p]);
        if (lane == 0) {
            sCntNew[w * NP + p] = (unsigned int)__popcll(bn);
            sCntM[w * NP + p] = (unsigned int)__popcll(balM[p]);
        }
    }
    __syncthreads();
    if (tid == 0) {
        unsigned int tn = 0, tm = 0;
        for (int i = 0; i < NW * NP; ++i) {
            tn += sCntNew[i];
            sOff[i] = tm;
            tm += sCntM[i];
        }
        if (tn)
            atomicAdd(&f.nnew[k - 1], (unsigned long long)tn);
        sBase = tm ? atomicAdd(&f.listlen[k - 1], tm) : 0u;
    }
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (mine[p]) {
            const int gy = y0 + w * NP + p;
            const unsigned int off = sBase + sOff[w * NP + p] + (unsigned int)__popcll(balM[p] & below);
            f.list[off] = (uint32_t)gy * (uint32_t)W + (uint32_t)gx;
        }
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

__global__ __launch_bounds__(kThreads) void k_replace(const DevFrame *__restrict__ frames,
                                                      int nframes, DevFrame single, int kiter) {
    const int nf = frames ? nframes : 1;
    for (int fi = 0; fi < nf; ++fi) {
        const DevFrame f = frames ? frames[fi] : single;
        const int k = kiter ? kiter : f.k;
        if (frame_skips(f, k))
            continue;
        const unsigned int n = f.listlen[k - 1];
        for (unsigned int i = blockIdx.x * kThreads + threadIdx.x; i < n;
             i += gridDim.x * kThreads)
            replace_one(f, f.list[i]);
    }
}

// ---------------------------------------------------------------------------
// init and stats
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_init(const DevFrame *__restrict__ frames,
                                                   int nframes, DevFrame single, int zero_mask) {
    const int nf = frames ? nframes : 1;
    const size_t gid = (size_t)blockIdx.x * kThreads + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (int fi = 0; fi < nf; ++fi) {
        const DevFrame f = frames ? frames[fi] : single;
        const size_t n = (size_t)f.H * (size_t)f.W;
        if (f.img != f.J)
            for (size_t i = gid; i < n; i += stride)
                f.J[i] = f.img[i];
        if (zero_mask)
            for (size_t i = gid; i < n; i += stride)
                f.mask[i] = 0;
        if (gid < (size_t)kMaxIter) {
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

// ---------------------------------------------------------------------------
// parity-test kernels: the median networks alone, binary64 sqrt and division
// ---------------------------------------------------------------------------

template <int R>
__global__ __launch_bounds__(kThreads) void k_debug_median(const float *__restrict__ in, int H,
                                                           int W, float *__restrict__ out) {
    constexpr int TY = (R == 1) ? 1 : 2, TX = (R == 1) ? 8 : 4;
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
        float a[10], b[10], c[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            a[j] = v[j];
            b[j] = v[PW + j];
            c[j] = v[2 * PW + j];
        }
        med3_run8(a, b, c, o);
    } else if constexpr (R == 2) {
        med5_t2x4(v, o);
    } else {
        med7_t2x4(v, o);
    }
#pragma unroll
    for (int i = 0; i < TY; ++i)
#pragma unroll
        for (int j = 0; j < TX; ++j)
            if (y0 + i < H && x0 + j < W)
                out[(size_t)(y0 + i) * W + x0 + j] = o[i * TX + j];
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
                       size_t max_pixels, bool zero_mask, hipStream_t s) {
    const unsigned int grid = grid_for(max_pixels > (size_t)kMaxIter ? max_pixels : kMaxIter, 4096);
    k_init<<<grid, kThreads, 0, s>>>(d_frames, nframes, single, zero_mask ? 1 : 0);
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
    if (d_tiles) {
        if (ntiles <= 0)
            return hipSuccess;
        k_grow<<<ntiles, kThreads, 0, s>>>(d_frames, d_tiles, single, k);
    } else {
        dim3 grid((single.W + kGrowTX - 1) / kGrowTX, (single.H + kGrowTY - 1) / kGrowTY);
        k_grow<<<grid, kThreads, 0, s>>>(nullptr, nullptr, single, k);
    }
    return hipGetLastError();
}

hipError_t launch_replace(const DevFrame *d_frames, int nframes, const DevFrame &single, int k,
                          int grid, hipStream_t s) {
    k_replace<<<grid < 1 ? 1 : grid, kThreads, 0, s>>>(d_frames, nframes, single, k);
    return hipGetLastError();
}

hipError_t launch_stats(const DevFrame *d_frames, int nframes, long long *d_stats,
                        hipStream_t s) {
    k_stats<<<(nframes + 63) / 64, 64, 0, s>>>(d_frames, nframes, d_stats);
    return hipGetLastError();
}

hipError_t launch_debug_median(const float *in, int H, int W, int r, float *out, hipStream_t s) {
    const int ty = (r == 1) ? 1 : 2, tx = (r == 1) ? 8 : 4;
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
