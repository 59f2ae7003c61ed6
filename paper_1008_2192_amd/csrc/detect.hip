// Detection kernel of libcrb for gfx950 (MI355X): the first stage of an L.A.Cosmic
// iteration (Mighell, Section 5) -- L+ (2x-subsampled clipped Laplacian, rebinned),
// N from med5(J), S = L+/(2N), S' = S - med5(S), F^ from med3(J) - med7(med3(J)),
// the first selection and the two threshold bits the grow reads -- on LDS tiles of 64
// columns by 16, 32 or 64 rows with the halo each quantity needs, one block per tile or
// persistent blocks taking tiles from ticket counters, plus the parity-test kernels of
// its median networks.
//
// Numerics: medians are exact selections by min/max networks.  Every decision (a
// threshold bit, the contrast test) is the one the binary64 definition takes: S is
// estimated in FP32 with a proven error bound, a decision is taken from the estimate
// only when the bound settles it, and otherwise from binary64 statistics evaluated in
// the definition's operation order (no contraction: built with -ffp-contract=off).
// So the codes for a given J are independent of the tiling and of the launch shape.
#include "kernels.h"
#include "device_common.h"

#include <math.h>

namespace crb {

#include "medtile.inc"

// Exclusive prefix sum over the lanes of a wave (all lanes active), from the device
// library's cross-lane (DPP) primitives.
extern "C" __device__ unsigned int __ockl_wfscan_add_u32(unsigned int, bool);

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

// Fourth word of a raw buffer resource on gfx9-family GPUs: 32-bit data format, no
// swizzle, range-checked against the byte count given with the base.
constexpr int kBufferWord3 = 0x00020000;

// FP32 parameters of the S estimate; ok is false for gains outside [2^-100, 2^100]
// (where g/8 could round), which leaves every decision to the binary64 evaluation.
struct SEstParams {
    float gain, g8, inv_gain, sky, rn2;
    bool ok;
};

__device__ __forceinline__ SEstParams sest_params(const DevFrame &f) {
    SEstParams p;
    p.gain = f.gain;
    p.g8 = f.g8;
    p.inv_gain = f.inv_gain;
    p.sky = f.sky;
    p.rn2 = f.rn2f;
    p.ok = f.est_ok != 0;
    return p;
}

// The sum l4 over the four sub-pixels of max(2c - v1 - v2, 0) (v1 in {up, dn}, v2 in
// {lf, rt}), which is 4 L+ at a pixel of value c with 4-neighbours up, dn, lf, rt.  The
// terms pair up by their vertical neighbour: with a = 2c - up, max(a - lf, 0) +
// max(a - rt, 0) = max(2a - (lf + rt), a - min(lf, rt), 0) (the first argument wins when
// a is above both horizontal neighbours, the second when it lies between them, 0 below
// both), and the same with b = 2c - dn.  Evaluated as written (two FMAs for a and b,
// lf + rt, the minimum, per pair one FMA, one subtraction and a max3, one final
// addition; 11 operations where the term-by-term sum takes 13), with u = 2^-24 and round
// to nearest: each pair is within 2u M_a of its exact value, M_a = 4|c| + 2|up| + |lf| +
// |rt| (likewise M_b), and the sum within 3u (M_a + M_b) = 6u M of 4 L+, M = 4|c| + |up|
// + |dn| + |lf| + |rt|.
__device__ __forceinline__ float lplus4(float c, float up, float dn, float lf, float rt) {
    const float a = fmaf(2.0f, c, -up), b = fmaf(2.0f, c, -dn);
    const float s = lf + rt, m = fminf(lf, rt);
    return max3f(fmaf(2.0f, a, -s), a - m, 0.0f) + max3f(fmaf(2.0f, b, -s), b - m, 0.0f);
}

// FP32 estimate s of S at a pixel of value c with 4-neighbours up, dn, lf, rt and
// med5(J) = m5, and a bound err >= |s - S|, S being the binary64 value of the
// definition (S = L+ / (2N), L+ = a quarter of the sum over the four sub-pixels of
// max(2c - v1 - v2, 0), N = sqrt(g m + rn^2) / g).  Error analysis, u = 2^-24,
// round to nearest with FP32 denormals preserved, M = 4|c| + |up| + |dn| + |lf| + |rt|:
//   the sub-pixel sum l4 (lplus4) is 4 L+ within 6.01 u M;
//   t = g m + rn^2 (positive terms, m itself rounded once) carries at most 3.03 u
//     relative error, so t^-1/2 at most 1.52 u; the reciprocal square root (v_rsq_f32,
//     within 1 ulp = 2u), the scaling by g/8 (exact) and the two products add 2u + 2u;
//   the binary64 evaluation is within 2^-49 (M R + S) of the exact value;
// so |s - S| <= 6.01 u M R + 5.52 u s with R = g/(8 sqrt t), which err = 2^-19 (M R + s)
// overstates at least four-fold (the s-term tolerates a reciprocal square root 14 ulp
// off).  Outside t in [2^-100, 2^100] and M <= 2^100 (where the
// analysis has no overflow, underflow or domain edge) s = err = +inf, which sends every
// decision that reads the pixel to the binary64 evaluation.
__device__ __forceinline__ float s_estimate(float c, float up, float dn, float lf, float rt,
                                            float m5, const SEstParams &p, float &err) {
    const float l4 = lplus4(c, up, dn, lf, rt);
    float m = m5 + p.sky;
    m = (m <= 0.0f) ? 1e-4f : m;
    const float t = fmaf(p.gain, m, p.rn2);
    const float R = p.g8 * __builtin_amdgcn_rsqf(t);
    const float s = l4 * R;
    const float M = fmaf(4.0f, fabsf(c), fabsf(up)) + fabsf(dn) + (fabsf(lf) + fabsf(rt));
    const bool sane = __builtin_amdgcn_fmed3f(t, 0x1p-100f, 0x1p100f) == t && M <= 0x1p100f && p.ok;
    err = sane ? (M * R + s) * 0x1p-19f : INFINITY;
    return sane ? s : INFINITY;
}

// The factor R = (g/8) t^-1/2 of the S estimate, t = g m + rn^2, for a lower bound x of
// med5(J): m = x + sky, or 0 where that is at most 1e-4 (N of the definition never falls
// below rn/g, while above the definition's floor it grows with med5(J)), so the estimate
// from R, with its error bound, bounds S from above for every med5(J) >= x.  INFINITY
// where the error analysis of the estimate does not hold.
__device__ __forceinline__ float r_bound(float x, const SEstParams &p) {
    float m = x + p.sky;
    m = (m <= 1e-4f) ? 0.0f : m;
    const float t = fmaf(p.gain, m, p.rn2);
    const bool sane = __builtin_amdgcn_fmed3f(t, 0x1p-100f, 0x1p100f) == t && p.ok;
    return sane ? p.g8 * __builtin_amdgcn_rsqf(t) : INFINITY;
}

// An upper bound of S at a pixel of value c with 4-neighbours up, dn, lf, rt, given
// Rp = R (1 + 2^-19) rounded, R = r_bound(x) finite for a lower bound x of its med5(J),
// and E = 2^-19 * 8 v * R with v >= each |value| read and 8 v <= 2^100.  With l4 =
// lplus4 (within 6u M of 4 L+) and R's own error (at most 5u relative, as in
// s_estimate), S <= (l4 + 6u M) R (1 + 5u), while fl(l4 Rp + E) >= l4 R (1 + 2^-19 -
// 2.1u) + E (1 - u) and E >= 32u M R (1 - u): the returned value exceeds S, so where it
// is at most sigclip (less 2^-20), S <= sigclip.
__device__ __forceinline__ float s_upper(float c, float up, float dn, float lf, float rt,
                                         float Rp, float E) {
    return fmaf(lplus4(c, up, dn, lf, rt), Rp, E);
}

// The dense bound of a 2 x 5 cell tile from its 6 x 9 patch of J (patch row i, column j
// is cell row i - 2, column j - 2; clamped where the patch leaves the frame): u[5 i + j]
// >= S at cell (i, j) for every cell of the tile, unless the function returns false (R
// not finite or a value above 2^96 in magnitude: the analysis of the bound does not
// hold, and every cell must count as a candidate).
//   x: a lower bound of med5(J) shared by the tile's ten windows, the least value of
//   patch rows 1-4 (every window holds those four rows of its five columns, so 20 of its
//   25 values are >= x; 18 three-input minima).  S does not increase with med5(J), so
//   the estimate at x with its error bound bounds S from above.  (The least over the
//   columns of each column's second smallest in rows 1-4 is a tighter bound, with 15
//   values >= it, but costs 63 operations; with the least value H' grows by about 3%
//   and the region of exact med5(J) by about 7%.)
//   E: one error term for the ten cells: every value their M reads lies in patch rows
//   1-4, columns 1-7, so M <= 8 vmax.
__device__ __forceinline__ bool dense_bounds(const float (&v)[6 * 9], const SEstParams &sp,
                                             float (&u)[10]) {
    constexpr int PW = 9, NV = 4 * PW;
    float x = v[PW];
#pragma unroll
    for (int k = 1; k + 1 < NV; k += 2)
        x = min3f(x, v[PW + k], v[PW + k + 1]);
    if (NV % 2 == 0)
        x = fminf(x, v[PW + NV - 1]);
    const float R = r_bound(x, sp);
    float vmax = 0.0f;
#pragma unroll
    for (int i = 1; i <= 4; ++i)
#pragma unroll
        for (int j = 1; j <= 7; ++j)
            vmax = fmaxf(vmax, fabsf(v[i * PW + j]));
    const float E = (8.0f * vmax) * R * 0x1p-19f;
    const float Rp = fmaf(R, 0x1p-19f, R);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int pc = (i + 2) * PW + (j + 2);
            u[i * 5 + j] = s_upper(v[pc], v[pc - PW], v[pc + PW], v[pc - 1], v[pc + 1], Rp, E);
        }
    return R < INFINITY && vmax <= 0x1p96f;
}

// S exactly as the definition evaluates it (binary64, in its operation order), at the
// in-frame pixel (y, x) of J (clamped neighbours), read from global memory.
__device__ __forceinline__ double s_exact(const float *__restrict__ J, int H, int W, int y, int x,
                                          double gain, double sky, double rn2) {
    float w[25], m5[1];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j)
            w[i * 5 + j] = J[(size_t)clampi(y + i - 2, H) * W + clampi(x + j - 2, W)];
    med5_t1x1(w, m5);
    const double lp = lplus(w[12], w[7], w[17], w[11], w[13]);
    double m = (double)m5[0] + sky;
    if (m <= 0.0)
        m = 1e-4;
    const double N = sqrt(gain * m + rn2) / gain;
    return lp / (2.0 * N);
}

// N of the definition (binary64) from med5(J).
__device__ __forceinline__ double noise_exact(float m5, double gain, double sky, double rn2) {
    double m = (double)m5 + sky;
    if (m <= 0.0)
        m = 1e-4;
    return sqrt(gain * m + rn2) / gain;
}

// med3(J) at the pixel whose staged J cell is p (pitch jp).  The staged plane holds
// J at clamped positions, so for an in-frame pixel this is the clamped 3 x 3 window:
// with each column sorted, the median of nine is the median of the largest column
// minimum, the median of the column medians and the smallest column maximum.
__device__ __forceinline__ float med3_at(const float *p, int jp) {
    float lo[3], mi[3], hi[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float a = p[-jp + j - 1], b = p[j - 1], c = p[jp + j - 1];
        lo[j] = min3f(a, b, c);
        mi[j] = med3f(a, b, c);
        hi[j] = max3f(a, b, c);
    }
    return med3f(max3f(lo[0], lo[1], lo[2]), med3f(mi[0], mi[1], mi[2]),
                 min3f(hi[0], hi[1], hi[2]));
}

// Staged J cell (pitch jp, apron 4 around the tile at (y0, x0)) of the in-frame pixel
// nearest to tile position (r + dy, c + dx): where med3(J) is read for the 7 x 7 window
// of a tile pixel (the window is clamped to the frame).
__device__ __forceinline__ const float *med3_cell(const float *sJ, int jp, int y0, int x0,
                                                  int H, int W, int r, int c, int dy, int dx) {
    return &sJ[(clampi(y0 + r + dy, H) - y0 + 4) * jp + (clampi(x0 + c + dx, W) - x0 + 4)];
}

// The contrast test S'/F^ > objlim in binary64 at tile pixel (r, c), med3 taken from the
// staged J, F^ = max((med3 - med7(med3)) / N, 0.01).  The test, evaluated in the
// definition's operations with a value x in place of med7, is monotone in x (every step
// and every rounding is), and med7 is the 25th of the 49 window values, with 24 on
// either side; so the test holds at med7 iff it holds at 25 or more of them.
__device__ __forceinline__ bool contrast_exact(const float *sJ, int jp, int y0, int x0, int H,
                                               int W, int r, int c, double spr, double N,
                                               double objlim) {
    const double m3 = (double)med3_at(med3_cell(sJ, jp, y0, x0, H, W, r, c, 0, 0), jp);
    int n = 0;
#pragma unroll 1
    for (int i = 0; i < 7; ++i) {
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const double x = (double)med3_at(med3_cell(sJ, jp, y0, x0, H, W, r, c, i - 3, j - 3), jp);
            double fh = (m3 - x) / N;
            fh = fh < 0.01 ? 0.01 : fh;
            n += spr / fh > objlim ? 1 : 0;
        }
    }
    return n >= 25;
}

// N at a pixel from its FP32 estimate s = l4 R of S (s_estimate; R = (g/8) rsq(t), and l4
// the pixel's L+ sum formed as the estimate formed it): N = 1 / (8 R) = l4 / (8 s).  R is
// within 4.52u of g / (8 sqrt(t)) for the definition's t (t to 3.03u, so its -1/2 power
// to 1.52u; the reciprocal square root to 1 ulp = 2u; the product by g/8 to u), s adds
// u and the division u: N is within 6.52u of the definition's (u = 2^-24), for any
// s > 0 with a finite error bound.
__device__ __forceinline__ float noise_from_estimate(float l4, float s) {
    return l4 / (8.0f * s);
}

// The switching values of the contrast test below, from med3 (m3) and N at the pixel:
// a window value x > t_sure makes the test hold for every S' >= lo, one with x >= t_maybe
// lets it hold for some S' <= hi.
__device__ __forceinline__ void contrast_thresholds(float m3, float N, float lo, float hi,
                                                    float inv_olim, float &t_sure,
                                                    float &t_maybe) {
    const float klo = N * lo * inv_olim, khi = N * hi * inv_olim;
    t_sure = (m3 - klo) + fmaf(0x1p-19f, fabsf(m3) + klo, 0x1p-126f);
    t_maybe = (m3 - khi) - fmaf(0x1p-19f, fabsf(m3) + khi, 0x1p-126f);
}

// The contrast test S'/F^ > objlim at tile pixel (r, c), for every S' in [lo, hi]
// (0 < lo), without selecting med7, by the calling wave (all lanes active, arguments
// uniform): 1 if it holds for all of them, 0 if it fails for all, -1 if undecided.
//   F^ does not increase with med7 (m3 - med7, the division by N > 0, the floor at 0.01
//   and their roundings are monotone), so at fixed S' the test, as a function of the
//   value x taken by med7, holds above a switching value and nowhere below it; med7 is
//   the 25th smallest of the 49 window values, so the test holds at med7 iff it holds
//   at 25 or more of them.
//   If fl(S'/0.01) <= objlim the test fails whatever x (F^ >= 0.01); 100 S' in FP32 is
//   within 1.01u of that binary64 quotient (u = 2^-24), so comparing it with objlim
//   widened or narrowed by 2^-21 relative decides this for the whole interval (the
//   caller does, before listing the pixel).
//   Otherwise the test holds at x iff m3 - x < K (1 + e), K = N S'/objlim, |e| <=
//   4 * 2^-53.  K from N in FP32 (within 8u: noise_from_estimate gives 6.52u) and two
//   more products is within 11u, so x above T = m3 - K up to a band of 2^-19 (|m3| + K)
//   + 2^-126 (three-fold the roundings) decides the test.  The test is larger for larger
//   S', so lo bounds its certain holding and hi its possible holding.
// N is the noise at the pixel (noise_from_estimate); lane l < 49 takes the med3 value of
// window cell (l / 7 - 3, l % 7 - 3), and ballots count them.
__device__ __forceinline__ int contrast_by_count(const float *sJ, int jp, int y0, int x0,
                                                 int H, int W, int r, int c, float N, float lo,
                                                 float hi, float inv_olim, int lane) {
    const int l49 = lane < 49 ? lane : 24;
    const float x = med3_at(med3_cell(sJ, jp, y0, x0, H, W, r, c, l49 / 7 - 3, l49 % 7 - 3), jp);
    const float m3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 24));
    float t_sure, t_maybe;
    contrast_thresholds(m3, N, lo, hi, inv_olim, t_sure, t_maybe);
    const int sure = __popcll(__ballot(lane < 49 && x > t_sure));
    const int maybe = __popcll(__ballot(lane < 49 && x >= t_maybe));
    return sure >= 25 ? 1 : (maybe < 25 ? 0 : -1);
}

// The same test by one thread (for pixels beyond the contrast list): the 49 med3 values
// one after another.
__device__ __forceinline__ int contrast_by_count_lane(const float *sJ, int jp, int y0, int x0,
                                                      int H, int W, int r, int c, float N,
                                                      float lo, float hi, float inv_olim) {
    const float m3 = med3_at(med3_cell(sJ, jp, y0, x0, H, W, r, c, 0, 0), jp);
    float t_sure, t_maybe;
    contrast_thresholds(m3, N, lo, hi, inv_olim, t_sure, t_maybe);
    int sure = 0, maybe = 0;
#pragma unroll 1
    for (int i = 0; i < 7; ++i) {
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const float x = med3_at(med3_cell(sJ, jp, y0, x0, H, W, r, c, i - 3, j - 3), jp);
            sure += x > t_sure ? 1 : 0;
            maybe += x >= t_maybe ? 1 : 0;
        }
    }
    return sure >= 25 ? 1 : (maybe < 25 ? 0 : -1);
}

// Exclusive prefix sums of the set-bit counts of the NWORDS words of a bitmap into
// pre[0 .. NWORDS-1], the total into pre[NWORDS]; by the first wave (all 64 lanes), each
// lane taking NWORDS / 64 consecutive words (or one, or none past NWORDS, when NWORDS is
// at most 64).
template <int NWORDS>
__device__ __forceinline__ void bitmap_prefix(const uint32_t *bits, uint32_t *pre) {
    static_assert(NWORDS <= 64 || NWORDS % 64 == 0, "whole words per lane");
    constexpr int WPL = NWORDS > 64 ? NWORDS / 64 : 1;
    const int lane = threadIdx.x & 63;
    unsigned int c[WPL], tot = 0u;
#pragma unroll
    for (int i = 0; i < WPL; ++i) {
        const int w = lane * WPL + i;
        c[i] = w < NWORDS ? (unsigned int)__popc(bits[w]) : 0u;
        tot += c[i];
    }
    unsigned int ex = __ockl_wfscan_add_u32(tot, false);
#pragma unroll
    for (int i = 0; i < WPL; ++i) {
        const int w = lane * WPL + i;
        if (w < NWORDS)
            pre[w] = ex;
        ex += c[i];
    }
    if (lane == 63)
        pre[NWORDS] = ex;
}

// Position (word * 32 + bit) of the q-th set bit of an NWORDS-word bitmap with prefix pre.
template <int NWORDS>
__device__ __forceinline__ int bitmap_select(const uint32_t *bits, const uint32_t *pre, int q) {
    int lo = 0, hi = NWORDS - 1;    // last word whose prefix is <= q
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int)pre[mid] <= q)
            lo = mid;
        else
            hi = mid - 1;
    }
    uint32_t b = bits[lo];
    for (int n = q - (int)pre[lo]; n > 0; --n)
        b &= b - 1u;
    return lo * 32 + __ffs(b) - 1;
}

// Appends pos0 + b for every set bit b of m (one word per lane; called by whole waves) to
// an LDS list: places within the wave by a DPP prefix sum, the wave's base by one LDS
// atomic on *count, so that several waves append in any order.  Entries at or beyond cap
// are not stored; *count ends as the number of bits appended by all waves.
__device__ __forceinline__ void list_append(uint32_t m, int pos0, uint16_t *list,
                                            unsigned int *count, unsigned int cap, int lane) {
    const unsigned int cnt = (unsigned int)__popc(m);
    unsigned int at = __ockl_wfscan_add_u32(cnt, false);
    const unsigned int total = (unsigned int)__builtin_amdgcn_readlane((int)(at + cnt), 63);
    unsigned int base = 0u;
    if (lane == 0 && total)
        base = atomicAdd(count, total);
    at += (unsigned int)__builtin_amdgcn_readfirstlane((int)base);
    for (uint32_t mm = m; mm; mm &= mm - 1u, ++at)
        if (at < cap)
            list[at] = (uint16_t)(pos0 + __ffs(mm) - 1);
}

// Work shapes inside a detection block: a lower bound of med5(J), L+ and an upper bound
// of S in 2 x 5 thread tiles over the whole tile and its 2-pixel apron; med5(J) and the S
// estimate in 2 x 2 quads near where S may exceed sigclip.  The remaining statistics,
// med3 among them, are evaluated only where a code bit can matter.
// Run length of the 3x3 median network's parity kernel (sorted columns shared by runs).
constexpr int kRun3 = 14;

// A detection tile is TY rows of 64 columns, one block of 8 * TY threads: each thread
// writes 8 codes of one row, so wave w holds rows 8w .. 8w+7.  TY in {16, 32, 64} (the
// tile shapes the autotuner picks from; 32 is the default).
template <int TY>
struct DetectLayout {
    static constexpr int TX = 64, NT = 8 * TY, NW = NT / 64;
    // logical extents of the LDS planes and their row pitches; the pitches spread the
    // stage-1 and stage-2 scalar accesses over the LDS banks
    static constexpr int JH = TY + 8, JW = TX + 8, JWP = TX + 9;    // J, apron 4
    static constexpr int SH = TY + 4, SW = TX + 4, SWP = TX + 6;    // S estimate, apron 2
    static constexpr int HW = (SW + 31) / 32;   // words per row of the hot bitmap
    // the hot bitmap is stored with 4 zero rows above and below and a zero word before
    // each row (which is also the word after the previous row; one more zero word ends
    // the array), so that its dilations read it without bounds tests
    static constexpr int HWP = HW + 1, HR = SH + 8;
    static constexpr int QW = TX / 32;          // words per row of the tile bitmaps
    static constexpr int kTileWords = TY * QW;
    // pixels per round of the binary64 re-evaluation (25 threads each)
    static constexpr int kExactBatch = NT / 25;
    // pixels whose contrast test a block lists for its contrast phase (one wave each);
    // further ones take the same test in their own lanes
    static constexpr int kConMax = TY;
    // work-set pixels a block lists; a larger work set is taken from its bitmap instead
    static constexpr int kListMax = 8 * TY;
    // LDS budget for the resident blocks per CU (the CU hands out LDS in 1 KiB units):
    // 12 blocks of 16 rows, 6 of 32 rows, 3 of 64 rows (about 24 waves per CU)
    static constexpr int kLdsBudget = TY == 16 ? 15360 : (TY == 32 ? 26624 : 53248);
    static_assert(TY == 16 || TY == 32 || TY == 64, "tile heights 16, 32, 64");
    static_assert(NW * 64 == NT && QW == 2, "whole waves; two bitmap words per tile row");
    static_assert(QW + 1 <= HW, "dilation reads two bitmap words per work word");
    static_assert(SH * SWP * 4 >= kExactBatch * 26 * 8, "re-evaluation buffer in the S plane");
};

// The detection of one tile (origin y0, x0 of frame f, iteration k), by the whole block.
// Every early return is taken by all threads alike.
//
// Which pixels need S', F^ and the threshold bits.  With H = {S > sigclip} (S' > t
// implies S > t for t >= 0: med5(S) >= 0 because S >= 0, and rounding is monotone):
//   first(p) can be 1 only on H;
//   G1(p) needs an A pixel within distance 1, so hi(p) matters only on D1(H);
//   G2(p) needs a G1 pixel within distance 1, so lo(p) matters only on D2(H);
// and lo(p) = hi(p) = 0 wherever S(p) <= sigfrac * sigclip (sigfrac <= 1).  The block
// bounds S from above on the tile and its apron (from a lower bound of med5(J)), then
// computes the FP32 estimate s of S with its error bound err within 4 of where that
// bound exceeds sigclip, takes H' = {s + err > sigclip (less a margin)} (a superset of
// H), and evaluates the codes on Q' = D2(H') & {s + err > sigfrac * sigclip (less a
// margin)}, a superset of Q = D2(H) & {S > sigfrac*sigclip}: med5 of the estimates
// gives S' within twice the block's largest error (the median moves no more than its
// inputs), which decides the two bits, and F^ with the interval of S' decides the
// contrast test; a pixel where an interval straddles a threshold is re-evaluated in
// binary64 from J.  So every code written is the full definition's, codes outside Q'
// are 0, and the grow, which reads codes only through its two dilations, sees the full
// definition.
template <int TY>
__device__ __forceinline__ void detect_tile(const DevFrame &f, int y0, int x0, int k, int tid) {
    using L = DetectLayout<TY>;
    constexpr int TX = L::TX, NT = L::NT;
    constexpr int kConMax = L::kConMax, kListMax = L::kListMax, kExactBatch = L::kExactBatch;
    __shared__ __align__(16) float sJ[L::JH * L::JWP];       // J, clamped extension
    __shared__ __align__(16) float sS[L::SH * L::SWP];      // later: re-evaluation buffer
    __shared__ __align__(16) uint8_t sCode[TY * TX];
    __shared__ uint32_t sHotP[L::HR * L::HWP + 1];          // H', apron 2, in-frame
    // word w of region row r of H' (r in [-4, SH + 4), w in [-1, HW]; zero outside)
    uint32_t *const sHot = &sHotP[4 * L::HWP + 1];
    __shared__ uint32_t sU[L::kTileWords], sUpre[L::kTileWords + 1];
    // tile cells where S may exceed sigfrac*sigclip; after the work-set build, Q' itself
    __shared__ uint32_t sLow[L::kTileWords];
    __shared__ unsigned int sErrBits, sContrast, sUncertain, sQcount, sNeedCount, sExactCells,
        sConCount;
    double *const sX = reinterpret_cast<double *>(sS);
    __shared__ uint16_t sList[kListMax];                    // work set Q' (up to kListMax)
    // pixels whose contrast test is left to the contrast phase: position, S' interval, N
    __shared__ uint32_t sConInfo[kConMax];
    __shared__ float sConLo[kConMax], sConHi[kConMax], sConN[kConMax];
    static_assert(sizeof(sJ) + sizeof(sS) + sizeof(sCode) + sizeof(sHotP) + sizeof(sU) +
                          sizeof(sUpre) + sizeof(sLow) + sizeof(sList) + sizeof(sConInfo) +
                          sizeof(sConLo) + sizeof(sConHi) + sizeof(sConN) + 7 * 4 + 16 <=
                      L::kLdsBudget,
                  "the LDS of a detection block must let its resident blocks share a CU");

    if (frame_skips(f, k))
        return;
    const int H = f.H, W = f.W;
    const int lane = tid & 63;
    // incremental mode: from iteration 2 on, a tile is re-evaluated only when the
    // previous replacement changed J within 4 pixels of it, which it records by stamping
    // the 32 x 64 summary tiles it reached with its iteration (every thread reads the
    // same stamps, so the return is uniform)
    if ((f.flags & kIncremental) && f.dirty && k >= 2) {
        // a tile of at most 64 rows meets one or two rows of summary tiles
        static_assert(TY <= 2 * kSumTY, "at most two summary rows per tile");
        const int ntx = (W + kSumTX - 1) / kSumTX, c = x0 / kSumTX;
        const int r0 = y0 / kSumTY, r1 = (min(y0 + TY, H) - 1) / kSumTY;
        const uint8_t want = (uint8_t)(k - 1);
        if (f.dirty[r0 * ntx + c] != want && f.dirty[r1 * ntx + c] != want)
            return;
    }
    // iteration 1 reads the input frame and initialises J with the tile's own pixels
    const float *__restrict__ J = (k == 1) ? f.img : f.J;
    // thresholds widened by 2^-20 relative: fl(x) beyond them decides the real x
    // against the binary64 thresholds sigclip and sigfrac * sigclip (exact products)
    const float sc_lo = f.sc_lo, sc_hi = f.sc_hi, ll_lo = f.ll_lo, ll_hi = f.ll_hi;

    for (int i = tid; i < L::HR * L::HWP + 1; i += NT)
        sHotP[i] = 0u;
    for (int i = tid; i < L::kTileWords; i += NT) {
        sU[i] = 0u;
        sLow[i] = 0u;
    }
    if (tid == 0) {
        sErrBits = 0u;
        sQcount = 0u;
        sContrast = 0u;
        sUncertain = 0u;
        sNeedCount = 0u;
        sExactCells = 0u;
        sConCount = 0u;
    }
    // J over [y0-4, y0+TY+4) x [x0-4, x0+TX+4), clamped reads.  Thread t loads column
    // t % JW of rows t / JW + kJStep * b, so its clamped column is computed once and, on
    // tiles whose rows are all inside the frame, each further row costs one address
    // step.  A thread's loads (all of them, or half when there are more than 16) are
    // issued before its first LDS store, so their latencies overlap.
    {
        constexpr int kJStep = NT / L::JW;
        constexpr int NB = (L::JH + kJStep - 1) / kJStep;
        constexpr int NC = NB > 16 ? (NB + 1) / 2 : NB;      // loads in flight per round
        const int c = tid % L::JW, r0 = tid / L::JW;
        if (r0 < kJStep) {
            const int cc = clampi(x0 - 4 + c, W);
            if (y0 >= 4 && y0 + TY + 4 <= H && (long long)L::JH * W * 4 <= 0x7fffffffll) {
                // buffer loads over the JH staged rows (below 2^31 bytes, so the byte
                // count, the lane offsets and the row steps below are exact in int): a
                // per-lane byte offset and a uniform row step, so a further row costs no
                // vector instruction
                const __amdgpu_buffer_rsrc_t rows = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(J + (size_t)(y0 - 4) * W), (short)0, L::JH * W * 4, kBufferWord3);
                const int boff = (r0 * W + cc) * 4;
#pragma unroll
                for (int b0 = 0; b0 < NB; b0 += NC) {
                    float v[NC];
#pragma unroll
                    for (int b = 0; b < NC; ++b)
                        if (b0 + b < NB && r0 + kJStep * (b0 + b) < L::JH)
                            v[b] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                                rows, boff, kJStep * (b0 + b) * W * 4, 0));
#pragma unroll
                    for (int b = 0; b < NC; ++b)
                        if (b0 + b < NB && r0 + kJStep * (b0 + b) < L::JH)
                            sJ[(r0 + kJStep * (b0 + b)) * L::JWP + c] = v[b];
                }
            } else {
#pragma unroll
                for (int b0 = 0; b0 < NB; b0 += NC) {
                    float v[NC];
#pragma unroll
                    for (int b = 0; b < NC; ++b)
                        if (b0 + b < NB && r0 + kJStep * (b0 + b) < L::JH)
                            v[b] = J[(size_t)clampi(y0 - 4 + r0 + kJStep * (b0 + b), H) * W + cc];
#pragma unroll
                    for (int b = 0; b < NC; ++b)
                        if (b0 + b < NB && r0 + kJStep * (b0 + b) < L::JH)
                            sJ[(r0 + kJStep * (b0 + b)) * L::JWP + c] = v[b];
                }
            }
        }
    }
    __syncthreads();
    // iteration 1: the tile's own pixels of the input become J, 8 per thread
    static_assert(TY * TX == 8 * NT, "one 8-pixel row segment per thread");
    if (k == 1 && f.img != f.J) {
        const int r = tid / (TX / 8), cs = (tid - r * (TX / 8)) * 8;
        const int gy = y0 + r, gx = x0 + cs;
        if (gy < H && gx < W) {
            const float *src = &sJ[(r + 4) * L::JWP + cs + 4];
            float *dst = f.J + (size_t)gy * W + gx;
            if (gx + 8 <= W && ((uintptr_t)dst & 15u) == 0u) {
                reinterpret_cast<float4 *>(dst)[0] = make_float4(src[0], src[1], src[2], src[3]);
                reinterpret_cast<float4 *>(dst)[1] = make_float4(src[4], src[5], src[6], src[7]);
            } else {
                const int nb = min(8, W - gx);
                for (int j = 0; j < nb; ++j)
                    dst[j] = src[j];
            }
        }
    }
    // iteration 1 on an uninitialised mask: the tile's mask bytes are cleared here, so
    // the grow writes only the rows that gain a flag
    if (k == 1 && (f.flags & kFreshMask) && f.mask) {
        const int r = tid / (TX / 8), cs = (tid - r * (TX / 8)) * 8;
        const int gy = y0 + r, gx = x0 + cs;
        if (gy < H && gx < W) {
            uint8_t *dst = f.mask + (size_t)gy * W + gx;
            if (gx + 8 <= W && ((uintptr_t)dst & 7u) == 0u) {
                *reinterpret_cast<uint2 *>(dst) = make_uint2(0u, 0u);
            } else {
                const int nb = min(8, W - gx);
                for (int j = 0; j < nb; ++j)
                    dst[j] = 0;
            }
        }
    }

    // Over [y0-2, y0+TY+2) x [x0-2, x0+TX+2), in 2 x 5 cell tiles (one per thread and
    // pass).  Dense pass: the upper bound of S from a lower bound of med5(J) shared by the
    // tile's ten windows (dense_bounds); H' = the in-frame cells where that bound exceeds
    // sigclip (less a margin) holds H.
    constexpr int TTY = 2, TTX = 5, PW = TTX + 4;
    static_assert(TTY == 2 && TTX == 5, "dense_bounds takes 2 x 5 cell tiles");
    constexpr int NTY = (L::SH + TTY - 1) / TTY, NTX = (L::SW + TTX - 1) / TTX;
    const SEstParams sp = sest_params(f);
#pragma unroll 1
    for (int ti = tid; ti < NTY * NTX; ti += NT) {
        // column-major over the 2 x 5 tiles in groups of 16 row pairs, then the remaining
        // row pairs: a row pair's loads sit 2 * 73 = 18 banks (mod 32) after the previous
        // one's, so the 16 row pairs of a column tile take 16 distinct banks of one parity
        // and a half-wave's two column tiles (5 columns apart) the two parities; the
        // patch loads of a whole group are free of bank conflicts
        static_assert(2 * L::JWP % 32 == 18, "the bank spread assumes a J pitch of 9 mod 32");
        constexpr int NFULL = (NTY / 16) * 16;
        constexpr int NREM = NTY > NFULL ? NTY - NFULL : 1;     // (unused when 0)
        int tx, k;
        if (ti < NFULL * NTX) {
            const int g = ti / (16 * NTX), e = ti - g * (16 * NTX);
            tx = e >> 4;
            k = 16 * g + (e & 15);
        } else {
            const int e = ti - NFULL * NTX;
            tx = e / NREM;
            k = NFULL + (e - tx * NREM);
        }
        const int r5 = min(k * TTY, L::SH - TTY);
        const int c5 = min(tx * TTX, L::SW - TTX);
        float v[(TTY + 4) * PW], u[TTY * TTX];
#pragma unroll
        for (int i = 0; i < TTY + 4; ++i)
#pragma unroll
            for (int j = 0; j < PW; ++j)
                v[i * PW + j] = sJ[(r5 + i) * L::JWP + c5 + j];
        const bool bound_ok = dense_bounds(v, sp, u);
        const int gx0 = x0 - 2 + c5;
        // in-frame columns of the tile's five, as a bit mask
        const uint32_t colmask = (gx0 >= 0 && gx0 + TTX <= W)
                                     ? (1u << TTX) - 1u
                                     : (((1u << TTX) - 1u) << max(-gx0, 0)) &
                                           ((1u << max(min(W - gx0, TTX), 0)) - 1u);
#pragma unroll
        for (int i = 0; i < TTY; ++i) {
            uint32_t bits = 0u;
#pragma unroll
            for (int j = 0; j < TTX; ++j)
                bits |= u[i * TTX + j] > sc_lo ? 1u << j : 0u;
            // where the analysis of the estimate does not hold at the bound, every cell
            bits = bound_ok ? bits : (1u << TTX) - 1u;
            const int gy = y0 - 2 + r5 + i;
            bits = (gy >= 0 && gy < H) ? bits & colmask : 0u;
            if (bits) {
                const int w = c5 >> 5, sh = c5 & 31;
                atomicOr(&sHot[(r5 + i) * L::HWP + w], bits << sh);
                if (sh > 32 - TTX && (bits >> (32 - sh)))
                    atomicOr(&sHot[(r5 + i) * L::HWP + w + 1], bits >> (32 - sh));
            }
        }
    }
    __syncthreads();
    // The later stages read S (to within the block's largest error bound) and med5(J)
    // only within 4 cells of H': the work set lies within 2 of H', and med5(S) at a work
    // pixel reads 2 further (a clamped neighbour's cell is no farther).  That region, in
    // 2 x 2 cell quads (row pair p, even column c: one 32-column word per lane), is
    // listed by the first waves and the quads take the exact med5 network in list order.
    constexpr int NP = L::SH / 2;
    constexpr int kQuadWords = NP * L::HW;
    constexpr int kQuadWaves = (kQuadWords + 63) / 64;
    static_assert(L::SH % 2 == 0 && L::SW % 2 == 0 && kQuadWaves <= L::NW,
                  "whole quads; the quad bitmap words fit the block's waves");
    constexpr int kQuads = NP * L::SW / 2;
    static_assert(kQuads <= TY * TX / 2, "the quad list fits in the code plane");
    uint16_t *const sQuads = reinterpret_cast<uint16_t *>(sCode);   // codes start later
    if (tid < 64 * kQuadWaves) {
        uint32_t m = 0u;
        const int pr = tid / L::HW, w = tid - pr * L::HW;
        if (tid < kQuadWords) {
            uint32_t a = 0u, b = 0u, c = 0u;        // words w - 1, w, w + 1 of the rows
            const uint32_t *row = &sHot[(2 * pr - 4) * L::HWP + w];
#pragma unroll
            for (int kk = 0; kk < 10; ++kk) {
                a |= row[kk * L::HWP - 1];
                b |= row[kk * L::HWP];
                c |= row[kk * L::HWP + 1];
            }
            // column 32w + k is needed when a bit lies in columns 32w + k - 4 .. + 4
            const unsigned long long hi = ((unsigned long long)c << 32) | b;
            const unsigned long long lo = ((unsigned long long)b << 32) | a;
#pragma unroll
            for (int d = 0; d <= 4; ++d)
                m |= (uint32_t)(hi >> d);
#pragma unroll
            for (int d = 1; d <= 4; ++d)
                m |= (uint32_t)(lo >> (32 - d));
            const int valid = L::SW - 32 * w;
            if (valid < 32)
                m &= (1u << valid) - 1u;
            // quads by their even column
            m = (m | (m >> 1)) & 0x55555555u;
        }
        list_append(m, pr * L::SW + 32 * w, sQuads, &sNeedCount, (unsigned int)kQuads, lane);
    }
    __syncthreads();
    // Exact pass: med5(J), L+ and the S estimate with its error bound; the block's largest
    // bound is taken over these cells, the only ones read, and H' drops the cells where
    // the estimate at med5(J) settles S <= sigclip (so H' is {s + err > sigclip less the
    // margin} on the in-frame cells, as with the estimate everywhere).
    const int nquads = (int)sNeedCount;
    {
        float emax = 0.0f;
        unsigned int ncells = 0u;
        const bool counting = (f.flags & kCountWork) != 0;
        // The cells (rr, cc) and (rr, cc + 1) of a quad row (cc even), given their
        // med5(J) and their 4-neighbours (u above, d below, l left of the first cell, r
        // right of the second): the S estimates, the block's error bound, and one H' word
        // and one low word updated per row.  A quad's two columns share their word of
        // each bitmap and lie both inside the tile's columns or both outside.
        auto exact_row = [&](int rr, int cc, float u0, float u1, float l, float c0, float c1,
                             float r, float d0, float d1, float m0, float m1) {
            const int cx = cc - 2, cy = rr - 2;
            const bool tile_row = cx >= 0 && cx < TX && cy >= 0 && cy < TY;
            float e0, e1;
            const float s0 = s_estimate(c0, u0, d0, l, c1, m0, sp, e0);
            const float s1 = s_estimate(c1, u1, d1, c0, r, m1, sp, e1);
            sS[rr * L::SWP + cc] = s0;
            sS[rr * L::SWP + cc + 1] = s1;
            emax = fmaxf(emax, fmaxf(e0, e1));
            // H' keeps the cells whose estimate at med5(J) may exceed sigclip
            const uint32_t drop = (!(s0 + e0 > sc_lo) ? 1u << (cc & 31) : 0u) |
                                  (!(s1 + e1 > sc_lo) ? 1u << ((cc + 1) & 31) : 0u);
            // S may exceed sigfrac * sigclip here (the cell's own bound)
            const uint32_t low = (s0 + e0 > ll_lo ? 1u << (cx & 31) : 0u) |
                                 (s1 + e1 > ll_lo ? 1u << ((cx + 1) & 31) : 0u);
            uint32_t *hw = &sHot[rr * L::HWP + (cc >> 5)];
            if (drop & *hw)
                atomicAnd(hw, ~drop);
            if (tile_row && low)
                atomicOr(&sLow[cy * L::QW + (cx >> 5)], low);
            if (counting)
                ncells += tile_row ? 2u : 0u;
        };
        // Wave w takes the list's entries 64 w, 64 w + 256, ...: one quad per lane (the
        // 2 x 2 network) while more than 32 remain, and a last run of at most 32 quads
        // two lanes per quad, one row each (the 1 x 2 network and two estimates, about
        // 60% of a quad's instructions), as most tiles end their list with such a run.
#pragma unroll 1
        for (int q0 = tid - lane; q0 < nquads; q0 += NT) {
            const int left = nquads - q0;                 // uniform in the wave
            if (left > 32) {
                if (lane < left) {
                    const int q = (int)sQuads[q0 + lane];
                    const int pr = q / L::SW, cc = q - pr * L::SW, r0 = 2 * pr;
                    float v[6 * 6];
#pragma unroll
                    for (int i = 0; i < 6; ++i)
#pragma unroll
                        for (int j = 0; j < 6; ++j)
                            v[i * 6 + j] = sJ[(r0 + i) * L::JWP + cc + j];
                    float m5[4];
                    med5_t2x2(v, m5);
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        constexpr int P = 6;
                        const int pc = (i + 2) * P + 2;
                        exact_row(r0 + i, cc, v[pc - P], v[pc + 1 - P], v[pc - 1], v[pc],
                                  v[pc + 1], v[pc + 2], v[pc + P], v[pc + 1 + P], m5[2 * i],
                                  m5[2 * i + 1]);
                    }
                }
            } else if (lane < 2 * left) {
                const int q = (int)sQuads[q0 + (lane >> 1)];
                const int pr = q / L::SW, cc = q - pr * L::SW, rr = 2 * pr + (lane & 1);
                float v[5 * 6];
#pragma unroll
                for (int i = 0; i < 5; ++i)
#pragma unroll
                    for (int j = 0; j < 6; ++j)
                        v[i * 6 + j] = sJ[(rr + i) * L::JWP + cc + j];
                float m5[2];
                med5_t1x2(v, m5);
                constexpr int P = 6, pc = 2 * P + 2;
                exact_row(rr, cc, v[pc - P], v[pc + 1 - P], v[pc - 1], v[pc], v[pc + 1],
                          v[pc + 2], v[pc + P], v[pc + 1 + P], m5[0], m5[1]);
            }
        }
        // non-negative floats order as their bit patterns: the device library's
        // cross-lane (DPP) maximum, then one LDS atomic per wave
        emax = __uint_as_float(__ockl_wfred_max_u32(__float_as_uint(emax)));
        if (lane == 0)
            atomicMax(&sErrBits, __float_as_uint(emax));
        if (counting) {
            ncells = __ockl_wfred_add_u32(ncells);
            if (lane == 0 && ncells)
                atomicAdd(&sExactCells, ncells);
        }
    }
    __syncthreads();

    // Region cells outside the image must hold the value of their clamped cell: the
    // windows of the work set read S at clamped neighbour positions.
    if (y0 < 2 || x0 < 2 || y0 + TY + 2 > H || x0 + TX + 2 > W) {
        for (int i = tid; i < L::SH * L::SW; i += NT) {
            const int r = i / L::SW, c = i - r * L::SW;
            const int gy = y0 - 2 + r, gx = x0 - 2 + c;
            if (gy < 0 || gy >= H || gx < 0 || gx >= W)
                sS[r * L::SWP + c] =
                    sS[(clampi(gy, H) - (y0 - 2)) * L::SWP + (clampi(gx, W) - (x0 - 2))];
        }
    }
    for (int i = tid; i < TY * TX / 4; i += NT)
        reinterpret_cast<uint32_t *>(sCode)[i] = 0u;
    const float emax = __uint_as_float(sErrBits);
    // no estimate of the block is usable: every work pixel is re-evaluated
    const bool all_exact = !(emax < INFINITY) || (f.flags & kExactDetect);
    // work set Q' on the tile's in-frame pixels, one 32-pixel word per lane of the first
    // waves, appended to a compact list of tile positions (in any order)
    constexpr int kWorkWaves = (L::kTileWords + 63) / 64;
    if (tid < 64 * kWorkWaves) {
        uint32_t q = 0u;
        if (tid < L::kTileWords) {
            const int r = tid / L::QW, w = tid - r * L::QW;
            unsigned long long x = 0ull;
#pragma unroll
            for (int dr = 0; dr < 5; ++dr) {
                const uint32_t *row = &sHot[(r + dr) * L::HWP + w];
                x |= (unsigned long long)row[0] | ((unsigned long long)row[1] << 32);
            }
            // bit b of the dilation covers region columns 32w+b .. 32w+b+4, centred on
            // the tile column 32w+b
            q = (uint32_t)(x | (x >> 1) | (x >> 2) | (x >> 3) | (x >> 4));
            const int vc = W - x0 - 32 * w;
            if (y0 + r >= H || vc <= 0)
                q = 0u;
            else if (vc < 32)
                q &= (1u << vc) - 1u;
            q &= sLow[tid];
            sLow[tid] = q;
            if (all_exact)
                sU[tid] = q;
        }
        // word tid covers tile positions tid * 32 .. (r * TX + 32 w with two words a row)
        list_append(q, tid * 32, sList, &sQcount, (unsigned int)kListMax, lane);
    }
    __syncthreads();

    const int total = (int)sQcount;
    // the work set, compacted: thread t takes the t-th, (t+NT)-th, ... pixel of Q' (of
    // the tile, tested against the Q' bitmap, when the list could not hold Q').
    // S' from the estimates lies within B of the binary64 S' (B covers twice the
    // block's largest error and, with 4u, the roundings of the differences)
    const bool listed_q = total <= kListMax;
    if (!all_exact) {
        const float b2 = 2.02f * emax;
        const float olim_lo = f.olim_lo, olim_hi = f.olim_hi;
        unsigned int ncontrast = 0u, nunc = 0u;
        for (int qi = tid; qi < (listed_q ? total : TY * TX); qi += NT) {
            const int pos = listed_q ? (int)sList[qi] : qi;
            if (!listed_q && !((sLow[pos >> 5] >> (pos & 31)) & 1u))
                continue;
            const int r = pos / TX, c = pos - r * TX;
            float w[25], ms[1];
#pragma unroll
            for (int i = 0; i < 5; ++i)
#pragma unroll
                for (int j = 0; j < 5; ++j)
                    w[i * 5 + j] = sS[(r + i) * L::SWP + c + j];
            med5_t1x1(w, ms);
            const float spr = w[12] - ms[0];
            const float B = fmaf(fabsf(spr), 0x1p-22f, b2);
            const float lo = spr - B, hi = spr + B;
            const bool h1 = lo > sc_hi, h0 = hi <= sc_lo, l1 = lo > ll_hi, l0 = hi <= ll_lo;
            bool unc = !((h1 || h0) && (l1 || l0));
            bool listed = false, first = false;
            if (!unc && h1) {
                // S'/F^ <= S'/0.01 <= objlim for the whole interval: the test fails
                if (hi * 100.0f <= olim_lo) {
                    ++ncontrast;
                } else if (!(lo * 100.0f > olim_hi)) {
                    unc = true;
                } else {
                    const unsigned int slot = atomicAdd(&sConCount, 1u);
                    // N from the pixel's estimate (w[12], positive here) and its L+ sum
                    const float *pj = &sJ[(r + 4) * L::JWP + c + 4];
                    const float nz = noise_from_estimate(
                        lplus4(pj[0], pj[-L::JWP], pj[L::JWP], pj[-1], pj[1]), w[12]);
                    if (slot < (unsigned int)kConMax) {
                        sConInfo[slot] = (uint32_t)pos | (l1 ? 1u << 16 : 0u);
                        sConLo[slot] = lo;
                        sConHi[slot] = hi;
                        sConN[slot] = nz;
                        listed = true;
                    } else {
                        const int t = contrast_by_count_lane(sJ, L::JWP, y0, x0, H, W, r, c,
                                                             nz, lo, hi, f.inv_olim);
                        first = t > 0;
                        unc = t < 0;
                        ncontrast += unc ? 0u : 1u;
                    }
                }
            }
            if (unc) {
                atomicOr(&sU[pos >> 5], 1u << (pos & 31));
                ++nunc;
            } else if (!listed) {
                sCode[pos] = (uint8_t)((first ? 1 : 0) | (h1 ? 2 : 0) | (l1 ? 4 : 0));
            }
        }
        if (ncontrast && (f.flags & kCountWork))
            atomicAdd(&sContrast, ncontrast);
        if (nunc)
            atomicAdd(&sUncertain, nunc);
    } else if (tid == 0) {
        sUncertain = (unsigned int)total;     // sU holds Q'
    }
    __syncthreads();

    // contrast tests of the listed pixels (S' > sigclip certain), one wave per pixel
    const int ncon = min((int)sConCount, kConMax);
    if (ncon) {
        const float inv_olim = f.inv_olim;
        unsigned int ncontrast = 0u, nunc = 0u;
        for (int it = tid >> 6; it < ncon; it += L::NW) {
            const uint32_t info = sConInfo[it];
            const int pos = (int)(info & 0xFFFFu);
            const int r = pos / TX, c = pos - r * TX;
            const int t = contrast_by_count(sJ, L::JWP, y0, x0, H, W, r, c, sConN[it],
                                            sConLo[it], sConHi[it], inv_olim, lane);
            if (lane == 0) {
                if (t < 0) {
                    atomicOr(&sU[pos >> 5], 1u << (pos & 31));
                    ++nunc;
                } else {
                    sCode[pos] = (uint8_t)((t > 0 ? 1 : 0) | 2 | ((info >> 16) ? 4 : 0));
                    ++ncontrast;
                }
            }
        }
        if (ncontrast && (f.flags & kCountWork))
            atomicAdd(&sContrast, ncontrast);
        if (nunc)
            atomicAdd(&sUncertain, nunc);
        __syncthreads();
    }

    // binary64 re-evaluation of the undecided pixels from J, kExactBatch per round:
    // 25 threads compute the S window of a pixel, then one thread its codes
    const int nunc = (int)sUncertain;
    if (nunc) {
        // the binary64 parameters (read here, on this rare path only)
        const double gain = f.gain, sky = f.sky, rn = f.readnoise;
        const double rn2 = rn * rn, sigclip = f.sigclip, objlim = f.objlim;
        const double lowlim = (double)f.sigfrac * (double)f.sigclip;
        if (tid < 64)
            bitmap_prefix<L::kTileWords>(sU, sUpre);
        __syncthreads();
        unsigned int ncontrast = 0u;
        for (int base = 0; base < nunc; base += kExactBatch) {
            const int slot = tid / 25, cell = tid - slot * 25;
            if (slot < kExactBatch && base + slot < nunc) {
                const int pos = bitmap_select<L::kTileWords>(sU, sUpre, base + slot);
                const int r = pos / TX, c = pos - r * TX;
                const int i = cell / 5, j = cell - i * 5;
                // window cell in frame coordinates, clamped
                const int gy = clampi(y0 + r + i - 2, H), gx = clampi(x0 + c + j - 2, W);
                sX[slot * 25 + cell] = s_exact(J, H, W, gy, gx, gain, sky, rn2);
            }
            __syncthreads();
            // med5 of the window by ranks: the value with at most 12 smaller and at
            // least 13 not larger (equal values write the same median)
            if (slot < kExactBatch && base + slot < nunc) {
                const double v = sX[slot * 25 + cell];
                int lt = 0, le = 0;
#pragma unroll 5
                for (int q = 0; q < 25; ++q) {
                    const double u = sX[slot * 25 + q];
                    lt += u < v ? 1 : 0;
                    le += u <= v ? 1 : 0;
                }
                if (lt <= 12 && le >= 13)
                    sX[kExactBatch * 25 + slot] = v;
            }
            __syncthreads();
            if (tid < kExactBatch && base + tid < nunc) {
                const int pos = bitmap_select<L::kTileWords>(sU, sUpre, base + tid);
                const int r = pos / TX, c = pos - r * TX;
                const double spr = sX[tid * 25 + 12] - sX[kExactBatch * 25 + tid];
                const bool hbit = spr > sigclip, lbit = spr > lowlim;
                bool first = false;
                if (hbit) {
                    float w5[25], m5[1];
#pragma unroll
                    for (int i = 0; i < 5; ++i)
#pragma unroll
                        for (int j = 0; j < 5; ++j)
                            w5[i * 5 + j] = sJ[(r + 2 + i) * L::JWP + c + 2 + j];
                    med5_t1x1(w5, m5);
                    first = contrast_exact(sJ, L::JWP, y0, x0, H, W, r, c, spr,
                                           noise_exact(m5[0], gain, sky, rn2), objlim);
                    ++ncontrast;
                }
                sCode[pos] = (uint8_t)((first ? 1 : 0) | (hbit ? 2 : 0) | (lbit ? 4 : 0));
            }
            __syncthreads();
        }
        if (ncontrast && (f.flags & kCountWork))
            atomicAdd(&sContrast, ncontrast);
        __syncthreads();
    }

    // codes of the tile, 8 per thread: thread t writes 8 pixels of row t / 8, so wave w
    // holds rows 8w .. 8w+7 and writes its byte of the summary word of the 32 x 64
    // summary tile those rows lie in: bit 0 where A is set in those rows, bit 1 where in
    // the summary tile's rows 0-1, bit 2 where in its rows 30-31
    static_assert(TX == kSumTX && kSumTY == 32 && TY % 8 == 0, "8-row waves on the summary grid");
    uint8_t *__restrict__ codes = f.codes;
    {
        const int r = tid / (TX / 8), c = (tid - r * (TX / 8)) * 8;
        const int gy = y0 + r, gx = x0 + c;
        const uint2 word = *reinterpret_cast<const uint2 *>(&sCode[r * TX + c]);
        if (f.tile_first) {
            const unsigned long long rows_a = __ballot(((word.x | word.y) & 0x01010101u) != 0u);
            const int gr = y0 + 8 * (tid >> 6);      // first row of the wave
            if (lane == 0 && gr < H) {
                const int sb = (gr & (kSumTY - 1)) >> 3;
                const unsigned int bits = (rows_a ? 1u : 0u) |
                                          (sb == 0 && (rows_a & 0xFFFFull) ? 2u : 0u) |
                                          (sb == 3 && (rows_a >> 48) ? 4u : 0u);
                f.tile_first[4 * ((gr / kSumTY) * ((W + kSumTX - 1) / kSumTX) + x0 / kSumTX) +
                             sb] = (uint8_t)bits;
            }
        }
        if (gy < H && gx < W) {
            uint8_t *dst = codes + (size_t)gy * W + gx;
            if (gx + 8 <= W && ((uintptr_t)dst & 7u) == 0u) {
                *reinterpret_cast<uint2 *>(dst) = word;
            } else {
                const int nb = min(8, W - gx);
                for (int b = 0; b < nb; ++b)
                    dst[b] = sCode[r * TX + c + b];
            }
        }
    }
    if ((f.flags & kCountWork) && tid == 0 && f.work) {
        if (total)
            atomicAdd(&f.work[0], (unsigned long long)total);
        if (sContrast)
            atomicAdd(&f.work[1], (unsigned long long)sContrast);
        if (nunc)
            atomicAdd(&f.work[2], (unsigned long long)nunc);
        if (sExactCells)
            atomicAdd(&f.work[3], (unsigned long long)sExactCells);
    }
}

// (frame, tile origin) of tile t of a launch: from the work list, or for a single frame
// (tiles == null) the row-major tile t of its grid.
template <int TY>
__device__ __forceinline__ void tile_of(const DevFrame *__restrict__ frames,
                                        const TileRef *__restrict__ tiles, const DevFrame &single,
                                        int t, DevFrame &f, int &y0, int &x0) {
    if (tiles) {
        const TileRef r = tiles[t];
        f = frames[r.frame];
        y0 = r.y0;
        x0 = r.x0;
    } else {
        f = single;
        const int ntx = (single.W + kSumTX - 1) / kSumTX;
        y0 = (t / ntx) * TY;
        x0 = (t - (t / ntx) * ntx) * kSumTX;
    }
}

// One block per tile.
template <int TY>
__global__ __launch_bounds__(8 * TY) __attribute__((amdgpu_waves_per_eu(TY == 16 ? 4 : 6)))
void k_detect(const DevFrame *__restrict__ frames, const TileRef *__restrict__ tiles,
              DevFrame single, int kiter) {
    DevFrame f;
    int y0, x0;
    tile_of<TY>(frames, tiles, single, (int)blockIdx.x, f, y0, x0);
    detect_tile<TY>(f, y0, x0, kiter ? kiter : f.k, (int)threadIdx.x);
}

// Persistent blocks over a (frame, tile) work list: the grid holds about as many
// blocks as are resident at once, and each block takes runs of kRun consecutive tiles
// from kDetectQueues ticket counters (zero at launch, each on its own cache line),
// counter q over the q-th contiguous part of the list.  Blocks are dispatched
// round-robin over the XCDs, so block b starts on part b mod kDetectQueues, and the
// tiles in flight on one XCD are neighbours sharing halo rows and columns in its L2; a
// block whose part is used up moves to the next, and it returns once all parts are
// (every counter only grows, so every block gets there).
template <int TY>
__global__ __launch_bounds__(8 * TY) __attribute__((amdgpu_waves_per_eu(TY == 16 ? 4 : 6)))
void k_detect_persistent(const DevFrame *__restrict__ frames, const TileRef *__restrict__ tiles,
                         int kiter, int ntiles, unsigned int *__restrict__ tickets) {
    constexpr int kRun = 2;
    __shared__ int sTile, sEnd;
    int q = (int)(blockIdx.x % kDetectQueues), tried = 0;
    for (;;) {
        __syncthreads();      // the previous run is done with the LDS and with sTile
        if (threadIdx.x == 0) {
            int t = -1, end = -1;
            while (tried < kDetectQueues) {
                const unsigned int lo = (unsigned int)((long long)ntiles * q / kDetectQueues);
                const unsigned int hi =
                    (unsigned int)((long long)ntiles * (q + 1) / kDetectQueues);
                const unsigned int got =
                    lo + (unsigned int)kRun * atomicAdd(&tickets[q * kTicketStride], 1u);
                if (got < hi) {
                    t = (int)got;
                    end = (int)min(got + (unsigned int)kRun, hi);
                    break;
                }
                q = (q + 1) % kDetectQueues;
                ++tried;
            }
            sTile = t;
            sEnd = end;
        }
        __syncthreads();
        // uniform over the block: the tile and frame records then load into scalar
        // registers, as with blockIdx.x in the one-block-per-tile kernel
        const int t0 = __builtin_amdgcn_readfirstlane(sTile);
        const int t1 = __builtin_amdgcn_readfirstlane(sEnd);
        if (t0 < 0)
            return;
        for (int t = t0; t < t1; ++t) {
            if (t > t0)
                __syncthreads();   // the previous tile is done with the LDS
            const TileRef r = tiles[t];
            // the frame record is read in place, each field where the tile first needs it,
            // rather than copied whole into scalar registers at the start of every tile
            const DevFrame &f = frames[r.frame];
            // the thread index passes through an empty asm statement each round, so that
            // values derived from it are recomputed per tile rather than held in registers
            // across the loop
            int tid = (int)threadIdx.x;
            asm volatile("" : "+v"(tid));
            detect_tile<TY>(f, r.y0, r.x0, kiter ? kiter : f.k, tid);
        }
    }
}

// ---------------------------------------------------------------------------
// parity-test kernels: the median networks alone
// ---------------------------------------------------------------------------

// Output tile of one thread of k_debug_median: the shapes the kernels use (med3 in runs,
// med5 in 2 x 2 quads, by the quad network on even tile rows and the one-row network on
// odd ones, med7 single).
__host__ __device__ constexpr int debug_median_ty(int r) { return r == 2 ? 2 : 1; }
__host__ __device__ constexpr int debug_median_tx(int r) { return r == 1 ? kRun3 : (r == 2 ? 2 : 1); }

template <int R>
__global__ __launch_bounds__(kThreads) void k_debug_median(const float *__restrict__ in, int H,
                                                           int W, float *__restrict__ out) {
    constexpr int TY = debug_median_ty(R), TX = debug_median_tx(R);
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
        if (((t / ntx) & 1) == 0) {
            med5_t2x2(v, o);
        } else {
            // odd tile rows: the one-row network (two outputs) on each of the two rows
            float a[5 * PW], b[5 * PW], oa[2], ob[2];
#pragma unroll
            for (int i = 0; i < 5 * PW; ++i) {
                a[i] = v[i];
                b[i] = v[PW + i];
            }
            med5_t1x2(a, oa);
            med5_t1x2(b, ob);
            o[0] = oa[0];
            o[1] = oa[1];
            o[2] = ob[0];
            o[3] = ob[1];
        }
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

// 5x5 clamped median of binary64 values by the single-output network (the one the
// detection applies to the FP32 estimates of S, here on binary64 inputs).
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

// The detection kernel's FP32 estimate of S and its error bound, one pixel per thread
// (clamped neighbours and med5(J) from a single-output network).
__global__ __launch_bounds__(kThreads) void k_debug_s_estimate(DevFrame f,
                                                               float *__restrict__ out_s,
                                                               float *__restrict__ out_err) {
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const int H = f.H, W = f.W;
    if (t >= (long long)H * W)
        return;
    const int y = (int)(t / W), x = (int)(t - (long long)y * W);
    float w[25], m5[1];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j)
            w[i * 5 + j] = f.img[(size_t)clampi(y - 2 + i, H) * W + clampi(x - 2 + j, W)];
    med5_t1x1(w, m5);
    float err;
    out_s[t] = s_estimate(w[12], w[7], w[17], w[11], w[13], m5[0], sest_params(f), err);
    out_err[t] = err;
}

// The detection's dense upper bound of S at every pixel of one frame: 2 x 5 cell tiles
// aligned at the frame's origin, one per thread, each from its clamped 6 x 9 patch;
// INFINITY where the bound's analysis does not hold.
__global__ __launch_bounds__(kThreads) void k_debug_s_bound(DevFrame f, float *__restrict__ out_u) {
    const int H = f.H, W = f.W;
    const int ntx = (W + 4) / 5, nty = (H + 1) / 2;
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t >= (long long)ntx * nty)
        return;
    const int y0 = (int)(t / ntx) * 2, x0 = (int)(t % ntx) * 5;
    float v[6 * 9], u[10];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 9; ++j)
            v[i * 9 + j] = f.img[(size_t)clampi(y0 - 2 + i, H) * W + clampi(x0 - 2 + j, W)];
    const bool ok = dense_bounds(v, sest_params(f), u);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j)
            if (y0 + i < H && x0 + j < W)
                out_u[(size_t)(y0 + i) * W + x0 + j] = ok ? u[i * 5 + j] : INFINITY;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_debug_s_bound(const DevFrame &f, float *out_u, hipStream_t s) {
    const size_t n = (size_t)((f.W + 4) / 5) * (size_t)((f.H + 1) / 2);
    k_debug_s_bound<<<(unsigned int)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(f, out_u);
    return hipGetLastError();
}

hipError_t launch_debug_s_estimate(const DevFrame &f, float *out_s, float *out_err,
                                   hipStream_t s) {
    const size_t n = (size_t)f.H * (size_t)f.W;
    k_debug_s_estimate<<<(unsigned int)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        f, out_s, out_err);
    return hipGetLastError();
}

// Resident blocks of a persistent detection launch: the occupancy the runtime reports
// for the kernel, times the compute units (looked up once per device and tile height).
template <int TY>
static int persistent_grid() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 0;
    if (!cached[dev]) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_detect_persistent<TY>,
                                                         8 * TY, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess)
            return 0;
        cached[dev] = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    }
    return cached[dev];
}

template <int TY>
static hipError_t launch_detect_ty(const DevFrame *d_frames, const TileRef *d_tiles,
                                   int ntiles, const DevFrame &single, int k, bool persistent,
                                   unsigned int *tickets, hipStream_t s) {
    if (ntiles <= 0)
        return hipSuccess;
    if (persistent && tickets && d_tiles) {
        const int cap = persistent_grid<TY>();
        if (cap <= 0)
            return hipErrorInvalidValue;
        const int grid = ntiles < cap ? ntiles : cap;
        k_detect_persistent<TY><<<grid, 8 * TY, 0, s>>>(d_frames, d_tiles, k, ntiles, tickets);
    } else {
        k_detect<TY><<<ntiles, 8 * TY, 0, s>>>(d_frames, d_tiles, single, k);
    }
    return hipGetLastError();
}

hipError_t launch_detect(const DevFrame *d_frames, const TileRef *d_tiles, int ntiles,
                         const DevFrame &single, int k, const LaunchCfg &cfg,
                         unsigned int *tickets, hipStream_t s) {
    if (!d_tiles)
        ntiles = detect_tiles(single.H, single.W, cfg.tile_h);
    switch (cfg.tile_h) {
    case 16:
        return launch_detect_ty<16>(d_frames, d_tiles, ntiles, single, k, cfg.persistent != 0,
                                    tickets, s);
    case 32:
        return launch_detect_ty<32>(d_frames, d_tiles, ntiles, single, k, cfg.persistent != 0,
                                    tickets, s);
    case 64:
        return launch_detect_ty<64>(d_frames, d_tiles, ntiles, single, k, cfg.persistent != 0,
                                    tickets, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_debug_median5_f64(const double *in, int H, int W, double *out,
                                   hipStream_t s) {
    const size_t n = (size_t)H * (size_t)W;
    k_debug_median5_f64<<<(unsigned int)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(in, H,
                                                                                         W, out);
    return hipGetLastError();
}

hipError_t launch_debug_median(const float *in, int H, int W, int r, float *out, hipStream_t s) {
    const int ty = debug_median_ty(r), tx = debug_median_tx(r);
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
