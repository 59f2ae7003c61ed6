/*
 * crb_ref.c -- plain single-threaded FP64 L.A.Cosmic oracle (test infrastructure).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  It shares no code, header or table with the GPU
 * library and is deliberately slow: sort-based medians, the 2x-subsampled grid
 * materialised, every plane stored.
 *
 * Method (Mighell, Section 5, L.A.Cosmic as used by CRBLASTER; the paper fixes
 * double precision for the subimage data, Section 6.2, and says the C code
 * follows van Dokkum's script closely, Section 7).  One iteration on J_k with
 * cumulative mask M_{k-1}:
 *   1. L+  : 2x block replication, 4-neighbour Laplacian, clip at zero, 2x2 mean
 *   2. N   : m5 = med5(J) + sky (floored at 1e-4 when <= 0); N = sqrt(g m5 + rn^2)/g
 *   3. S   : S = L+ / (2 N);  S' = S - med5(S)
 *   4. F^  : m3 = med3(J); F = m3 - med7(m3); F^ = max(F / N, 0.01)
 *   5. A   : S' > sigclip and S'/F^ > objlim
 *   6. G1  : 3x3 dilation of A, kept where S' > sigclip
 *   7. G2  : 3x3 dilation of G1, kept where S' > sigfrac * sigclip
 *   8. n_k = #(G2 and not M_{k-1});  M_k = M_{k-1} or G2
 *   9. J_{k+1}(p) = median of the unflagged J_k in the clamped 5x5 window of
 *      each p in M_k (even count: mean of the two middle values; empty: J_k(p));
 *      all other pixels keep J_k(p)
 *  10. stop when n_k = 0 (if requested) or after niter iterations.
 */
#include "crb_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

/* ascending insertion sort */
static void sort_doubles(double *v, int n)
{
    for (int i = 1; i < n; ++i) {
        double x = v[i];
        int j = i - 1;
        while (j >= 0 && v[j] > x) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = x;
    }
}

/* median of n >= 1 values (v is reordered): odd n -> middle order statistic,
 * even n -> mean of the two middle values */
static double median_of(double *v, int n)
{
    sort_doubles(v, n);
    if (n % 2 == 1)
        return v[n / 2];
    return 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

int crb_ref_median_filter(const double *in, int H, int W, int r, double *out)
{
    if (!in || !out || H < 1 || W < 1 || r < 0)
        return -1;
    int k = 2 * r + 1;
    double *win = (double *)malloc(sizeof(double) * (size_t)k * (size_t)k);
    if (!win)
        return -2;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int n = 0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx)
                    win[n++] = in[(size_t)clampi(y + dy, H) * W + clampi(x + dx, W)];
            out[(size_t)y * W + x] = median_of(win, n);
        }
    }
    free(win);
    return 0;
}

int crb_ref_lplus(const double *J, int H, int W, double *out)
{
    if (!J || !out || H < 1 || W < 1)
        return -1;
    int H2 = 2 * H, W2 = 2 * W;
    double *J2 = (double *)malloc(sizeof(double) * (size_t)H2 * (size_t)W2);
    double *L2 = (double *)malloc(sizeof(double) * (size_t)H2 * (size_t)W2);
    if (!J2 || !L2) {
        free(J2);
        free(L2);
        return -2;
    }
    /* 2x subsample: every pixel becomes a 2x2 block of its own value */
    for (int Y = 0; Y < H2; ++Y)
        for (int X = 0; X < W2; ++X)
            J2[(size_t)Y * W2 + X] = J[(size_t)(Y / 2) * W + (X / 2)];
    /* Laplacian [[0,-1,0],[-1,4,-1],[0,-1,0]] on the 2x grid, negatives set to zero */
    for (int Y = 0; Y < H2; ++Y) {
        for (int X = 0; X < W2; ++X) {
            double c = J2[(size_t)Y * W2 + X];
            double u = J2[(size_t)clampi(Y - 1, H2) * W2 + X];
            double d = J2[(size_t)clampi(Y + 1, H2) * W2 + X];
            double l = J2[(size_t)Y * W2 + clampi(X - 1, W2)];
            double r = J2[(size_t)Y * W2 + clampi(X + 1, W2)];
            double v = 4.0 * c - u - d - l - r;
            L2[(size_t)Y * W2 + X] = v > 0.0 ? v : 0.0;
        }
    }
    /* 2x2 rebin by block mean */
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            double a = L2[(size_t)(2 * y) * W2 + 2 * x];
            double b = L2[(size_t)(2 * y) * W2 + 2 * x + 1];
            double c = L2[(size_t)(2 * y + 1) * W2 + 2 * x];
            double d = L2[(size_t)(2 * y + 1) * W2 + 2 * x + 1];
            out[(size_t)y * W + x] = (a + b + c + d) / 4.0;
        }
    }
    free(J2);
    free(L2);
    return 0;
}

/* 8-connected 3x3 dilation of a 0/1 plane, clamped window */
static void dilate3(const uint8_t *in, int H, int W, uint8_t *out)
{
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            uint8_t any = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    any |= in[(size_t)clampi(y + dy, H) * W + clampi(x + dx, W)];
            out[(size_t)y * W + x] = any ? 1 : 0;
        }
    }
}

static int params_ok(const crb_ref_params *p)
{
    if (!p)
        return 0;
    if (!isfinite(p->gain) || !isfinite(p->readnoise) || !isfinite(p->sky) ||
        !isfinite(p->sigclip) || !isfinite(p->sigfrac) || !isfinite(p->objlim))
        return 0;
    return p->gain > 0.0 && p->readnoise >= 0.0 && p->sigclip > 0.0 &&
           p->sigfrac >= 0.0 && p->sigfrac <= 1.0 && p->objlim > 0.0;
}

int crb_ref_iterate(const double *J, const uint8_t *Mprev, int H, int W,
                    const crb_ref_params *p, uint8_t *out_G2, uint8_t *out_M,
                    double *out_Jnext, long long *out_nnew, crb_ref_trace *trace)
{
    if (!J || !Mprev || H < 1 || W < 1 || !params_ok(p))
        return -1;
    size_t n = (size_t)H * (size_t)W;
    int rc = -2;
    double *m5 = malloc(sizeof(double) * n), *N = malloc(sizeof(double) * n);
    double *Lp = malloc(sizeof(double) * n), *S = malloc(sizeof(double) * n);
    double *mS = malloc(sizeof(double) * n), *Sp = malloc(sizeof(double) * n);
    double *m3 = malloc(sizeof(double) * n), *m7 = malloc(sizeof(double) * n);
    double *Fh = malloc(sizeof(double) * n);
    uint8_t *A = malloc(n), *G1 = malloc(n), *G2 = malloc(n), *M = malloc(n), *D = malloc(n);
    double *win = malloc(sizeof(double) * 25);
    if (!m5 || !N || !Lp || !S || !mS || !Sp || !m3 || !m7 || !Fh || !A || !G1 || !G2 ||
        !M || !D || !win)
        goto done;

    /* 2. noise model from the 5x5 median */
    if (crb_ref_median_filter(J, H, W, 2, m5))
        goto done;
    for (size_t i = 0; i < n; ++i) {
        double m = m5[i] + p->sky;
        if (m <= 0.0)
            m = 1e-4;
        N[i] = sqrt(p->gain * m + p->readnoise * p->readnoise) / p->gain;
    }
    /* 1. L+ and 3. S, S' */
    if (crb_ref_lplus(J, H, W, Lp))
        goto done;
    for (size_t i = 0; i < n; ++i)
        S[i] = Lp[i] / (2.0 * N[i]);
    if (crb_ref_median_filter(S, H, W, 2, mS))
        goto done;
    for (size_t i = 0; i < n; ++i)
        Sp[i] = S[i] - mS[i];
    /* 4. fine-structure image */
    if (crb_ref_median_filter(J, H, W, 1, m3) || crb_ref_median_filter(m3, H, W, 3, m7))
        goto done;
    for (size_t i = 0; i < n; ++i) {
        double f = (m3[i] - m7[i]) / N[i];
        Fh[i] = f < 0.01 ? 0.01 : f;
    }
    /* 5. first selection */
    for (size_t i = 0; i < n; ++i)
        A[i] = (Sp[i] > p->sigclip && Sp[i] / Fh[i] > p->objlim) ? 1 : 0;
    /* 6-7. two-stage neighbour growing */
    double lowlim = p->sigfrac * p->sigclip;
    dilate3(A, H, W, D);
    for (size_t i = 0; i < n; ++i)
        G1[i] = (D[i] && Sp[i] > p->sigclip) ? 1 : 0;
    dilate3(G1, H, W, D);
    for (size_t i = 0; i < n; ++i)
        G2[i] = (D[i] && Sp[i] > lowlim) ? 1 : 0;
    /* 8. new-flag count and cumulative mask */
    long long nnew = 0;
    for (size_t i = 0; i < n; ++i) {
        if (G2[i] && !Mprev[i])
            ++nnew;
        M[i] = (Mprev[i] || G2[i]) ? 1 : 0;
    }
    /* 9. replacement by the median of the unflagged clamped 5x5 neighbours */
    if (out_Jnext) {
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                size_t i = (size_t)y * W + x;
                double v = J[i];
                if (M[i]) {
                    int cnt = 0;
                    for (int dy = -2; dy <= 2; ++dy) {
                        for (int dx = -2; dx <= 2; ++dx) {
                            size_t q = (size_t)clampi(y + dy, H) * W + clampi(x + dx, W);
                            if (!M[q])
                                win[cnt++] = J[q];
                        }
                    }
                    if (cnt > 0)
                        v = median_of(win, cnt);
                }
                out_Jnext[i] = v;
            }
        }
    }
    if (out_G2)
        memcpy(out_G2, G2, n);
    if (out_M)
        memcpy(out_M, M, n);
    if (out_nnew)
        *out_nnew = nnew;
    if (trace) {
        if (trace->lplus) memcpy(trace->lplus, Lp, sizeof(double) * n);
        if (trace->noise) memcpy(trace->noise, N, sizeof(double) * n);
        if (trace->s) memcpy(trace->s, S, sizeof(double) * n);
        if (trace->sprime) memcpy(trace->sprime, Sp, sizeof(double) * n);
        if (trace->fhat) memcpy(trace->fhat, Fh, sizeof(double) * n);
        if (trace->first) memcpy(trace->first, A, n);
        if (trace->g1) memcpy(trace->g1, G1, n);
        if (trace->g2) memcpy(trace->g2, G2, n);
    }
    rc = 0;
done:
    free(m5); free(N); free(Lp); free(S); free(mS); free(Sp); free(m3); free(m7); free(Fh);
    free(A); free(G1); free(G2); free(M); free(D); free(win);
    return rc;
}

int crb_ref_lacosmic(const float *img, int H, int W, const crb_ref_params *p,
                     int niter, int early_stop, double *out_clean, uint8_t *out_mask,
                     int *out_iters, long long *out_counts)
{
    if (!img || !out_clean || !out_mask || H < 1 || W < 1 || niter < 0 || !params_ok(p))
        return -1;
    size_t n = (size_t)H * (size_t)W;
    double *J = malloc(sizeof(double) * n), *Jn = malloc(sizeof(double) * n);
    uint8_t *M = calloc(n, 1), *Mn = malloc(n);
    if (!J || !Jn || !M || !Mn) {
        free(J); free(Jn); free(M); free(Mn);
        return -2;
    }
    for (size_t i = 0; i < n; ++i)
        J[i] = (double)img[i];
    int iters = 0;
    for (int k = 1; k <= niter; ++k) {
        long long nk = 0;
        int rc = crb_ref_iterate(J, M, H, W, p, NULL, Mn, Jn, &nk, NULL);
        if (rc) {
            free(J); free(Jn); free(M); free(Mn);
            return rc;
        }
        double *tj = J; J = Jn; Jn = tj;
        uint8_t *tm = M; M = Mn; Mn = tm;
        if (out_counts)
            out_counts[k - 1] = nk;
        iters = k;
        if (early_stop && nk == 0)
            break;
    }
    memcpy(out_clean, J, sizeof(double) * n);
    memcpy(out_mask, M, n);
    if (out_iters)
        *out_iters = iters;
    free(J); free(Jn); free(M); free(Mn);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* POISSON work function (test infrastructure, as above)                      */
/* ------------------------------------------------------------------------- */

/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC 2011): ten rounds of two 32x32->64 multiplications with the
 * round constants below, the key bumped by the Weyl constants after each round. */
void crb_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* exp(-x) for 0 <= x <= 745: x = k ln2 + r with |r| <= ln2/2 (ln2 split in a high
 * part with trailing zero bits and a low part, so k * ln2_hi is exact), then the
 * Taylor series of exp(r) to degree 13 by Horner's rule, scaled by 2^-k. */
double crb_ref_expneg(double x)
{
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    const double inv_ln2 = 1.44269504088896338700e+00;
    double y = -x;
    double kf = floor(y * inv_ln2 + 0.5);
    double r = (y - kf * ln2_hi) - kf * ln2_lo;
    double p = 1.0 / 6227020800.0;                   /* 1/13! */
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)kf);
}

int crb_ref_poisson(const float *in, long long n, unsigned long long seed, float *out)
{
    if (!in || !out || n < 0)
        return -1;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (long long i = 0; i < n; ++i) {
        double mean = (double)in[i];
        if (!(mean > 0.0))
            mean = 0.0;           /* also maps NaN to 0 */
        if (mean > 500.0)
            mean = 500.0;
        const double limit = crb_ref_expneg(mean);
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((unsigned long long)i >> 32), 0, 0};
        uint32_t words[4];
        long long k = 0;
        double prod = 1.0;
        for (uint32_t j = 0;; ++j) {
            if (j % 4 == 0) {
                ctr[2] = j / 4;
                crb_ref_philox4x32_10(ctr, key, words);
            }
            const double u = ((double)words[j % 4] + 0.5) * (1.0 / 4294967296.0);
            prod = prod * u;
            if (!(prod > limit))
                break;
            ++k;
        }
        out[i] = (float)k;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* SOURCES work function (test infrastructure, as above)                      */
/* ------------------------------------------------------------------------- */

/* Is q = (yq, xq) allowed to sit beside the peak candidate p = (y, x) of value v?
 * Only a smaller value, or an equal value later in raster order. */
static int yields_to(float vq, int yq, int xq, float v, int y, int x)
{
    if (vq < v)
        return 1;
    if (vq == v)
        return yq > y || (yq == y && xq > x);
    return 0;
}

int crb_ref_sources(const float *in, int H, int W, float threshold, float sky, int r, int a,
                    crb_ref_source *out, long long capacity, long long *count)
{
    if (!in || !count || H < 1 || W < 1 || r < 1 || r > 8 || a < 0 || a > 8 ||
        capacity < 0 || (capacity > 0 && !out) || !isfinite(threshold) || !isfinite(sky))
        return -1;
    long long found = 0;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const float v = in[(size_t)y * W + x];
            if (!(v > threshold))
                continue;
            int peak = 1;
            for (int yq = y - r; yq <= y + r && peak; ++yq) {
                if (yq < 0 || yq >= H)
                    continue;
                for (int xq = x - r; xq <= x + r; ++xq) {
                    if (xq < 0 || xq >= W || (yq == y && xq == x))
                        continue;
                    if (!yields_to(in[(size_t)yq * W + xq], yq, xq, v, y, x)) {
                        peak = 0;
                        break;
                    }
                }
            }
            if (!peak)
                continue;
            if (found < capacity) {
                crb_ref_source rec;
                rec.y = y;
                rec.x = x;
                rec.peak = v;
                rec.npix = 0;
                rec.flux = 0.0;
                rec.sy = 0.0;
                rec.sx = 0.0;
                for (int dy = -a; dy <= a; ++dy) {
                    if (y + dy < 0 || y + dy >= H)
                        continue;
                    for (int dx = -a; dx <= a; ++dx) {
                        if (x + dx < 0 || x + dx >= W)
                            continue;
                        const double d = (double)in[(size_t)(y + dy) * W + (x + dx)] - (double)sky;
                        rec.flux = rec.flux + d;
                        rec.sy = rec.sy + (double)dy * d;
                        rec.sx = rec.sx + (double)dx * d;
                        rec.npix += 1;
                    }
                }
                out[found] = rec;
            }
            ++found;
        }
    }
    *count = found;
    return 0;
}
