/*
 * crb_ref.h -- plain single-threaded FP64 L.A.Cosmic oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference that the
 * GPU library is checked against; it shares no code with it.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * It computes, slowly and literally, the per-iteration cosmic-ray detection and
 * cleaning pass that CRBLASTER distributes over subimages (Mighell, Section 5:
 * L.A.Cosmic, "a variation of Laplacian edge detection", iterated up to about
 * four times; parameters gain, read noise, sigfrac, objlim).  The paper defers
 * the equations to van Dokkum (2001), which is not quoted here; the step list
 * and the readings of silent points are recorded at each function.
 *
 * Conventions shared by every function:
 *   - images are row-major H x W arrays, pitch W;
 *   - every stencil reads clamped indices c(i,n) = min(max(i,0),n-1)
 *     (the paper leaves the outer pixels undefined, Section 6.1);
 *   - all arithmetic is IEEE binary64, evaluated in the order written in the
 *     source, with no contraction into fused multiply-adds;
 *   - median windows are (2r+1)^2 multisets of clamped neighbours; an odd count
 *     takes the middle order statistic, an even count the mean of the two
 *     middle values.
 * Return values: 0 on success, -1 on invalid arguments, -2 on allocation failure.
 */
#ifndef CRB_REF_H
#define CRB_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double gain;       /* electrons per ADU, > 0                               */
    double readnoise;  /* electrons, >= 0                                      */
    double sky;        /* sky level already subtracted from the frame, ADU     */
    double sigclip;    /* detection limit on S' (in sigma), > 0                */
    double sigfrac;    /* fractional limit for neighbouring pixels, in [0, 1]  */
    double objlim;     /* contrast limit between hits and objects, > 0         */
} crb_ref_params;

/* Per-iteration intermediate planes; every pointer may be NULL (not written). */
typedef struct {
    double  *lplus;    /* L+ : clipped 2x-subsampled Laplacian, rebinned        */
    double  *noise;    /* N  : noise model from the 5x5 median                  */
    double  *s;        /* S  = L+ / (2 N)                                       */
    double  *sprime;   /* S' = S - med5(S)                                      */
    double  *fhat;     /* F^ = max((med3 - med7(med3)) / N, 0.01)               */
    uint8_t *first;    /* first selection A                                     */
    uint8_t *g1;       /* after the first neighbour grow                        */
    uint8_t *g2;       /* after the second neighbour grow                       */
} crb_ref_trace;

/* Median filter with a (2r+1)x(2r+1) clamped window; r >= 0. */
int crb_ref_median_filter(const double *in, int H, int W, int r, double *out);

/* L+ by the literal route: replicate each pixel into a 2x2 block, convolve the
 * 2H x 2W grid with the 4-neighbour Laplacian [[0,-1,0],[-1,4,-1],[0,-1,0]]
 * (clamped on the 2x grid), set negative values to zero, average each 2x2 block. */
int crb_ref_lplus(const double *J, int H, int W, double *out);

/* One iteration k: input J_k (H x W) and cumulative mask M_{k-1} (0/1 bytes).
 * Writes G2 (newly selected set of this iteration), M_k = M_{k-1} | G2,
 * J_{k+1} and n_k = #(G2 & !M_{k-1}).  Any output pointer may be NULL.
 * out_Jnext must not alias J. */
int crb_ref_iterate(const double *J, const uint8_t *Mprev, int H, int W,
                    const crb_ref_params *p, uint8_t *out_G2, uint8_t *out_M,
                    double *out_Jnext, long long *out_nnew, crb_ref_trace *trace);

/* Full run: up to niter iterations from the FP32 frame img.  With early_stop != 0
 * the loop ends after the first iteration whose n_k is zero.  out_clean is the
 * last J (FP64), out_mask the last M.  out_iters (nullable) receives the number
 * of iterations executed; out_counts (nullable, niter entries) receives n_k. */
int crb_ref_lacosmic(const float *img, int H, int W, const crb_ref_params *p,
                     int niter, int early_stop, double *out_clean, uint8_t *out_mask,
                     int *out_iters, long long *out_counts);

/* ---- POISSON work function (the paper's framework probe, Section 6.3.2) ----
 * out[i] = a Poisson deviate with mean in[i], drawn by Knuth's multiplication
 * method: multiply uniforms until the product falls to exp(-mean) or below; the
 * count of factors minus one is the deviate.  Means are clamped to [0, 500]
 * (non-finite means give 0).  Uniform j of pixel i is
 * (x + 0.5) * 2^-32 for the 32-bit word x = Philox4x32-10(counter = (i_lo, i_hi,
 * j / 4, 0), key = (seed_lo, seed_hi)) word j % 4.  exp is computed by the
 * range-reduced polynomial in crb_ref_expneg (basic operations only, fixed order). */
void crb_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double crb_ref_expneg(double x);            /* exp(-x) for x in [0, 745] */
int crb_ref_poisson(const float *in, long long n, unsigned long long seed, float *out);

/* ---- SOURCES work function (the paper's example of a work function whose
 * actors return structures instead of subimages: stellar photometry, Section 7) --
 * A pixel p = (y, x) is a source when its value v exceeds `threshold` and, over
 * every other pixel q of the frame with |y'-y| <= r and |x'-x| <= r, either
 * in[q] < v, or in[q] == v and q comes after p in raster order (so a plateau of
 * equal values yields its first pixel).  The record holds the peak and aperture
 * sums over the in-frame pixels of the (2a+1)^2 box around p, in binary64,
 * accumulated row by row (dy = -a..a, then dx = -a..a):
 *   flux = sum (in[q] - sky),  sy = sum dy * (in[q] - sky),  sx = sum dx * (in[q] - sky),
 *   npix = number of in-frame aperture pixels.
 * Records come out in raster order of their peaks; at most `capacity` are written
 * and *count receives the total.  r in [1, 8], a in [0, 8], threshold and sky finite.
 * The dependency radius of this work function is max(r, a). */
typedef struct {
    int32_t y, x;
    float peak;
    int32_t npix;
    double flux, sy, sx;
} crb_ref_source;

int crb_ref_sources(const float *in, int H, int W, float threshold, float sky, int r, int a,
                    crb_ref_source *out, long long capacity, long long *count);

#ifdef __cplusplus
}
#endif
#endif /* CRB_REF_H */
