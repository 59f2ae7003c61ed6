/*
 * crb.h -- C ABI of libcrb, an MI355X (gfx950) implementation of the per-iteration
 * L.A.Cosmic cosmic-ray detection and cleaning pass that CRBLASTER distributes over
 * subimages (K. J. Mighell, "CRBLASTER: A Parallel-Processing Computational
 * Framework for Embarrassingly-Parallel Image-Analysis Algorithms", Section 5 for
 * the algorithm and its parameters gain, read noise, sigfrac and objlim; Section 6
 * for its use on subimages with overlapping borders).
 *
 * One iteration k on the image J_k with cumulative mask M_{k-1}:
 *   L+  = 2x2 mean of the clipped (>= 0) 4-neighbour Laplacian of the 2x
 *         block-replicated image;
 *   N   = sqrt(gain * m5 + readnoise^2) / gain with m5 = med5(J) + sky
 *         (m5 <= 0 is replaced by 1e-4);
 *   S   = L+ / (2 N),  S' = S - med5(S);
 *   F^  = max((med3(J) - med7(med3(J))) / N, 0.01);
 *   A   = [S' > sigclip] and [S' / F^ > objlim];
 *   G1  = dilate3x3(A) and [S' > sigclip];
 *   G2  = dilate3x3(G1) and [S' > sigfrac * sigclip];
 *   n_k = #(G2 and not M_{k-1});  M_k = M_{k-1} or G2;
 *   J_{k+1}(p) = median of the unflagged J_k in the 5x5 window of p, for p in M_k
 *         (even count: mean of the two middle values; no unflagged pixel: J_k(p)).
 * Every stencil reads clamped ("nearest") indices; the paper leaves the outer
 * pixels undefined (Section 6.1).  The loop runs up to niter iterations (the paper:
 * typically 4) and, unless disabled, stops after the first iteration with n_k = 0,
 * which is result-neutral because that iteration reproduces its input.
 *
 * Numerics: pixels are FP32.  Medians are exact selections.  Every detection
 * decision (the three threshold tests and the contrast test) is the one that L+, N,
 * S, S' and F^ evaluated in IEEE binary64 in the definition's operation order would
 * take (the paper's subimage data are doubles, Section 6.2): the kernels decide from
 * an FP32 estimate of S where a proven error bound shows that binary64 decides the
 * same way, and evaluate the statistics in binary64 where it does not.  So the
 * decisions for a given J_k do not depend on tiling, launch shape or rounding order.
 * A replaced pixel with an even number of unflagged neighbours receives the binary64
 * mean of the two middle values rounded to FP32.
 *
 * Conventions for every entry point:
 *   - image pointers are DEVICE pointers on the current HIP device, row-major,
 *     contiguous, pitch == W; masks are uint8 0/1;
 *   - the caller owns every buffer it passes; the library owns only internal
 *     workspace (device memory it allocates and keeps per stream until
 *     crb_release_workspace or process exit);
 *   - calls are stream-ordered and asynchronous unless stated otherwise; the
 *     returned status covers argument validation and launch errors only;
 *   - on any status other than CRB_OK nothing has been enqueued, and
 *     crb_last_error() returns a message for the calling thread;
 *   - pixel values must be finite (unspecified output otherwise);
 *   - out_clean may equal img (in-place cleaning); partial overlap is not allowed;
 *   - calls are thread-safe; two calls on one stream from different threads are
 *     serialised by the library.
 */
#ifndef CRB_H
#define CRB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CRB_OK = 0,
    CRB_EINVAL = -1,   /* invalid argument (null pointer, size < 1, parameter out of range) */
    CRB_ENOMEM = -2,   /* device allocation failed                                          */
    CRB_EDEVICE = -3,  /* HIP runtime or launch error                                       */
    CRB_ETOOBIG = -4,  /* H * W exceeds 2^31 - 1 pixels                                     */
    CRB_EBUSY = -5     /* serving: no admission possible now (retry later)                  */
} crb_status;

/* crb_frame.flags */
#define CRB_FLAG_NO_EARLY_STOP 1   /* always run niter iterations */
/* From iteration 2 on, re-run the detection only on the tiles whose codes can change: a
 * code depends on J within Chebyshev distance 4 (Section 5: S reads J within 2 pixels
 * through med5(J) and L+, S' reads S within 2 more, F^ reads med3 within 3, and med3
 * reads J within 1), and an iteration changes J only where its replacement wrote a new
 * value; the other tiles keep their codes.  The results are identical to the full
 * re-run. */
#define CRB_FLAG_INCREMENTAL 2

/* Options for crb_set_option. */
#define CRB_OPT_EARLY_STOP 1       /* value 1 (default) or 0: early stop in crb_lacosmic */
#define CRB_OPT_INCREMENTAL 2      /* value 0 (default) or 1: CRB_FLAG_INCREMENTAL for
                                      crb_lacosmic and crb_lacosmic_partitioned */
/* Launch shapes of crb_lacosmic, crb_lacosmic_noalloc and crb_debug_* (see crb_tuning;
 * every shape gives identical results): */
#define CRB_OPT_TILE_H 3           /* detection tile rows: 16, 32 (default) or 64        */
#define CRB_OPT_FUSED 4            /* 0 (default) or 1: grow and replacement fused        */
#define CRB_OPT_GROW_H 5           /* first-iteration grow strip rows: 0 (default), 8, 16
                                      or 32                                              */

/*
 * Clean one frame (the method above).
 *   img        device, H*W FP32 input (read only unless out_clean == img)
 *   H, W       >= 1, H*W <= 2^31-1
 *   gain       electrons per ADU, > 0
 *   readnoise  electrons, >= 0
 *   sky        sky level already subtracted from img (ADU); enters the noise only
 *   sigclip    detection limit (> 0), sigfrac in [0, 1], objlim > 0
 *   niter      >= 0 (0 copies img and clears the mask)
 *   out_clean  device, H*W FP32 cleaned image
 *   out_mask   device, H*W uint8 cumulative mask
 * Runs on the calling thread's stream (crb_set_stream).  All parameters must be
 * finite.
 */
crb_status crb_lacosmic(const float *img, int32_t H, int32_t W, float gain, float readnoise,
                        float sky, float sigclip, float sigfrac, float objlim, int32_t niter,
                        float *out_clean, uint8_t *out_mask);

/*
 * crb_lacosmic for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * results (bit-identical to crb_lacosmic) and stream (crb_set_stream) as crb_lacosmic;
 * it calls no hipMalloc, hipFree or other allocating routine.  Its workspace is a fixed
 * device array of CRB_NOALLOC_MAX_WORKSPACE bytes inside the library, one per GPU,
 * held from the first call on that GPU until the process ends.  A frame whose
 * workspace (crb_workspace_bytes) exceeds it is rejected with CRB_ETOOBIG before
 * anything is enqueued; 4096 x 4096 fits.  Every call on one GPU uses that GPU's
 * array: calls that overlap on one GPU (two streams, or two threads with their own
 * streams) race on it and give undefined results, so order them (one stream, or an
 * event between them).  Each call resets the counters it reads, so a call never sees
 * the previous call's state.
 */
#define CRB_NOALLOC_MAX_WORKSPACE ((size_t)96 << 20)
crb_status crb_lacosmic_noalloc(const float *img, int32_t H, int32_t W, float gain,
                                float readnoise, float sky, float sigclip, float sigfrac,
                                float objlim, int32_t niter, float *out_clean,
                                uint8_t *out_mask);

/* One frame of a batch (host struct; pointers are device pointers). */
typedef struct {
    const float *img;     /* input  (device, H*W FP32)                           */
    float *out_clean;     /* output (device, H*W FP32); may equal img            */
    uint8_t *out_mask;    /* output (device, H*W uint8)                          */
    int32_t H, W;
    float gain, readnoise, sky, sigclip, sigfrac, objlim;
    int32_t niter;
    int32_t flags;        /* CRB_FLAG_*                                          */
    int32_t iters_run;    /* output: iterations executed                        */
    int32_t reserved;
    int64_t n_flagged;    /* output: pixels in the final mask                   */
} crb_frame;

/*
 * Clean n independent frames of any sizes in one batched pass (one launch per
 * stage and iteration over a (frame, tile) work list): the paper's subimages handed
 * to actors (Section 6.2), here whole frames of uneven size sharing each launch.
 * Each frame's outputs are bit-identical to a crb_lacosmic call with the same
 * parameters (Section 5 for the method).  Synchronous, unlike the other cleaning
 * calls: it writes the host fields iters_run and n_flagged of frames[] at completion
 * and frees its per-call workspace before returning, so it waits for the batch on
 * hip_stream (NULL: default stream).  The stream-ordered, asynchronous form is the
 * batch plan below (crb_plan_run, then crb_plan_stats for the per-frame results).
 */
crb_status crb_lacosmic_batched(crb_frame *frames, int32_t n, void *hip_stream);

/*
 * Batch plans: the batched pass prepared once (work lists, descriptor table,
 * workspace) and captured as a HIP graph, then replayed.  The frames' device
 * pointers and sizes are fixed by the plan; the pixel contents may change between
 * runs.  crb_plan_run is asynchronous on its stream; crb_plan_stats waits for the
 * stream and fills iters_run / n_flagged of frames (n entries, same order).
 */
typedef struct crb_plan crb_plan;
crb_status crb_plan_create(const crb_frame *frames, int32_t n, void *hip_stream,
                           int32_t use_graph, crb_plan **out_plan);
crb_status crb_plan_run(crb_plan *plan);
crb_status crb_plan_stats(crb_plan *plan, crb_frame *frames, int32_t n);
void crb_plan_destroy(crb_plan *plan);
/* Per-launch timing of a plan created without a graph: when enabled, every launch
 * of crb_plan_run is bracketed by a pair of HIP events on the plan's stream.
 * crb_plan_kernel_times waits for the recorded work and returns, per kernel class
 * (0 init, 1 detection, 2 grow/count, 3 replacement), the summed milliseconds and
 * the number of launches since timing was enabled (ms[4], launches[4]). */
crb_status crb_plan_set_timing(crb_plan *plan, int32_t enable);
crb_status crb_plan_kernel_times(crb_plan *plan, double *ms, int64_t *launches);
/* Work counters of the detection kernel (for roofline accounting).  The detection
 * evaluates med5(S), S' and the threshold bits only on its work set, the pixels
 * within 2 of a pixel with S > sigclip whose own S exceeds sigfrac * sigclip (taken
 * from an FP32 estimate of S widened by its error bound, so the set can hold a few
 * more pixels), and the fine-structure contrast test (S'/F^ > objlim, decided by
 * counting the med7 window of med3 against the test's switching value) only where
 * S' > sigclip.  A work-set pixel whose S' interval from the estimate straddles a
 * threshold is re-evaluated in binary64 from J.  With counting enabled every
 * detection launch adds, per frame, the size of its work set, its number of contrast
 * tests and its number of re-evaluations; crb_plan_set_counting (which waits for the
 * plan's stream) clears the counters, crb_plan_work_counts waits for the stream and
 * returns the totals over all frames since then: counts[0] work-set pixels,
 * counts[1] contrast tests, counts[2] binary64 re-evaluations, counts[3] pixels whose
 * med5(J) was selected exactly (counts has 4 elements).  med5(J) and the estimate of
 * S are needed only within 4 pixels of a pixel where S may exceed sigclip; the
 * detection finds those pixels from a cheap lower bound of med5(J) (S does not grow
 * with it) and selects med5(J) only in the 2 x 2 pixel cells that meet that
 * region. */
crb_status crb_plan_set_counting(crb_plan *plan, int32_t enable);
crb_status crb_plan_work_counts(crb_plan *plan, int64_t *counts);

/*
 * Launch shapes of a plan (the autotuner's search space).  The paper finds the cost of a
 * subimage set by its overlap with its neighbours and by the imbalance between subimages
 * (Section 6.3.1: a 6 x 6 split beats 1 x 36, and the slowest subimage sets the pace);
 * here the same trade-offs are the halo share of a tile or strip and how tiles are
 * handed to the compute units.  Every shape computes identical results.
 *   tile_h      detection tile rows, 16, 32 or 64 (64 columns; the halo is 4 rows and
 *               columns of J, 2 of S): taller tiles re-read less halo per pixel, shorter
 *               ones fit more blocks per compute unit;
 *   persistent  0: one block per (frame, tile); 1: about as many blocks as are resident
 *               at once, each taking tiles from 8 atomic ticket counters (one per XCD,
 *               each over a contiguous part of the tile list, a block helping the others
 *               once its part is used up), as CRBLASTER's actors take subimages;
 *   fused       0: grow/count, list prefix and replacement as three launches per
 *               iteration; 1: one launch, each 8-row strip recomputing its 2-row mask
 *               halo (rows its neighbours own) and replacing its own flagged pixels;
 *   grow_h      rows of a first-iteration grow strip when fused is 0 (8, 16 or 32; 0 =
 *               32 for batches), with a 2-row code halo above and below.
 * The default is {32, 0, 0, 0}.
 */
typedef struct {
    int32_t tile_h;
    int32_t persistent;
    int32_t fused;
    int32_t grow_h;
} crb_tuning;

/* Set or read a plan's launch shapes; set waits for the plan's stream and re-captures
 * a graph plan.  A plan starts with the tune cache's entry for its batch layout (below)
 * or with the default. */
crb_status crb_plan_set_tuning(crb_plan *plan, const crb_tuning *tuning);
crb_status crb_plan_get_tuning(crb_plan *plan, crb_tuning *tuning);

/*
 * Autotune a plan: time whole runs (median of reps runs each, HIP events on the plan's
 * stream, after one untimed run) first over the six detection shapes (tile_h x
 * persistent), then over the four grow shapes (three launches with grow_h 8, 16 or 32,
 * or fused) under the best detection shape, keep the fastest and apply it to the plan.
 * The runs write the frames' outputs, so no frame may be cleaned in place (out_clean
 * == img gives CRB_EINVAL).  With use_cache != 0 and an entry for the plan's batch
 * layout in the tune cache, that entry is applied without timing (then *ms and
 * *default_ms are -1).  The cache is the text file named by the environment variable
 * CRB_TUNE_CACHE (none if unset): each tuning appends a line keyed by the device
 * (architecture, compute units) and the frames' sizes, iteration counts and flags, and
 * crb_plan_create applies the last matching line.  Outputs (each nullable): best, the
 * median ms of a run with it and with the default shapes.  Synchronous.
 */
crb_status crb_plan_autotune(crb_plan *plan, int32_t reps, int32_t use_cache, crb_tuning *best,
                             double *ms, double *default_ms);

/*
 * The paper's partitioned run (Section 6.2): the frame is split into ny x nx
 * rectangles of nearly equal area (row and column bounds floor(H*i/ny),
 * floor(W*j/nx)), each extended by `border` pixels beyond every edge it shares with
 * another rectangle (clamped to the frame), and each extended subimage is cleaned as
 * an independent frame (its own clamped edges, niter iterations, early stop on)
 * in one batched pass; only the interiors are written to out_clean / out_mask.
 * With border >= 8 * niter the result equals crb_lacosmic's (an iteration's
 * dependency radius is 8 pixels); smaller borders show the subimage edge effects
 * the paper's 6-pixel border trades against overlap.  border = -1 takes the declared
 * radius of the cleaning pass, 8 * niter (crb_work_radius of CRB_WORK_LACOSMIC).
 * Synchronous on the calling thread's stream; allocates temporary device memory for
 * the subimages.
 *   ny, nx >= 1 with ny <= H and nx <= W; border >= -1; other arguments as crb_lacosmic.
 */
crb_status crb_lacosmic_partitioned(const float *img, int32_t H, int32_t W, float gain,
                                    float readnoise, float sky, float sigclip, float sigfrac,
                                    float objlim, int32_t niter, int32_t ny, int32_t nx,
                                    int32_t border, float *out_clean, uint8_t *out_mask);

/*
 * The tile farm (the paper's computational framework, Sections 6.3 and 7).  A work
 * function declares its dependency radius: how far from a pixel it reads (positions
 * outside the frame are never read), and so the border a partition into independent
 * subimages must give it.  The farm cuts the frame into tile_h x tile_w rectangles
 * and hands them to `workers` persistent actors through atomic tickets, as
 * CRBLASTER's director hands subimages to free actors; the whole frame is resident,
 * so an actor reads a tile's neighbourhood directly.  Work functions:
 *   CRB_WORK_LACOSMIC (radius query only): the cleaning pass; radius 8 * niter, the
 *     border independent subimages need to reproduce a whole-frame run (one iteration
 *     reaches 8 pixels: 4 for the detection statistics, 1 for each of the two grows,
 *     2 for the replacement window);
 *   CRB_WORK_POISSON (Section 6.3.2), image output, radius 0: out = a Poisson deviate
 *     with mean in (Knuth's multiplication method; mean clamped to [0, 500],
 *     non-finite -> 0; uniforms from Philox4x32-10 keyed by `seed`, counter = (pixel
 *     index, draw / 4); e^-mean by range reduction and a degree-13 polynomial),
 *     bit-identical to the oracle's crb_ref_poisson;
 *   CRB_WORK_WAITER (Section 6.3.3), image output, radius 0: waits in[i]
 *     microseconds per pixel (clamped to [0, 1e6]), out = in;
 *   CRB_WORK_SOURCES (Section 7: actors returning structures, e.g. stellar
 *     photometry), list output, radius max(peak_radius, aperture_radius): a pixel p
 *     of value v is a source when v > threshold and every other in-frame pixel q
 *     within Chebyshev distance peak_radius has in[q] < v, or in[q] == v and q later
 *     in raster order.  Its crb_source record holds p, v and binary64 sums over the
 *     in-frame pixels q of the (2a+1)^2 box around p (a = aperture_radius), taken row
 *     by row: flux = sum(in[q] - sky), sy = sum(dy * (in[q] - sky)),
 *     sx = sum(dx * (in[q] - sky)), npix = their count.  Pixel values must be finite.
 */
#define CRB_WORK_LACOSMIC 0
#define CRB_WORK_POISSON 1
#define CRB_WORK_WAITER 2
#define CRB_WORK_SOURCES 3

typedef struct {
    int32_t kind;              /* CRB_WORK_*                                        */
    int32_t niter;             /* LACOSMIC: iterations (radius query only), >= 0     */
    uint64_t seed;             /* POISSON: generator key                            */
    float threshold;           /* SOURCES: peak threshold, finite                   */
    float sky;                 /* SOURCES: level subtracted in the sums, finite     */
    int32_t peak_radius;       /* SOURCES: r in [1, 8]                              */
    int32_t aperture_radius;   /* SOURCES: a in [0, 8]                              */
} crb_work;                    /* 32 bytes */

typedef struct {
    int32_t y, x;              /* peak position                                     */
    float peak;                /* in[y, x]                                          */
    int32_t npix;              /* in-frame aperture pixels                          */
    double flux, sy, sx;       /* aperture sums (see CRB_WORK_SOURCES)              */
} crb_source;                  /* 40 bytes */

/* Declared dependency radius of the work function described by w, or -1 (with
 * crb_last_error set) if w is null or its parameters are invalid. */
int32_t crb_work_radius(const crb_work *w);

/*
 * Run a farm work function (POISSON, WAITER or SOURCES) over the H x W FP32 device
 * frame `in` with `workers` actors, each a wave of 64 lanes (four per workgroup);
 * workers in [1, 2^22]; tile_h, tile_w >= 1.  SOURCES passes every pixel through the
 * threshold and runs the peak test and the sums only on the pixels above it, a
 * wave's candidates compacted so that all its lanes share that work.
 *   Image kinds: out_image (device, H x W FP32; may equal in, must not partially
 *     overlap it); out_list and out_count must be null.
 *   SOURCES: out_count (device int64, 8-byte aligned) receives the number of sources;
 *     the first min(count, list_capacity) of them are written to out_list (device,
 *     8-byte aligned; null only when list_capacity is 0) in no particular order --
 *     sort by (y, x) for raster order; a count above list_capacity means the list
 *     was truncated and a rerun with a larger list returns all.  out_image must be null.
 * Tiles are handed out through 32 ticket counters, each over a contiguous range of
 * tiles, in runs of several tiles; an actor drains its own range first and then
 * helps with the others.  Asynchronous on the calling thread's stream; uses 32 bytes
 * of that stream's workspace, so calls on one stream are ordered and calls on
 * different streams are independent.
 */
crb_status crb_farm_run(const crb_work *w, const float *in, int32_t H, int32_t W,
                        int32_t workers, int32_t tile_h, int32_t tile_w, float *out_image,
                        crb_source *out_list, int64_t list_capacity, int64_t *out_count);

/* POISSON or WAITER on bands of band_rows full rows: crb_farm_run with tile_h =
 * band_rows and tile_w = W. */
crb_status crb_work_run(int32_t kind, const float *in, int32_t H, int32_t W, uint64_t seed,
                        int32_t workers, int32_t band_rows, float *out);

/* Per-thread stream used by crb_lacosmic (NULL: default stream). */
crb_status crb_set_stream(void *hip_stream);
/* Library-wide option (CRB_OPT_*). */
crb_status crb_set_option(int32_t key, int64_t value);
/* Message of the calling thread's last error ("" if none). */
const char *crb_last_error(void);
/* Device workspace a frame of H x W needs beyond its input and outputs (bytes). */
size_t crb_workspace_bytes(int32_t H, int32_t W);
/* Free the workspace cached for hip_stream (waits for the stream first). */
crb_status crb_release_workspace(void *hip_stream);

/*
 * Serving: continuous (iteration-level) batching of frames that arrive over time.
 * A server owns device memory up to hbm_budget bytes for admitted frames' state
 * (image, mask and workspace) and runs rounds: each round performs one iteration
 * for every admitted frame, so frames at different iterations share the GPU.
 * Frames leave after niter iterations or an early stop; their results are copied
 * to the caller's host buffers and a completion is reported.
 *   crb_server_submit: FP32 image, read when the request is admitted (it must stay
 *     valid and unchanged until the request completes), outputs written at
 *     completion; returns CRB_EBUSY when the request can never fit the budget.
 *     Requests wait in FIFO order until slots and memory allow.  The image and both
 *     outputs are all host memory or all device memory of the server's device
 *     (CRB_EINVAL otherwise).  Device buffers are copied on the device (the caller
 *     makes the input ready before submitting, e.g. by synchronizing its stream);
 *     page-locked host buffers (hipHostMalloc) are transferred directly; pageable ones
 *     pass through the server's pinned staging buffers.
 *   crb_server_poll: enqueue the next round when the previous one has finished,
 *     admit waiting requests, retire finished frames; never blocks.  Writes up to
 *     max_done completed request ids to done_ids and their latency (seconds from
 *     submit to completion) to done_latency; returns the count in *n_done.
 *   crb_server_pending: requests submitted and not yet retired.
 */
typedef struct crb_server crb_server;
crb_status crb_server_create(size_t hbm_budget, int32_t max_slots, crb_server **out);
crb_status crb_server_submit(crb_server *srv, const float *host_img, int32_t H, int32_t W,
                             float gain, float readnoise, float sky, float sigclip,
                             float sigfrac, float objlim, int32_t niter, float *host_clean,
                             uint8_t *host_mask, int64_t *out_id);
crb_status crb_server_poll(crb_server *srv, int64_t *done_ids, double *done_latency,
                           int32_t max_done, int32_t *n_done);
int32_t crb_server_pending(crb_server *srv);
void crb_server_destroy(crb_server *srv);

/* ---- entry points for parity tests ------------------------------------------ */

/*
 * Run exactly one iteration of the method (Section 5) on a given (J_k, M_{k-1}), for
 * teacher-forced parity tests: J (FP32) and M_prev (uint8 0/1) are H x W device
 * arrays; writes G2 (uint8, the pixels selected this iteration), M_k = M_{k-1} | G2,
 * J_{k+1} (FP32) and n_k = #(G2 & !M_{k-1}) (one device int64).  params supplies gain,
 * readnoise, sky, sigclip, sigfrac and objlim; its pointers, sizes, niter and flags are
 * ignored.  out_J_next must not alias J.  Stream-ordered and asynchronous on the
 * calling thread's stream (crb_set_stream); uses that stream's workspace.
 */
crb_status crb_debug_iterate(const float *J, const uint8_t *M_prev, int32_t H, int32_t W,
                             const crb_frame *params, uint8_t *out_G2, uint8_t *out_M,
                             float *out_J_next, int64_t *out_n_new);
/* Detection stage only: code = A | [S' > sigclip] << 1 | [S' > sigfrac sigclip] << 2
 * on the pixels within distance 2 (8-connected) of a pixel with S > sigclip; elsewhere
 * either 0 or that same code (the detection's work set may hold a few more pixels,
 * see crb_plan_work_counts).  The grow reads a code only through its two 3x3
 * dilations of A, and A lies inside {S' > sigclip}, which lies inside {S > sigclip};
 * so the codes equal the full definition wherever they can change G1 or G2. */
crb_status crb_debug_detect(const float *J, const crb_frame *params, uint8_t *out_codes);
/* As crb_debug_detect, with S' of every work-set pixel evaluated in binary64 from J
 * (the path the detection takes where the FP32 estimate cannot decide). */
crb_status crb_debug_detect_exact(const float *J, const crb_frame *params,
                                  uint8_t *out_codes);
/* The detection's FP32 estimate of S (Section 5: S = L+ / (2N)) and its error bound
 * at every pixel of J (device pointers, H x W each, no overlap): |out_s - S| <=
 * out_err, S being the binary64 value; out_s = out_err = +inf where the bound is not
 * established (then the detection decides in binary64). */
crb_status crb_debug_s_estimate(const float *J, const crb_frame *params, float *out_s,
                                float *out_err);
/* The detection's dense upper bound of S (Section 5: S = L+ / (2N)) at every pixel of J
 * (device pointers, H x W each, no overlap): out_u >= S, S being the binary64 value,
 * from a lower bound of med5(J) shared by 2 x 5 pixel tiles (aligned at the frame's
 * origin here); out_u = +inf where the bound's analysis does not hold.  The detection
 * evaluates the other statistics only near the pixels where out_u exceeds sigclip.
 * Runs on the calling thread's stream. */
crb_status crb_debug_s_bound(const float *J, const crb_frame *params, float *out_u);
/* Clamped (2r+1)^2 median filter, r in {1, 2, 3}, by the kernels' networks (3x3 by
 * sorted columns, 5x5 by the network for a 2 x 2 tile of outputs on even pairs of rows
 * and the one for a row of two outputs on odd pairs, 7x7 by the single-output one). */
crb_status crb_debug_median(const float *in, int32_t H, int32_t W, int32_t r, float *out);
/* Clamped 5x5 median filter of binary64 values by the single-output network that the
 * detection applies to its FP32 estimates of S (here on binary64 inputs). */
crb_status crb_debug_median5_f64(const double *in, int32_t H, int32_t W, double *out);
/* Copy n FP32 elements (device, no overlap) by 4-byte buffer loads and stores, the
 * access width with which the detection stages J: a kernel of known traffic (4n bytes
 * read, 4n written) that calibrates the HBM byte counters for that width.  Runs on the
 * calling thread's stream. */
crb_status crb_debug_copy_b32(const float *src, float *dst, int64_t n);
/* Elementwise binary64 sqrt(x) and x / y on the device (rounding checks). */
crb_status crb_debug_fp64(const double *x, const double *y, int32_t n, double *out_sqrt,
                          double *out_div);

#ifdef __cplusplus
}
#endif
#endif /* CRB_H */
