// Device-side frame descriptor and kernel launchers of libcrb (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace crb {

// Upper bound on iterations per frame (sizes the per-frame counters).
constexpr int kMaxIter = 1024;
// Detection tiles are kDetectTX = 64 columns by 16, 32 (default) or 64 rows, one block of
// 8 threads per row.  The per-tile records shared by detection, grow and replacement
// (where A occurs, the last iteration with a new flag, the incremental-detection stamps)
// live on a fixed grid of kSumTY x kSumTX summary tiles, whatever the detection tile.
constexpr int kDetectTX = 64;
constexpr int kDetectTYDefault = 32;
constexpr int kSumTY = 32;
constexpr int kSumTX = 64;
// ticket counters of one persistent detection launch (one per XCD), each on its own
// 128-byte line (kTicketStride words apart) so that the XCDs do not contend for one line
constexpr int kDetectQueues = 8;
constexpr int kTicketStride = 32;
constexpr int kTicketWords = kDetectQueues * kTicketStride;   // per launch
// Grow tile (outputs per wave: 62 groups of 16 pixels by kGrowTY rows).
constexpr int kGrowTY = 32;
constexpr int kGrowTYSmall = 8;     // strip height for single frames below 2^22 pixels and
                                    // for every frame after iteration 1
constexpr int kGrowTX = 992;
static_assert(kGrowTY % kGrowTYSmall == 0, "a grow strip splits into short strips");
constexpr int kThreads = 256;

// Kernel classes for per-launch timing (crb_plan_kernel_times order).
constexpr int kKindInit = 0, kKindDetect = 1, kKindGrow = 2, kKindReplace = 3;
constexpr int kNumKernelKinds = 4;

// DevFrame::flags bits.  kNoEarlyStop has the value of CRB_FLAG_NO_EARLY_STOP;
// kFreshMask: the mask is uninitialised before iteration 1, whose detection clears it.
// kCountWork: detection adds its work-set size, contrast-test count and number of
// binary64 re-evaluations to f.work[0..2].
// kExactDetect: detection evaluates S' of every work-set pixel in binary64 from J
// (parity tests of that path).
constexpr int kNoEarlyStop = 1;
constexpr int kFreshMask = 1 << 8;
constexpr int kCountWork = 1 << 9;
constexpr int kExactDetect = 1 << 10;
// kIncremental (the value of CRB_FLAG_INCREMENTAL): from iteration 2 on, detection
// re-evaluates only the tiles near a summary tile stamped in f.dirty with the previous
// iteration (replacement stamps the summary tiles whose codes can change); the others
// keep their codes, which the unchanged J determines.
constexpr int kIncremental = 2;
constexpr int kWorkCounters = 4;

// Everything a kernel needs to know about one frame.  All pointers are device
// pointers; J is the image being cleaned in place (out_clean).
struct DevFrame {
    const float *img;             // input frame (copied into J by the init kernel)
    float *J;                     // working / output image, H x W
    uint8_t *mask;                // cumulative mask, H x W (0/1)
    uint8_t *codes;               // detection codes, H x W (workspace)
    uint8_t *g2;                  // optional: selection of this iteration (debug), or null
    uint32_t *list;               // indices of flagged pixels, H x W capacity (workspace)
    unsigned long long *nnew;     // n_k per iteration [kMaxIter] (workspace)
    unsigned int *listlen;        // [0]: length of the flagged list, which holds the pixels of
                                  // the mask in the order they were flagged (workspace)
    unsigned long long *work;     // with kCountWork: kWorkCounters counters, or null
    // per summary tile, row-major (kIncremental): the last iteration (mod 256) whose
    // replacement changed J within 4 pixels of it, or null
    uint8_t *dirty;
    // 4 bytes per summary tile, row-major, written by detection (byte w for rows
    // 8w .. 8w+7): bit 0 some pixel of those rows has A (the first selection), bit 1 one
    // of the tile's first two rows, bit 2 one of its last two; the grow skips strips with
    // no A within its 2-pixel reach.  Or null
    uint8_t *tile_first;
    // per summary tile: the last iteration whose grow flagged a new pixel in it (the
    // replacement leaves alone pixels with no new flag within 2 pixels), or null
    unsigned int *tile_new;
    int H, W;
    float gain, readnoise, sky, sigclip, sigfrac, objlim;
    int niter;
    int flags;
    int k;                        // current iteration when a kernel is launched with k = 0
    int pad;
    // Detection constants, derived from the parameters above by derive_detect_consts (on
    // the host, in the operations the detection would otherwise repeat per tile): the
    // FP32 thresholds sigclip and sigfrac * sigclip widened and narrowed by 2^-20
    // relative, objlim by 2^-21, 1 / objlim; and the parameters of the FP32 estimate of S
    // (gain / 8, 1 / gain, readnoise^2, and whether gain lies in [2^-100, 2^100]).
    float sc_lo, sc_hi, ll_lo, ll_hi;
    float olim_lo, olim_hi, inv_olim;
    float g8, inv_gain, rn2f;
    int est_ok;
    int pad2;
};

// Fills the detection constants of f from its parameters (every DevFrame passes through
// it: make_devframe calls it).  Plain IEEE single-precision operations, each rounded
// once, as the device would evaluate them.
inline void derive_detect_consts(DevFrame &f) {
    const float ll = f.sigfrac * f.sigclip;
    f.sc_lo = f.sigclip * (1.0f - 0x1p-20f);
    f.sc_hi = f.sigclip * (1.0f + 0x1p-20f);
    f.ll_lo = ll * (1.0f - 0x1p-20f);
    f.ll_hi = ll * (1.0f + 0x1p-20f);
    f.olim_lo = f.objlim * (1.0f - 0x1p-21f);
    f.olim_hi = f.objlim * (1.0f + 0x1p-21f);
    f.inv_olim = 1.0f / f.objlim;
    f.g8 = f.gain * 0.125f;
    f.inv_gain = 1.0f / f.gain;
    f.rn2f = f.readnoise * f.readnoise;
    f.est_ok = (f.gain >= 0x1p-100f && f.gain <= 0x1p100f) ? 1 : 0;
    f.pad2 = 0;
}

struct TileRef {                  // one (frame, tile origin) work item
    int frame, y0, x0, pad;
};

// Clears the counters and the nticket launch tickets; for frames with niter == 0 also
// copies img into J and clears the mask (otherwise iteration 1 does both: detection
// copies img into J and, when kFreshMask is set, clears the mask).  max_pixels: the
// largest frame with niter == 0 (0 if none), which sizes the grid.
hipError_t launch_init(const DevFrame *d_frames, int nframes, const DevFrame &single,
                       size_t max_pixels, unsigned int *tickets, int nticket, hipStream_t s);

// How a pass is launched (the autotuner's choices; every choice gives identical
// results).  tile_h: detection tile rows (16, 32 or 64); persistent: detection by
// resident blocks taking tiles from ticket counters instead of one block per tile;
// fused: grow, count and replacement in one launch per iteration (each strip recomputes
// its 2-row mask halo) instead of grow, list prefix and replacement; grow_h: rows of a
// first-iteration grow strip of the three-launch path (8, 16 or 32).
struct LaunchCfg {
    int tile_h = kDetectTYDefault;
    int persistent = 0;
    int fused = 0;
    int grow_h = 0;          // 0: 32 for batches and large frames, 8 for small frames
};

// Detection (codes) for one frame (d_tiles == null: tiles over `single`) or a work list
// of (frame, tile) built for cfg.tile_h.  Persistent launches take kTicketWords zeroed
// words of ticket counters.
hipError_t launch_detect(const DevFrame *d_frames, const TileRef *d_tiles, int ntiles,
                         const DevFrame &single, int k, const LaunchCfg &cfg,
                         unsigned int *tickets, hipStream_t s);
// Number of detection tiles of an H x W frame at tile height tile_h.
inline int detect_tiles(int H, int W, int tile_h) {
    return ((H + tile_h - 1) / tile_h) * ((W + kDetectTX - 1) / kDetectTX);
}
// Two-stage grow, new-flag count, cumulative mask and flagged list; with cfg.fused (and
// no debug G2 plane) also the replacement, in one launch (then no list prefix and
// replacement launch follow).  d_tiles lists 32-row strips of kGrowTX columns.  fresh:
// every frame of the launch carries kFreshMask (then iteration 1 reads no mask rows; the
// frames without it are tested at run time either way).
hipError_t launch_grow(const DevFrame *d_frames, const TileRef *d_tiles, int ntiles,
                       const DevFrame &single, int k, bool fresh, const LaunchCfg &cfg,
                       hipStream_t s);
// Offsets of each frame's flagged list in one flat index space (batched path):
// d_prefix[i] = sum of the list lengths of frames before i; d_prefix[n] = total.
hipError_t launch_list_prefix(const DevFrame *d_frames, int nframes, int k,
                              unsigned int *d_prefix, hipStream_t s);
// Masked-median replacement of every pixel on the flagged lists (d_prefix from
// launch_list_prefix for a batch; null for `single`).
hipError_t launch_replace(const DevFrame *d_frames, int nframes, const unsigned int *d_prefix,
                          const DevFrame &single, int k, int grid, hipStream_t s);
// Per-frame (iters_run, n_flagged) into d_stats[2 * i].
hipError_t launch_stats(const DevFrame *d_frames, int nframes, long long *d_stats,
                        hipStream_t s);

// Serving rounds: per frame, n_k of the iteration f.k just run and the running total
// of flagged pixels, into d_stats[2 * i] and d_stats[2 * i + 1].
hipError_t launch_round_stats(const DevFrame *d_frames, int nframes, long long *d_stats,
                              hipStream_t s);

// Subimage of a frame: the extended rectangle [a0, a0+h) x [b0, b0+w) is copied into
// sub (pitch w); its interior [y0, y1) x [x0, x1) (image coordinates) is written back.
struct SubRect {
    float *sub_img;        // h x w copy of the extended rectangle
    float *sub_clean;      // h x w cleaned subimage
    uint8_t *sub_mask;     // h x w mask of the subimage
    int a0, b0, h, w;      // extended rectangle
    int y0, y1, x0, x1;    // interior
};
hipError_t launch_extract(const float *img, int W, const SubRect *d_subs, int nsub,
                          size_t max_pixels, hipStream_t s);
hipError_t launch_stitch(float *out_clean, uint8_t *out_mask, int W, const SubRect *d_subs,
                         int nsub, size_t max_pixels, hipStream_t s);

hipError_t launch_debug_median(const float *in, int H, int W, int r, float *out, hipStream_t s);
// FP32 estimate of S and its error bound at every pixel of one frame (the detection
// kernel's estimate, for parity tests of the bound).
hipError_t launch_debug_s_estimate(const DevFrame &f, float *out_s, float *out_err,
                                   hipStream_t s);
hipError_t launch_debug_median5_f64(const double *in, int H, int W, double *out,
                                   hipStream_t s);
// The detection's dense upper bound of S at every pixel of one frame (+inf where its
// analysis does not hold), for parity tests of the bound.
hipError_t launch_debug_s_bound(const DevFrame &f, float *out_u, hipStream_t s);
// n FP32 elements copied by 4-byte buffer loads and stores (counter calibration).
hipError_t launch_debug_copy_b32(const float *src, float *dst, long long n, hipStream_t s);
hipError_t launch_debug_fp64(const double *x, const double *y, int n, double *out_sqrt,
                             double *out_div, hipStream_t s);

}  // namespace crb
