// C ABI of libcrb: argument validation, per-stream workspace, single-frame and
// batched passes, graph-captured batch plans and the parity-test entry points.
// The serving loop lives in server.hip.
#include "api_internal.h"

#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace crb {

static thread_local std::string t_err;
static thread_local hipStream_t t_stream = nullptr;
static std::atomic<int> g_early_stop{1};
static std::atomic<int> g_incremental{0};

crb_status fail(crb_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_err = buf;
    return st;
}

crb_status ok() {
    t_err.clear();
    return CRB_OK;
}

// bit-level test: robust under any floating-point compilation flags
static bool finite32(float x) {
    uint32_t u;
    memcpy(&u, &x, sizeof(u));
    return ((u >> 23) & 0xffu) != 0xffu;
}

crb_status check_frame_args(int32_t H, int32_t W, float gain, float readnoise, float sky,
                            float sigclip, float sigfrac, float objlim, int32_t niter) {
    if (H < 1 || W < 1)
        return fail(CRB_EINVAL, "image size %d x %d: both must be >= 1", H, W);
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX)
        return fail(CRB_ETOOBIG, "image of %lld pixels exceeds 2^31-1", (long long)H * W);
    if (!finite32(gain) || !finite32(readnoise) || !finite32(sky) || !finite32(sigclip) ||
        !finite32(sigfrac) || !finite32(objlim))
        return fail(CRB_EINVAL, "parameters must be finite");
    if (!(gain > 0.0f))
        return fail(CRB_EINVAL, "gain must be > 0 (got %g)", (double)gain);
    if (!(readnoise >= 0.0f))
        return fail(CRB_EINVAL, "readnoise must be >= 0 (got %g)", (double)readnoise);
    if (!(sigclip > 0.0f))
        return fail(CRB_EINVAL, "sigclip must be > 0 (got %g)", (double)sigclip);
    if (!(sigfrac >= 0.0f && sigfrac <= 1.0f))
        return fail(CRB_EINVAL, "sigfrac must lie in [0, 1] (got %g)", (double)sigfrac);
    if (!(objlim > 0.0f))
        return fail(CRB_EINVAL, "objlim must be > 0 (got %g)", (double)objlim);
    if (niter < 0 || niter > kMaxIter)
        return fail(CRB_EINVAL, "niter must lie in [0, %d] (got %d)", kMaxIter, niter);
    return CRB_OK;
}

static bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

crb_status check_buffers(const float *img, const float *clean, const uint8_t *mask,
                         size_t npix) {
    if (!img || !clean || !mask)
        return fail(CRB_EINVAL, "null image, output or mask pointer");
    if (img != clean && ranges_overlap(img, npix * 4, clean, npix * 4))
        return fail(CRB_EINVAL, "out_clean partially overlaps img");
    if (ranges_overlap(mask, npix, img, npix * 4) || ranges_overlap(mask, npix, clean, npix * 4))
        return fail(CRB_EINVAL, "out_mask overlaps an image buffer");
    return CRB_OK;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

FrameWs ws_layout(int32_t H, int32_t W) {
    const size_t n = (size_t)H * (size_t)W;
    FrameWs L;
    L.codes = 0;
    L.list = align_up(L.codes + n, 256);
    L.nnew = align_up(L.list + 4 * n, 256);
    L.listlen = align_up(L.nnew + 8 * (size_t)kMaxIter, 256);
    L.dirty = align_up(L.listlen + 4 * (size_t)kMaxIter, 256);
    const size_t ntiles = (size_t)((H + kSumTY - 1) / kSumTY) *
                          (size_t)((W + kSumTX - 1) / kSumTX);
    L.tile_first = align_up(L.dirty + ntiles, 256);
    L.tile_new = align_up(L.tile_first + 4 * ntiles, 256);
    L.total = align_up(L.tile_new + 4 * ntiles, 256);
    return L;
}

DevFrame make_devframe(const float *img, float *J, uint8_t *mask, char *ws, const FrameWs &L,
                       int32_t H, int32_t W, float gain, float readnoise, float sky,
                       float sigclip, float sigfrac, float objlim, int32_t niter, int32_t flags) {
    DevFrame f;
    memset(&f, 0, sizeof(f));
    f.img = img;
    f.J = J;
    f.mask = mask;
    f.g2 = nullptr;
    if (ws) {      // without a workspace every workspace pointer stays null
        f.codes = reinterpret_cast<uint8_t *>(ws + L.codes);
        f.list = reinterpret_cast<uint32_t *>(ws + L.list);
        f.nnew = reinterpret_cast<unsigned long long *>(ws + L.nnew);
        f.listlen = reinterpret_cast<unsigned int *>(ws + L.listlen);
        f.dirty = reinterpret_cast<uint8_t *>(ws + L.dirty);
        f.tile_first = reinterpret_cast<uint8_t *>(ws + L.tile_first);
        f.tile_new = reinterpret_cast<unsigned int *>(ws + L.tile_new);
    }
    f.H = H;
    f.W = W;
    f.gain = gain;
    f.readnoise = readnoise;
    f.sky = sky;
    f.sigclip = sigclip;
    f.sigfrac = sigfrac;
    f.objlim = objlim;
    f.niter = niter;
    f.flags = flags;
    f.k = 0;
    derive_detect_consts(f);
    return f;
}

int replace_grid(size_t npix) {
    size_t g = npix / 4096;
    if (g < 1)
        g = 1;
    if (g > 2048)
        g = 2048;
    return (int)g;
}

crb_status hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess)
        return CRB_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(CRB_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(CRB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// per-(device, stream) workspace
// ---------------------------------------------------------------------------

struct Workspace {
    std::mutex mu;
    char *buf = nullptr;
    size_t cap = 0;
    int device = 0;
    hipStream_t stream = nullptr;
};

static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

static crb_status ws_get(hipStream_t s, Workspace **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_status(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto key = std::make_pair(dev, s);
    auto it = g_ws.find(key);
    if (it == g_ws.end()) {
        Workspace *w = new (std::nothrow) Workspace();
        if (!w)
            return fail(CRB_ENOMEM, "host allocation failed");
        w->device = dev;
        w->stream = s;
        it = g_ws.emplace(key, w).first;
    }
    *out = it->second;
    return CRB_OK;
}

// caller holds ws->mu
static crb_status ws_reserve(Workspace *ws, size_t bytes) {
    if (ws->cap >= bytes)
        return CRB_OK;
    if (ws->buf) {
        hipError_t e = hipStreamSynchronize(ws->stream);
        if (e != hipSuccess)
            return hip_status(e, "hipStreamSynchronize");
        (void)hipFree(ws->buf);
        ws->buf = nullptr;
        ws->cap = 0;
    }
    const size_t want = align_up(bytes, (size_t)1 << 20);
    hipError_t e = hipMalloc((void **)&ws->buf, want);
    if (e != hipSuccess) {
        ws->buf = nullptr;
        (void)hipGetLastError();
        return fail(CRB_ENOMEM, "workspace of %zu bytes: %s", want, hipGetErrorString(e));
    }
    ws->cap = want;
    return CRB_OK;
}

// launch shapes of the single-frame entry points (CRB_OPT_TILE_H, CRB_OPT_FUSED,
// CRB_OPT_GROW_H; every shape gives identical results)
static std::atomic<int> g_single_tile_h{kDetectTYDefault};
static std::atomic<int> g_single_fused{0};
static std::atomic<int> g_single_grow_h{0};

static LaunchCfg single_cfg() {
    LaunchCfg c;
    c.tile_h = g_single_tile_h.load();
    c.fused = g_single_fused.load();
    c.grow_h = g_single_grow_h.load();
    return c;
}

// enqueue niter iterations for one frame whose DevFrame is complete
static crb_status enqueue_single(const DevFrame &f, const LaunchCfg &cfg, hipStream_t s) {
    const size_t npix = (size_t)f.H * (size_t)f.W;
    const bool fused = cfg.fused && !f.g2;
    // the init kernel touches pixels only for niter == 0 (a copy); else just counters
    hipError_t e = launch_init(nullptr, 1, f, f.niter == 0 ? npix : 0, nullptr, 0, s);
    for (int k = 1; e == hipSuccess && k <= f.niter; ++k) {
        e = launch_detect(nullptr, nullptr, 0, f, k, cfg, nullptr, s);
        if (e == hipSuccess)
            e = launch_grow(nullptr, nullptr, 0, f, k, (f.flags & kFreshMask) != 0, cfg, s);
        if (e == hipSuccess && !fused)
            e = launch_replace(nullptr, 1, nullptr, f, k, replace_grid(npix), s);
    }
    return hip_status(e, "kernel launch");
}

// ---------------------------------------------------------------------------
// fixed device scratch of the allocation-free entry point
// ---------------------------------------------------------------------------

// Workspace of crb_lacosmic_noalloc: one array per device, loaded with the code object
// and held until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in for the symbol): it takes the
// device address from hipGetSymbolAddress, once per device, and uses that.
constexpr size_t kScratchBytes = CRB_NOALLOC_MAX_WORKSPACE;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_dev[kMaxScratchDevices];    // device address per device, or null

// Device address of the current device's scratch array (looked up on the first call on
// that device, with the device current).
static crb_status scratch_ptr(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_status(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(CRB_EDEVICE, "device %d beyond the %d the scratch table holds", dev,
                    kMaxScratchDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(CRB_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        }
        g_scratch_dev[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_dev[dev];
    return CRB_OK;
}

}  // namespace crb

using namespace crb;

extern "C" {

crb_status crb_set_stream(void *hip_stream) {
    t_stream = (hipStream_t)hip_stream;
    return ok();
}

crb_status crb_set_option(int32_t key, int64_t value) {
    if (key == CRB_OPT_EARLY_STOP) {
        if (value != 0 && value != 1)
            return fail(CRB_EINVAL, "CRB_OPT_EARLY_STOP takes 0 or 1");
        g_early_stop.store((int)value);
        return ok();
    }
    if (key == CRB_OPT_INCREMENTAL) {
        if (value != 0 && value != 1)
            return fail(CRB_EINVAL, "CRB_OPT_INCREMENTAL takes 0 or 1");
        g_incremental.store((int)value);
        return ok();
    }
    if (key == CRB_OPT_TILE_H) {
        if (value != 16 && value != 32 && value != 64)
            return fail(CRB_EINVAL, "CRB_OPT_TILE_H takes 16, 32 or 64");
        g_single_tile_h.store((int)value);
        return ok();
    }
    if (key == CRB_OPT_FUSED) {
        if (value != 0 && value != 1)
            return fail(CRB_EINVAL, "CRB_OPT_FUSED takes 0 or 1");
        g_single_fused.store((int)value);
        return ok();
    }
    if (key == CRB_OPT_GROW_H) {
        if (value != 0 && value != 8 && value != 16 && value != 32)
            return fail(CRB_EINVAL, "CRB_OPT_GROW_H takes 0, 8, 16 or 32");
        g_single_grow_h.store((int)value);
        return ok();
    }
    return fail(CRB_EINVAL, "unknown option %d", key);
}

const char *crb_last_error(void) { return t_err.c_str(); }

size_t crb_workspace_bytes(int32_t H, int32_t W) {
    if (H < 1 || W < 1)
        return 0;
    return ws_layout(H, W).total;
}

crb_status crb_release_workspace(void *hip_stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(CRB_EDEVICE, "no HIP device");
    Workspace *w = nullptr;
    {
        std::lock_guard<std::mutex> g(g_ws_mu);
        auto it = g_ws.find(std::make_pair(dev, (hipStream_t)hip_stream));
        if (it == g_ws.end())
            return ok();
        w = it->second;
    }
    std::lock_guard<std::mutex> g(w->mu);
    if (w->buf) {
        hipError_t e = hipStreamSynchronize(w->stream);
        if (e != hipSuccess)
            return hip_status(e, "hipStreamSynchronize");
        (void)hipFree(w->buf);
        w->buf = nullptr;
        w->cap = 0;
    }
    return ok();
}

crb_status crb_lacosmic_noalloc(const float *img, int32_t H, int32_t W, float gain,
                                float readnoise, float sky, float sigclip, float sigfrac,
                                float objlim, int32_t niter, float *out_clean,
                                uint8_t *out_mask) {
    crb_status st = check_frame_args(H, W, gain, readnoise, sky, sigclip, sigfrac, objlim, niter);
    if (st != CRB_OK)
        return st;
    const size_t npix = (size_t)H * (size_t)W;
    if ((st = check_buffers(img, out_clean, out_mask, npix)) != CRB_OK)
        return st;
    const FrameWs L = ws_layout(H, W);
    if (L.total > kScratchBytes)
        return fail(CRB_ETOOBIG,
                    "crb_lacosmic_noalloc: a %d x %d frame needs %zu bytes of workspace, above "
                    "the fixed scratch of %zu bytes (CRB_NOALLOC_MAX_WORKSPACE)",
                    H, W, L.total, kScratchBytes);
    char *base = nullptr;
    if ((st = scratch_ptr(&base)) != CRB_OK)
        return st;
    const int flags = (g_early_stop.load() ? 0 : kNoEarlyStop) |
                      (g_incremental.load() ? kIncremental : 0) | kFreshMask;
    DevFrame f = make_devframe(img, out_clean, out_mask, base, L, H, W, gain, readnoise, sky,
                               sigclip, sigfrac, objlim, niter, flags);
    if ((st = enqueue_single(f, single_cfg(), t_stream)) != CRB_OK)
        return st;
    return ok();
}

crb_status crb_lacosmic(const float *img, int32_t H, int32_t W, float gain, float readnoise,
                        float sky, float sigclip, float sigfrac, float objlim, int32_t niter,
                        float *out_clean, uint8_t *out_mask) {
    crb_status st = check_frame_args(H, W, gain, readnoise, sky, sigclip, sigfrac, objlim, niter);
    if (st != CRB_OK)
        return st;
    const size_t npix = (size_t)H * (size_t)W;
    if ((st = check_buffers(img, out_clean, out_mask, npix)) != CRB_OK)
        return st;
    hipStream_t s = t_stream;
    Workspace *ws = nullptr;
    if ((st = ws_get(s, &ws)) != CRB_OK)
        return st;
    std::lock_guard<std::mutex> g(ws->mu);
    const FrameWs L = ws_layout(H, W);
    if ((st = ws_reserve(ws, L.total)) != CRB_OK)
        return st;
    const int flags = (g_early_stop.load() ? 0 : kNoEarlyStop) |
                      (g_incremental.load() ? kIncremental : 0) | kFreshMask;
    DevFrame f = make_devframe(img, out_clean, out_mask, ws->buf, L, H, W, gain, readnoise, sky,
                               sigclip, sigfrac, objlim, niter, flags);
    if ((st = enqueue_single(f, single_cfg(), s)) != CRB_OK)
        return st;
    return ok();
}

static crb_status check_work(const crb_work *w, WorkArgs *args) {
    if (!w)
        return fail(CRB_EINVAL, "null work description");
    memset(args, 0, sizeof(*args));
    switch (w->kind) {
    case CRB_WORK_LACOSMIC:
        if (w->niter < 0 || w->niter > kMaxIter)
            return fail(CRB_EINVAL, "niter %d outside [0, %d]", w->niter, kMaxIter);
        return CRB_OK;
    case CRB_WORK_POISSON:
        args->seed = (unsigned long long)w->seed;
        return CRB_OK;
    case CRB_WORK_WAITER:
        return CRB_OK;
    case CRB_WORK_SOURCES:
        if (w->peak_radius < 1 || w->peak_radius > kMaxWorkRadius || w->aperture_radius < 0 ||
            w->aperture_radius > kMaxWorkRadius)
            return fail(CRB_EINVAL, "SOURCES radii r = %d, a = %d: need 1 <= r <= %d, 0 <= a <= %d",
                        w->peak_radius, w->aperture_radius, kMaxWorkRadius, kMaxWorkRadius);
        if (!finite32(w->threshold) || !finite32(w->sky))
            return fail(CRB_EINVAL, "SOURCES threshold and sky must be finite");
        args->threshold = w->threshold;
        args->sky = w->sky;
        args->r = w->peak_radius;
        args->a = w->aperture_radius;
        return CRB_OK;
    default:
        return fail(CRB_EINVAL, "unknown work function %d", w->kind);
    }
}

int32_t crb_work_radius(const crb_work *w) {
    WorkArgs args;
    if (check_work(w, &args) != CRB_OK)
        return -1;
    ok();
    return work_radius(w->kind, args, w->niter);
}

crb_status crb_farm_run(const crb_work *w, const float *in, int32_t H, int32_t W,
                        int32_t workers, int32_t tile_h, int32_t tile_w, float *out_image,
                        crb_source *out_list, int64_t list_capacity, int64_t *out_count) {
    WorkArgs args;
    crb_status st = check_work(w, &args);
    if (st != CRB_OK)
        return st;
    if (w->kind == CRB_WORK_LACOSMIC)
        return fail(CRB_EINVAL, "the cleaning pass runs through crb_lacosmic*, not the farm");
    if (!in)
        return fail(CRB_EINVAL, "null pointer");
    if (H < 1 || W < 1)
        return fail(CRB_EINVAL, "image size %d x %d: both must be >= 1", H, W);
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX)
        return fail(CRB_ETOOBIG, "image exceeds 2^31-1 pixels");
    if (workers < 1 || workers > (1 << 22) || tile_h < 1 || tile_w < 1)
        return fail(CRB_EINVAL, "workers must lie in [1, 2^22] and tiles be at least 1 x 1");
    const size_t nbytes = (size_t)H * (size_t)W * 4;
    const bool list = w->kind == CRB_WORK_SOURCES;
    if (list) {
        if (out_image)
            return fail(CRB_EINVAL, "SOURCES writes a list: out_image must be null");
        if (!out_count || ((uintptr_t)out_count & 7))
            return fail(CRB_EINVAL, "out_count must be an 8-byte aligned device pointer");
        if (list_capacity < 0 || (list_capacity > 0 && (!out_list || ((uintptr_t)out_list & 7))))
            return fail(CRB_EINVAL, "out_list must be 8-byte aligned and hold list_capacity >= 0 "
                                    "records");
        const size_t lbytes = (size_t)list_capacity * sizeof(crb_source);
        if (list_capacity > 0 && (ranges_overlap(out_list, lbytes, in, nbytes) ||
                                  ranges_overlap(out_list, lbytes, out_count, 8)))
            return fail(CRB_EINVAL, "out_list overlaps the frame or the count");
        if (ranges_overlap(out_count, 8, in, nbytes))
            return fail(CRB_EINVAL, "out_count overlaps the frame");
    } else {
        if (!out_image)
            return fail(CRB_EINVAL, "null out_image");
        if (out_list || out_count)
            return fail(CRB_EINVAL, "image work functions take no out_list / out_count");
        if (in != out_image && ranges_overlap(in, nbytes, out_image, nbytes))
            return fail(CRB_EINVAL, "out_image partially overlaps in");
    }
    WorkArgs a2 = args;
    if (w->kind == CRB_WORK_WAITER) {
        int dev = 0, khz = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess)
            return hip_status(e, "device query");
        a2.wall_khz = khz;
    }
    hipStream_t s = t_stream;
    Workspace *ws = nullptr;
    if ((st = ws_get(s, &ws)) != CRB_OK)
        return st;
    std::lock_guard<std::mutex> g(ws->mu);
    if ((st = ws_reserve(ws, 256)) != CRB_OK)
        return st;
    unsigned int *tickets = reinterpret_cast<unsigned int *>(ws->buf);
    unsigned long long *count = reinterpret_cast<unsigned long long *>(out_count);
    hipError_t e = launch_farm_reset(tickets, count, s);
    if (e == hipSuccess)
        e = launch_farm(w->kind, a2, in, H, W, workers, tile_h, tile_w, out_image,
                        reinterpret_cast<SourceRec *>(out_list), (long long)list_capacity, count,
                        tickets, s);
    st = hip_status(e, "kernel launch");
    return st == CRB_OK ? ok() : st;
}

crb_status crb_work_run(int32_t kind, const float *in, int32_t H, int32_t W, uint64_t seed,
                        int32_t workers, int32_t band_rows, float *out) {
    if (kind != CRB_WORK_POISSON && kind != CRB_WORK_WAITER)
        return fail(CRB_EINVAL, "crb_work_run takes POISSON or WAITER, not %d", kind);
    crb_work w;
    memset(&w, 0, sizeof(w));
    w.kind = kind;
    w.seed = seed;
    return crb_farm_run(&w, in, H, W, workers, band_rows, W, out, nullptr, 0, nullptr);
}

crb_status crb_debug_iterate(const float *J, const uint8_t *M_prev, int32_t H, int32_t W,
                             const crb_frame *p, uint8_t *out_G2, uint8_t *out_M,
                             float *out_J_next, int64_t *out_n_new) {
    if (!p)
        return fail(CRB_EINVAL, "null params");
    crb_status st = check_frame_args(H, W, p->gain, p->readnoise, p->sky, p->sigclip,
                                     p->sigfrac, p->objlim, 1);
    if (st != CRB_OK)
        return st;
    const size_t npix = (size_t)H * (size_t)W;
    if (!J || !M_prev || !out_G2 || !out_M || !out_J_next || !out_n_new)
        return fail(CRB_EINVAL, "null pointer");
    if (J == out_J_next)
        return fail(CRB_EINVAL, "out_J_next must not alias J");
    hipStream_t s = t_stream;
    Workspace *ws = nullptr;
    if ((st = ws_get(s, &ws)) != CRB_OK)
        return st;
    std::lock_guard<std::mutex> g(ws->mu);
    const FrameWs L = ws_layout(H, W);
    if ((st = ws_reserve(ws, L.total)) != CRB_OK)
        return st;
    DevFrame f = make_devframe(J, out_J_next, out_M, ws->buf, L, H, W, p->gain,
                               p->readnoise, p->sky, p->sigclip, p->sigfrac, p->objlim, 1,
                               kNoEarlyStop);
    f.g2 = out_G2;
    hipError_t e = hipMemcpyAsync(out_M, M_prev, npix, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
        return hip_status(e, "hipMemcpyAsync");
    if ((st = enqueue_single(f, single_cfg(), s)) != CRB_OK)
        return st;
    e = hipMemcpyAsync(out_n_new, f.nnew, sizeof(int64_t), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
        return hip_status(e, "hipMemcpyAsync");
    return ok();
}

static crb_status debug_detect(const float *J, const crb_frame *p, uint8_t *out_codes,
                               int flags) {
    if (!p || !J || !out_codes)
        return fail(CRB_EINVAL, "null pointer");
    crb_status st = check_frame_args(p->H, p->W, p->gain, p->readnoise, p->sky, p->sigclip,
                                     p->sigfrac, p->objlim, 1);
    if (st != CRB_OK)
        return st;
    DevFrame f = make_devframe(J, const_cast<float *>(J), nullptr, nullptr, ws_layout(1, 1),
                               p->H, p->W, p->gain, p->readnoise, p->sky, p->sigclip,
                               p->sigfrac, p->objlim, 1, kNoEarlyStop | flags);
    f.codes = out_codes;
    return hip_status(launch_detect(nullptr, nullptr, 0, f, 1, single_cfg(), nullptr, t_stream),
                      "kernel launch") == CRB_OK
               ? ok()
               : CRB_EDEVICE;
}

crb_status crb_debug_detect(const float *J, const crb_frame *p, uint8_t *out_codes) {
    return debug_detect(J, p, out_codes, 0);
}

crb_status crb_debug_detect_exact(const float *J, const crb_frame *p, uint8_t *out_codes) {
    return debug_detect(J, p, out_codes, kExactDetect);
}

crb_status crb_debug_s_estimate(const float *J, const crb_frame *p, float *out_s,
                                float *out_err) {
    if (!p || !J || !out_s || !out_err)
        return fail(CRB_EINVAL, "null pointer");
    crb_status st = check_frame_args(p->H, p->W, p->gain, p->readnoise, p->sky, p->sigclip,
                                     p->sigfrac, p->objlim, 1);
    if (st != CRB_OK)
        return st;
    const size_t bytes = (size_t)p->H * (size_t)p->W * 4;
    if (ranges_overlap(out_s, bytes, out_err, bytes) || ranges_overlap(J, bytes, out_s, bytes) ||
        ranges_overlap(J, bytes, out_err, bytes))
        return fail(CRB_EINVAL, "buffers overlap");
    DevFrame f = make_devframe(J, const_cast<float *>(J), nullptr, nullptr, ws_layout(1, 1),
                               p->H, p->W, p->gain, p->readnoise, p->sky, p->sigclip,
                               p->sigfrac, p->objlim, 1, kNoEarlyStop);
    st = hip_status(launch_debug_s_estimate(f, out_s, out_err, t_stream), "kernel launch");
    return st == CRB_OK ? ok() : st;
}

crb_status crb_debug_s_bound(const float *J, const crb_frame *p, float *out_u) {
    if (!p || !J || !out_u)
        return fail(CRB_EINVAL, "null pointer");
    crb_status st = check_frame_args(p->H, p->W, p->gain, p->readnoise, p->sky, p->sigclip,
                                     p->sigfrac, p->objlim, 1);
    if (st != CRB_OK)
        return st;
    const size_t bytes = (size_t)p->H * (size_t)p->W * 4;
    if (ranges_overlap(J, bytes, out_u, bytes))
        return fail(CRB_EINVAL, "buffers overlap");
    DevFrame f = make_devframe(J, const_cast<float *>(J), nullptr, nullptr, ws_layout(1, 1),
                               p->H, p->W, p->gain, p->readnoise, p->sky, p->sigclip,
                               p->sigfrac, p->objlim, 1, kNoEarlyStop);
    st = hip_status(launch_debug_s_bound(f, out_u, t_stream), "kernel launch");
    return st == CRB_OK ? ok() : st;
}

crb_status crb_debug_median(const float *in, int32_t H, int32_t W, int32_t r, float *out) {
    if (!in || !out)
        return fail(CRB_EINVAL, "null pointer");
    if (H < 1 || W < 1 || (int64_t)H * W > (int64_t)INT32_MAX)
        return fail(CRB_EINVAL, "bad size %d x %d", H, W);
    if (r < 1 || r > 3)
        return fail(CRB_EINVAL, "radius must be 1, 2 or 3");
    if (ranges_overlap(in, (size_t)H * W * 4, out, (size_t)H * W * 4))
        return fail(CRB_EINVAL, "in and out overlap");
    crb_status st = hip_status(launch_debug_median(in, H, W, r, out, t_stream), "kernel launch");
    return st == CRB_OK ? ok() : st;
}

crb_status crb_debug_median5_f64(const double *in, int32_t H, int32_t W, double *out) {
    if (!in || !out)
        return fail(CRB_EINVAL, "null pointer");
    if (H < 1 || W < 1 || (int64_t)H * W > (int64_t)INT32_MAX)
        return fail(CRB_EINVAL, "bad size %d x %d", H, W);
    if (ranges_overlap(in, (size_t)H * W * 8, out, (size_t)H * W * 8))
        return fail(CRB_EINVAL, "in and out overlap");
    crb_status st = hip_status(launch_debug_median5_f64(in, H, W, out, t_stream), "kernel launch");
    return st == CRB_OK ? ok() : st;
}

crb_status crb_debug_copy_b32(const float *src, float *dst, int64_t n) {
    if (!src || !dst || n < 0)
        return fail(CRB_EINVAL, "bad arguments");
    if (ranges_overlap(src, (size_t)n * 4, dst, (size_t)n * 4))
        return fail(CRB_EINVAL, "src and dst overlap");
    crb_status st = hip_status(launch_debug_copy_b32(src, dst, (long long)n, t_stream),
                               "kernel launch");
    return st == CRB_OK ? ok() : st;
}

crb_status crb_debug_fp64(const double *x, const double *y, int32_t n, double *out_sqrt,
                          double *out_div) {
    if (!x || !y || !out_sqrt || !out_div || n < 0)
        return fail(CRB_EINVAL, "bad arguments");
    if (n == 0)
        return ok();
    crb_status st =
        hip_status(launch_debug_fp64(x, y, n, out_sqrt, out_div, t_stream), "kernel launch");
    return st == CRB_OK ? ok() : st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batch plans
// ---------------------------------------------------------------------------

namespace crb {
// detection tile heights a plan lists its tiles for
constexpr int kTileHeights[3] = {16, 32, 64};
static int tile_h_index(int h) { return h == 16 ? 0 : (h == 32 ? 1 : (h == 64 ? 2 : -1)); }
}  // namespace crb

struct crb_plan {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n = 0;
    int kmax = 0;
    size_t max_pix = 0;
    size_t init_pix = 0;                // largest frame with niter == 0 (0 if none)
    size_t all_pix = 0;
    char *dmem = nullptr;
    DevFrame *d_frames = nullptr;
    TileRef *d_tdet[3] = {nullptr, nullptr, nullptr};   // per detection tile height
    int ntdet[3] = {0, 0, 0};
    TileRef *d_tgrow = nullptr;
    int ntgrow = 0;
    long long *d_stats = nullptr;
    unsigned int *d_prefix = nullptr;   // flat offsets of the frames' flagged lists
    unsigned long long *d_work = nullptr;   // per frame: kWorkCounters detection counters
    unsigned int *d_tickets = nullptr;  // kTicketWords per iteration (persistent detection)
    std::vector<DevFrame> hframes;      // host copy of the frame table
    std::string key;                    // tune-cache key of the batch layout
    crb::LaunchCfg cfg;                 // launch shapes of crb_plan_run
    bool counting = false;
    int rgrid = 1;
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // eager timing: an event pair around every launch, summed per kernel class
    bool timing = false;
    std::vector<hipEvent_t> events;     // pool, 2 per recorded launch
    std::vector<int> ev_kind;           // kernel class of each recorded pair
    size_t ev_used = 0;                 // pairs recorded since the last query
    double acc_ms[crb::kNumKernelKinds] = {0};
    long long acc_n[crb::kNumKernelKinds] = {0};
};

namespace crb {

// records the start event of a timed launch (no-op unless timing)
static hipError_t tmark_begin(crb_plan *p, int kind) {
    if (!p->timing)
        return hipSuccess;
    if (2 * (p->ev_used + 1) > p->events.size()) {
        for (int i = 0; i < 2; ++i) {
            hipEvent_t ev;
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess)
                return e;
            p->events.push_back(ev);
        }
        p->ev_kind.push_back(0);
    }
    p->ev_kind[p->ev_used] = kind;
    return hipEventRecord(p->events[2 * p->ev_used], p->stream);
}

static hipError_t tmark_end(crb_plan *p) {
    if (!p->timing)
        return hipSuccess;
    hipError_t e = hipEventRecord(p->events[2 * p->ev_used + 1], p->stream);
    ++p->ev_used;
    return e;
}

static crb_status plan_enqueue(crb_plan *p) {
    hipStream_t s = p->stream;
    DevFrame none;
    memset(&none, 0, sizeof(none));
    const LaunchCfg &cfg = p->cfg;
    const int ti = tile_h_index(cfg.tile_h);
    if (ti < 0)
        return fail(CRB_EINVAL, "detection tile height %d", cfg.tile_h);
    // A plan of one frame passes the frame by value to one-block-per-tile and per-strip
    // grids, as crb_lacosmic does (no work-list lookups, no list prefix), unless its
    // detection is persistent, which needs the tile list.
    if (p->n == 1 && !cfg.persistent) {
        const DevFrame &f = p->hframes[0];
        const size_t npix = (size_t)f.H * (size_t)f.W;
        hipError_t e = tmark_begin(p, kKindInit);
        if (e == hipSuccess)
            e = launch_init(nullptr, 1, f, p->init_pix, nullptr, 0, s);
        if (e == hipSuccess)
            e = tmark_end(p);
        for (int k = 1; e == hipSuccess && k <= p->kmax; ++k) {
            if ((e = tmark_begin(p, kKindDetect)) == hipSuccess &&
                (e = launch_detect(nullptr, nullptr, 0, f, k, cfg, nullptr, s)) == hipSuccess &&
                (e = tmark_end(p)) == hipSuccess &&
                (e = tmark_begin(p, kKindGrow)) == hipSuccess &&
                (e = launch_grow(nullptr, nullptr, 0, f, k, (f.flags & kFreshMask) != 0, cfg,
                                 s)) == hipSuccess &&
                (e = tmark_end(p)) == hipSuccess && !cfg.fused &&
                (e = tmark_begin(p, kKindReplace)) == hipSuccess &&
                (e = launch_replace(nullptr, 1, nullptr, f, k, replace_grid(npix), s)) ==
                    hipSuccess)
                e = tmark_end(p);
        }
        if (e == hipSuccess)
            e = launch_stats(p->d_frames, p->n, p->d_stats, s);
        return hip_status(e, "kernel launch");
    }
    hipError_t e = tmark_begin(p, kKindInit);
    if (e == hipSuccess)
        e = launch_init(p->d_frames, p->n, none, p->init_pix, p->d_tickets,
                        p->kmax * kTicketWords, s);
    if (e == hipSuccess)
        e = tmark_end(p);
    for (int k = 1; e == hipSuccess && k <= p->kmax; ++k) {
        if ((e = tmark_begin(p, kKindDetect)) == hipSuccess &&
            (e = launch_detect(p->d_frames, p->d_tdet[ti], p->ntdet[ti], none, k, cfg,
                               p->d_tickets + (size_t)(k - 1) * kTicketWords, s)) ==
                hipSuccess &&
            (e = tmark_end(p)) == hipSuccess &&
            (e = tmark_begin(p, kKindGrow)) == hipSuccess &&
            // every frame of a plan carries kFreshMask
            (e = launch_grow(p->d_frames, p->d_tgrow, p->ntgrow, none, k, true, cfg, s)) ==
                hipSuccess &&
            (e = tmark_end(p)) == hipSuccess && !cfg.fused &&
            (e = tmark_begin(p, kKindReplace)) == hipSuccess &&
            (e = launch_list_prefix(p->d_frames, p->n, k, p->d_prefix, s)) == hipSuccess &&
            (e = launch_replace(p->d_frames, p->n, p->d_prefix, none, k, p->rgrid, s)) ==
                hipSuccess)
            e = tmark_end(p);
    }
    if (e == hipSuccess)
        e = launch_stats(p->d_frames, p->n, p->d_stats, s);
    return hip_status(e, "kernel launch");
}

static void plan_drop_graph(crb_plan *p) {
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

// capture the plan's launches (with its current launch shapes) as a graph
static crb_status plan_capture(crb_plan *p) {
    plan_drop_graph(p);
    hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return hip_status(e, "hipStreamBeginCapture");
    const bool timing = p->timing;
    p->timing = false;
    crb_status st = plan_enqueue(p);
    p->timing = timing;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->stream, &g);
    if (st != CRB_OK || e != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return st != CRB_OK ? st : hip_status(e, "hipStreamEndCapture");
    }
    p->graph = g;
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        plan_drop_graph(p);
        return hip_status(e, "hipGraphInstantiate");
    }
    return CRB_OK;
}

static void plan_free(crb_plan *p) {
    if (!p)
        return;
    plan_drop_graph(p);
    if (p->dmem) {
        (void)hipStreamSynchronize(p->stream);
        (void)hipFree(p->dmem);
    }
    for (hipEvent_t ev : p->events)
        (void)hipEventDestroy(ev);
    if (p->own_stream && p->stream)
        (void)hipStreamDestroy(p->stream);
    delete p;
}

// ---- the tune cache ---------------------------------------------------------------
// A text file named by CRB_TUNE_CACHE, one line per batch layout:
//   crb-tune 1 <key> tile_h=<h> persistent=<0|1> fused=<0|1> grow_h=<h> ms=<t> default_ms=<t>
// The key names the device (architecture and compute units) and the frames' sizes,
// iteration counts and flags; the last line for a key wins.

static std::mutex g_tune_mu;

static std::string layout_key(const std::vector<DevFrame> &frames, int device) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    for (char &c : arch)
        if (c == ' ' || c == ':')
            c = '_';
    // FNV-1a over the frame shapes in order
    unsigned long long h = 1469598103934665603ull;
    long long px = 0;
    for (const DevFrame &f : frames) {
        const int v[4] = {f.H, f.W, f.niter, f.flags & (kNoEarlyStop | kIncremental)};
        for (int x : v)
            for (int b = 0; b < 4; ++b) {
                h ^= (unsigned long long)((x >> (8 * b)) & 0xFF);
                h *= 1099511628211ull;
            }
        px += (long long)f.H * f.W;
    }
    char buf[160];
    snprintf(buf, sizeof(buf), "%s/cu%d/n%zu/px%lld/%016llx", arch.c_str(), cus, frames.size(), px,
             h);
    return buf;
}

static bool cfg_valid(const LaunchCfg &c) {
    return tile_h_index(c.tile_h) >= 0 && (c.persistent == 0 || c.persistent == 1) &&
           (c.fused == 0 || c.fused == 1) &&
           (c.grow_h == 0 || c.grow_h == 8 || c.grow_h == 16 || c.grow_h == 32);
}

static bool tune_cache_lookup(const std::string &key, LaunchCfg *out) {
    const char *path = getenv("CRB_TUNE_CACHE");
    if (!path || !*path)
        return false;
    std::lock_guard<std::mutex> g(g_tune_mu);
    FILE *fp = fopen(path, "r");
    if (!fp)
        return false;
    char line[512], k[256];
    bool found = false;
    while (fgets(line, sizeof(line), fp)) {
        LaunchCfg c;
        int ver = 0;
        if (sscanf(line, "crb-tune %d %255s tile_h=%d persistent=%d fused=%d grow_h=%d", &ver, k,
                   &c.tile_h, &c.persistent, &c.fused, &c.grow_h) == 6 &&
            ver == 1 && key == k && cfg_valid(c)) {
            *out = c;
            found = true;
        }
    }
    fclose(fp);
    return found;
}

static void tune_cache_store(const std::string &key, const LaunchCfg &c, double ms,
                             double default_ms) {
    const char *path = getenv("CRB_TUNE_CACHE");
    if (!path || !*path)
        return;
    std::lock_guard<std::mutex> g(g_tune_mu);
    FILE *fp = fopen(path, "a");
    if (!fp)
        return;
    fprintf(fp, "crb-tune 1 %s tile_h=%d persistent=%d fused=%d grow_h=%d ms=%.4f default_ms=%.4f\n",
            key.c_str(), c.tile_h, c.persistent, c.fused, c.grow_h, ms, default_ms);
    fclose(fp);
}

static LaunchCfg cfg_from(const crb_tuning &t) {
    LaunchCfg c;
    c.tile_h = t.tile_h;
    c.persistent = t.persistent;
    c.fused = t.fused;
    c.grow_h = t.grow_h;
    return c;
}

static crb_tuning tuning_from(const LaunchCfg &c) {
    crb_tuning t;
    t.tile_h = c.tile_h;
    t.persistent = c.persistent;
    t.fused = c.fused;
    t.grow_h = c.grow_h;
    return t;
}

// apply launch shapes to a plan (re-capturing its graph, if it has one)
static crb_status plan_apply(crb_plan *p, const LaunchCfg &c) {
    if (!cfg_valid(c))
        return fail(CRB_EINVAL, "launch shapes tile_h=%d persistent=%d fused=%d grow_h=%d: need "
                                "tile_h in {16, 32, 64}, persistent and fused in {0, 1}, grow_h "
                                "in {0, 8, 16, 32}",
                    c.tile_h, c.persistent, c.fused, c.grow_h);
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess)
        return hip_status(e, "hipStreamSynchronize");
    p->cfg = c;
    return p->use_graph ? plan_capture(p) : CRB_OK;
}

// median wall time (ms) of `reps` runs of the plan's launches with shapes c, timed by HIP
// events on the plan's stream after one untimed run
static crb_status time_cfg(crb_plan *p, const LaunchCfg &c, int reps, hipEvent_t a,
                           hipEvent_t b, double *ms) {
    const LaunchCfg keep = p->cfg;
    const bool timing = p->timing;
    p->cfg = c;
    p->timing = false;
    std::vector<double> t;
    crb_status st = plan_enqueue(p);
    for (int r = 0; st == CRB_OK && r < reps; ++r) {
        hipError_t e = hipEventRecord(a, p->stream);
        if (e == hipSuccess)
            st = plan_enqueue(p);
        if (st == CRB_OK && e == hipSuccess)
            e = hipEventRecord(b, p->stream);
        if (st == CRB_OK && e == hipSuccess)
            e = hipEventSynchronize(b);
        float x = 0.0f;
        if (st == CRB_OK && e == hipSuccess)
            e = hipEventElapsedTime(&x, a, b);
        if (st == CRB_OK && e != hipSuccess)
            st = hip_status(e, "autotune timing");
        t.push_back((double)x);
    }
    p->cfg = keep;
    p->timing = timing;
    if (st != CRB_OK)
        return st;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return CRB_OK;
}

}  // namespace crb

extern "C" {

crb_status crb_plan_create(const crb_frame *frames, int32_t n, void *hip_stream,
                           int32_t use_graph, crb_plan **out_plan) {
    if (!out_plan)
        return fail(CRB_EINVAL, "null out_plan");
    *out_plan = nullptr;
    if (!frames || n < 1)
        return fail(CRB_EINVAL, "need at least one frame");
    crb_status st;
    std::vector<FrameWs> lay(n);
    std::vector<size_t> off(n);
    size_t total = 0, max_pix = 0, all_pix = 0, init_pix = 0;
    int kmax = 0;
    size_t ntdet[3] = {0, 0, 0}, ntgrow = 0;
    for (int i = 0; i < n; ++i) {
        const crb_frame &f = frames[i];
        st = check_frame_args(f.H, f.W, f.gain, f.readnoise, f.sky, f.sigclip, f.sigfrac,
                              f.objlim, f.niter);
        if (st != CRB_OK)
            return fail(st, "frame %d: %s", i, crb_last_error());
        const size_t npix = (size_t)f.H * (size_t)f.W;
        if ((st = check_buffers(f.img, f.out_clean, f.out_mask, npix)) != CRB_OK)
            return fail(st, "frame %d: %s", i, crb_last_error());
        lay[i] = ws_layout(f.H, f.W);
        off[i] = total;
        total += lay[i].total;
        max_pix = npix > max_pix ? npix : max_pix;
        if (f.niter == 0)      // the init kernel copies these frames
            init_pix = npix > init_pix ? npix : init_pix;
        all_pix += npix;
        kmax = f.niter > kmax ? f.niter : kmax;
        for (int t = 0; t < 3; ++t)
            ntdet[t] += (size_t)detect_tiles(f.H, f.W, kTileHeights[t]);
        ntgrow += (size_t)((f.H + kGrowTY - 1) / kGrowTY) * ((f.W + kGrowTX - 1) / kGrowTX);
    }
    if (ntdet[0] > (size_t)INT32_MAX || ntgrow > (size_t)INT32_MAX / (kGrowTY / kGrowTYSmall))
        return fail(CRB_ETOOBIG, "batch too large");
    // also guard against buffers shared between frames
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const size_t ni = (size_t)frames[i].H * frames[i].W, nj = (size_t)frames[j].H * frames[j].W;
            if (ranges_overlap(frames[i].out_clean, ni * 4, frames[j].out_clean, nj * 4) ||
                ranges_overlap(frames[i].out_mask, ni, frames[j].out_mask, nj) ||
                ranges_overlap(frames[i].out_clean, ni * 4, frames[j].img, nj * 4) ||
                ranges_overlap(frames[j].out_clean, nj * 4, frames[i].img, ni * 4))
                return fail(CRB_EINVAL, "frames %d and %d share output memory", i, j);
        }
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o_frames = total;
    size_t o_tdet[3];
    o_tdet[0] = o_frames + al(n * sizeof(DevFrame));
    o_tdet[1] = o_tdet[0] + al(ntdet[0] * sizeof(TileRef));
    o_tdet[2] = o_tdet[1] + al(ntdet[1] * sizeof(TileRef));
    const size_t o_tgrow = o_tdet[2] + al(ntdet[2] * sizeof(TileRef));
    const size_t o_stats = o_tgrow + al(ntgrow * sizeof(TileRef));
    const size_t o_prefix = o_stats + al(2 * n * sizeof(long long));
    const size_t o_work = o_prefix + al((n + 1) * sizeof(unsigned int));
    const size_t o_tickets = o_work + al(kWorkCounters * n * sizeof(unsigned long long));
    const size_t bytes = o_tickets + al((size_t)(kmax > 0 ? kmax : 1) * kTicketWords * 4);

    crb_plan *p = new (std::nothrow) crb_plan();
    if (!p)
        return fail(CRB_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_status(e, "hipGetDevice");
    }
    p->stream = (hipStream_t)hip_stream;
    if (!p->stream && use_graph) {
        e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete p;
            return hip_status(e, "hipStreamCreate");
        }
        p->own_stream = true;
    }
    e = hipMalloc((void **)&p->dmem, bytes);
    if (e != hipSuccess) {
        p->dmem = nullptr;
        plan_free(p);
        (void)hipGetLastError();
        return fail(CRB_ENOMEM, "batch workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    p->n = n;
    p->kmax = kmax;
    p->max_pix = max_pix;
    p->init_pix = init_pix;
    p->all_pix = all_pix;
    p->d_frames = reinterpret_cast<DevFrame *>(p->dmem + o_frames);
    for (int t = 0; t < 3; ++t) {
        p->d_tdet[t] = reinterpret_cast<TileRef *>(p->dmem + o_tdet[t]);
        p->ntdet[t] = (int)ntdet[t];
    }
    p->d_tgrow = reinterpret_cast<TileRef *>(p->dmem + o_tgrow);
    p->d_stats = reinterpret_cast<long long *>(p->dmem + o_stats);
    p->d_prefix = reinterpret_cast<unsigned int *>(p->dmem + o_prefix);
    p->d_work = reinterpret_cast<unsigned long long *>(p->dmem + o_work);
    p->d_tickets = reinterpret_cast<unsigned int *>(p->dmem + o_tickets);
    p->ntgrow = (int)ntgrow;

    std::vector<DevFrame> hf(n);
    std::vector<TileRef> td[3], tg;
    for (int t = 0; t < 3; ++t)
        td[t].reserve(ntdet[t]);
    tg.reserve(ntgrow);
    for (int i = 0; i < n; ++i) {
        const crb_frame &f = frames[i];
        hf[i] = make_devframe(f.img, f.out_clean, f.out_mask, p->dmem + off[i], lay[i], f.H, f.W,
                              f.gain, f.readnoise, f.sky, f.sigclip, f.sigfrac, f.objlim,
                              f.niter,
                              (f.flags & CRB_FLAG_NO_EARLY_STOP ? kNoEarlyStop : 0) |
                                  (f.flags & CRB_FLAG_INCREMENTAL ? kIncremental : 0) |
                                  kFreshMask);
        hf[i].work = p->d_work + kWorkCounters * (size_t)i;
        for (int t = 0; t < 3; ++t)
            for (int y = 0; y < f.H; y += kTileHeights[t])
                for (int x = 0; x < f.W; x += kDetectTX)
                    td[t].push_back(TileRef{i, y, x, 0});
        for (int y = 0; y < f.H; y += kGrowTY)
            for (int x = 0; x < f.W; x += kGrowTX)
                tg.push_back(TileRef{i, y, x, 0});
    }
    p->rgrid = replace_grid(all_pix);
    // launch shapes: the tune cache's entry for this layout, if any, else the defaults
    const char *cache = getenv("CRB_TUNE_CACHE");
    if (cache && *cache) {
        p->key = layout_key(hf, p->device);
        LaunchCfg cached;
        if (tune_cache_lookup(p->key, &cached))
            p->cfg = cached;
    }
    // Tables and counters are written on the plan's stream and waited for: a
    // null-stream copy or memset is not ordered before work on a non-blocking stream,
    // and a pageable copy may return before its data has landed.
    e = hipMemcpyAsync(p->d_frames, hf.data(), n * sizeof(DevFrame), hipMemcpyHostToDevice,
                       p->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(p->d_work, 0, kWorkCounters * (size_t)n * sizeof(unsigned long long),
                           p->stream);
    for (int t = 0; t < 3 && e == hipSuccess; ++t)
        e = hipMemcpyAsync(p->d_tdet[t], td[t].data(), td[t].size() * sizeof(TileRef),
                           hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_tgrow, tg.data(), tg.size() * sizeof(TileRef),
                           hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(p->stream);
    p->hframes = hf;
    if (e != hipSuccess) {
        plan_free(p);
        return hip_status(e, "hipMemcpy");
    }
    if (use_graph) {
        p->use_graph = true;
        if ((st = plan_capture(p)) != CRB_OK) {
            plan_free(p);
            return st;
        }
    }
    *out_plan = p;
    return ok();
}

crb_status crb_plan_run(crb_plan *p) {
    if (!p)
        return fail(CRB_EINVAL, "null plan");
    if (p->use_graph)
        return hip_status(hipGraphLaunch(p->exec, p->stream), "hipGraphLaunch") == CRB_OK
                   ? ok()
                   : CRB_EDEVICE;
    crb_status st = plan_enqueue(p);
    return st == CRB_OK ? ok() : st;
}

crb_status crb_plan_stats(crb_plan *p, crb_frame *frames, int32_t n) {
    if (!p || !frames || n != p->n)
        return fail(CRB_EINVAL, "plan/frames mismatch");
    std::vector<long long> st(2 * (size_t)n);
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess)
        e = hipMemcpy(st.data(), p->d_stats, st.size() * sizeof(long long), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_status(e, "stats copy");
    for (int i = 0; i < n; ++i) {
        frames[i].iters_run = (int32_t)st[2 * i];
        frames[i].n_flagged = (int64_t)st[2 * i + 1];
    }
    return ok();
}

void crb_plan_destroy(crb_plan *p) { plan_free(p); }

crb_status crb_plan_set_tuning(crb_plan *p, const crb_tuning *t) {
    if (!p || !t)
        return fail(CRB_EINVAL, "null argument");
    crb_status st = plan_apply(p, cfg_from(*t));
    return st == CRB_OK ? ok() : st;
}

crb_status crb_plan_get_tuning(crb_plan *p, crb_tuning *t) {
    if (!p || !t)
        return fail(CRB_EINVAL, "null argument");
    *t = tuning_from(p->cfg);
    return ok();
}

crb_status crb_plan_autotune(crb_plan *p, int32_t reps, int32_t use_cache, crb_tuning *best,
                             double *out_ms, double *out_default_ms) {
    if (!p)
        return fail(CRB_EINVAL, "null plan");
    if (reps < 1 || reps > 1000)
        return fail(CRB_EINVAL, "reps must lie in [1, 1000] (got %d)", reps);
    for (const DevFrame &f : p->hframes)
        if (f.img == f.J)
            return fail(CRB_EINVAL, "autotuning runs the batch several times: a frame cleaned "
                                    "in place (out_clean == img) would lose its input");
    if (p->key.empty())
        p->key = layout_key(p->hframes, p->device);
    LaunchCfg chosen;
    if (use_cache && tune_cache_lookup(p->key, &chosen)) {
        crb_status st = plan_apply(p, chosen);
        if (st != CRB_OK)
            return st;
        if (best)
            *best = tuning_from(chosen);
        if (out_ms)
            *out_ms = -1.0;
        if (out_default_ms)
            *out_default_ms = -1.0;
        return ok();
    }
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess)
        return hip_status(e, "hipStreamSynchronize");
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    if (e != hipSuccess) {
        if (a)
            (void)hipEventDestroy(a);
        return hip_status(e, "hipEventCreate");
    }
    // Stage 1: detection shapes (tile height x one block per tile or persistent) under
    // the default grow; stage 2: grow shapes (three launches with first-iteration strips
    // of 8, 16 or 32 rows, or the fused grow and replacement) under the best detection.
    // The two stages time whole runs; detection and grow touch disjoint launches, so
    // their choices combine.
    crb_status st = CRB_OK;
    const LaunchCfg def;
    double t_def = 0.0;
    st = time_cfg(p, def, reps, a, b, &t_def);
    LaunchCfg cur = def;
    double t_cur = t_def;
    for (int ti = 0; st == CRB_OK && ti < 3; ++ti)
        for (int pers = 0; st == CRB_OK && pers <= 1; ++pers) {
            LaunchCfg c = def;
            c.tile_h = kTileHeights[ti];
            c.persistent = pers;
            if (c.tile_h == def.tile_h && c.persistent == def.persistent)
                continue;
            double t = 0.0;
            st = time_cfg(p, c, reps, a, b, &t);
            if (st == CRB_OK && t < t_cur) {
                t_cur = t;
                cur = c;
            }
        }
    const int growh[4] = {8, 16, 32, -1};      // -1: fused
    const LaunchCfg det = cur;
    for (int gi = 0; st == CRB_OK && gi < 4; ++gi) {
        LaunchCfg c = det;
        c.fused = growh[gi] < 0 ? 1 : 0;
        c.grow_h = growh[gi] < 0 ? 0 : growh[gi];
        double t = 0.0;
        st = time_cfg(p, c, reps, a, b, &t);
        if (st == CRB_OK && t < t_cur) {
            t_cur = t;
            cur = c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != CRB_OK)
        return st;
    if ((st = plan_apply(p, cur)) != CRB_OK)
        return st;
    tune_cache_store(p->key, cur, t_cur, t_def);
    if (best)
        *best = tuning_from(cur);
    if (out_ms)
        *out_ms = t_cur;
    if (out_default_ms)
        *out_default_ms = t_def;
    return ok();
}

crb_status crb_plan_set_timing(crb_plan *p, int32_t enable) {
    if (!p)
        return fail(CRB_EINVAL, "null plan");
    if (enable && p->use_graph)
        return fail(CRB_EINVAL, "per-launch timing needs a plan without a graph");
    p->timing = enable != 0;
    p->ev_used = 0;
    for (int i = 0; i < kNumKernelKinds; ++i) {
        p->acc_ms[i] = 0.0;
        p->acc_n[i] = 0;
    }
    return ok();
}

crb_status crb_plan_set_counting(crb_plan *p, int32_t enable) {
    if (!p)
        return fail(CRB_EINVAL, "null plan");
    hipError_t e = hipStreamSynchronize(p->stream);
    for (DevFrame &f : p->hframes)
        f.flags = enable ? (f.flags | kCountWork) : (f.flags & ~kCountWork);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_frames, p->hframes.data(), p->hframes.size() * sizeof(DevFrame),
                           hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(p->d_work, 0,
                           kWorkCounters * (size_t)p->n * sizeof(unsigned long long), p->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess)
        return hip_status(e, "counter setup");
    p->counting = enable != 0;
    // a one-frame plan passes its frame by value: its graph holds the old flags
    if (p->use_graph && p->n == 1) {
        crb_status st = plan_capture(p);
        if (st != CRB_OK)
            return st;
    }
    return ok();
}

crb_status crb_plan_work_counts(crb_plan *p, int64_t *counts) {
    if (!p || !counts)
        return fail(CRB_EINVAL, "null argument");
    std::vector<unsigned long long> w(kWorkCounters * (size_t)p->n);
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess)
        e = hipMemcpy(w.data(), p->d_work, w.size() * sizeof(unsigned long long),
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_status(e, "counter copy");
    for (int c = 0; c < kWorkCounters; ++c)
        counts[c] = 0;
    for (int i = 0; i < p->n; ++i)
        for (int c = 0; c < kWorkCounters; ++c)
            counts[c] += (int64_t)w[kWorkCounters * (size_t)i + c];
    return ok();
}

crb_status crb_plan_kernel_times(crb_plan *p, double *ms, int64_t *launches) {
    if (!p || !ms || !launches)
        return fail(CRB_EINVAL, "null argument");
    if (p->ev_used) {
        hipError_t e = hipEventSynchronize(p->events[2 * p->ev_used - 1]);
        if (e != hipSuccess)
            return hip_status(e, "hipEventSynchronize");
        for (size_t i = 0; i < p->ev_used; ++i) {
            float t = 0.0f;
            e = hipEventElapsedTime(&t, p->events[2 * i], p->events[2 * i + 1]);
            if (e != hipSuccess)
                return hip_status(e, "hipEventElapsedTime");
            p->acc_ms[p->ev_kind[i]] += (double)t;
            p->acc_n[p->ev_kind[i]] += 1;
        }
        p->ev_used = 0;
    }
    for (int i = 0; i < kNumKernelKinds; ++i) {
        ms[i] = p->acc_ms[i];
        launches[i] = p->acc_n[i];
    }
    return ok();
}

crb_status crb_lacosmic_batched(crb_frame *frames, int32_t n, void *hip_stream) {
    crb_plan *p = nullptr;
    crb_status st = crb_plan_create(frames, n, hip_stream, 0, &p);
    if (st != CRB_OK)
        return st;
    st = crb_plan_run(p);
    if (st == CRB_OK)
        st = crb_plan_stats(p, frames, n);
    plan_free(p);
    return st == CRB_OK ? ok() : st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// partitioned run (the paper's subimages with a border)
// ---------------------------------------------------------------------------

extern "C" crb_status crb_lacosmic_partitioned(const float *img, int32_t H, int32_t W, float gain,
                                               float readnoise, float sky, float sigclip,
                                               float sigfrac, float objlim, int32_t niter,
                                               int32_t ny, int32_t nx, int32_t border,
                                               float *out_clean, uint8_t *out_mask) {
    crb_status st = check_frame_args(H, W, gain, readnoise, sky, sigclip, sigfrac, objlim, niter);
    if (st != CRB_OK)
        return st;
    const size_t npix = (size_t)H * (size_t)W;
    if ((st = check_buffers(img, out_clean, out_mask, npix)) != CRB_OK)
        return st;
    if (border == -1) {
        WorkArgs none;
        memset(&none, 0, sizeof(none));
        border = work_radius(kWorkLacosmic, none, niter);
    }
    if (ny < 1 || nx < 1 || ny > H || nx > W || border < 0)
        return fail(CRB_EINVAL, "partition %d x %d with border %d does not fit %d x %d", ny, nx,
                    border, H, W);
    hipStream_t s = t_stream;
    const int nsub = ny * nx;
    std::vector<SubRect> subs(nsub);
    std::vector<size_t> off(nsub);
    size_t total = 0, max_sub = 0;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    for (int i = 0; i < ny; ++i) {
        for (int j = 0; j < nx; ++j) {
            SubRect &r = subs[i * nx + j];
            r.y0 = (int)((int64_t)H * i / ny);
            r.y1 = (int)((int64_t)H * (i + 1) / ny);
            r.x0 = (int)((int64_t)W * j / nx);
            r.x1 = (int)((int64_t)W * (j + 1) / nx);
            r.a0 = r.y0 - border > 0 ? r.y0 - border : 0;
            r.b0 = r.x0 - border > 0 ? r.x0 - border : 0;
            r.h = (r.y1 + border < H ? r.y1 + border : H) - r.a0;
            r.w = (r.x1 + border < W ? r.x1 + border : W) - r.b0;
            const size_t n = (size_t)r.h * r.w;
            off[i * nx + j] = total;
            total += 2 * al(4 * n) + al(n);
            max_sub = n > max_sub ? n : max_sub;
        }
    }
    const size_t o_tab = total;
    const size_t bytes = o_tab + al(nsub * sizeof(SubRect));
    char *tmp = nullptr;
    hipError_t e = hipMalloc((void **)&tmp, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CRB_ENOMEM, "subimages of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    std::vector<crb_frame> frames(nsub);
    for (int q = 0; q < nsub; ++q) {
        SubRect &r = subs[q];
        const size_t n = (size_t)r.h * r.w;
        r.sub_img = reinterpret_cast<float *>(tmp + off[q]);
        r.sub_clean = reinterpret_cast<float *>(tmp + off[q] + al(4 * n));
        r.sub_mask = reinterpret_cast<uint8_t *>(tmp + off[q] + 2 * al(4 * n));
        crb_frame &f = frames[q];
        memset(&f, 0, sizeof(f));
        f.img = r.sub_img;
        f.out_clean = r.sub_clean;
        f.out_mask = r.sub_mask;
        f.H = r.h;
        f.W = r.w;
        f.gain = gain;
        f.readnoise = readnoise;
        f.sky = sky;
        f.sigclip = sigclip;
        f.sigfrac = sigfrac;
        f.objlim = objlim;
        f.niter = niter;
        f.flags = g_incremental.load() ? CRB_FLAG_INCREMENTAL : 0;
    }
    SubRect *d_subs = reinterpret_cast<SubRect *>(tmp + o_tab);
    crb_plan *plan = nullptr;
    // the table goes in on the launch stream (ordered before the extraction on any
    // stream kind) and is waited for before `subs` can go out of scope
    e = hipMemcpyAsync(d_subs, subs.data(), nsub * sizeof(SubRect), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_extract(img, W, d_subs, nsub, max_sub, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(tmp);
        return hip_status(e, "subimage extraction");
    }
    st = crb_plan_create(frames.data(), nsub, s, 0, &plan);
    if (st == CRB_OK)
        st = crb_plan_run(plan);
    if (st == CRB_OK) {
        e = launch_stitch(out_clean, out_mask, W, d_subs, nsub, max_sub, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        st = hip_status(e, "subimage stitching");
    }
    if (plan)
        crb_plan_destroy(plan);
    (void)hipStreamSynchronize(s);
    (void)hipFree(tmp);
    return st == CRB_OK ? ok() : st;
}

static_assert(sizeof(crb_work) == 32, "crb_work layout");
static_assert(sizeof(crb_source) == 40 && sizeof(crb_source) == sizeof(crb::SourceRec),
              "crb_source layout");
static_assert(offsetof(crb_source, flux) == offsetof(crb::SourceRec, flux) &&
              offsetof(crb_source, sx) == offsetof(crb::SourceRec, sx),
              "crb_source layout");

static_assert(CRB_FLAG_INCREMENTAL == crb::kIncremental, "flag values agree");
