// Serving loop of libcrb: continuous (iteration-level) batching of frames that
// arrive over time, the GPU analogue of CRBLASTER's director polling its actors
// (Section 6.2: the director collects subimages as actors finish, without a
// barrier).
//
// Requests wait FIFO in pinned host staging.  A request is admitted when a slot is
// free and its device footprint (image, mask, workspace) fits the HBM budget; its
// upload runs on a copy stream.  Each round runs ONE iteration for every admitted
// frame, each at its own iteration index, with the batched kernels over a
// descriptor table rebuilt per round, so frames that arrive while others are on the
// GPU join at the next round.  A frame leaves after niter iterations or when an
// iteration selects no new pixel (early stop, result-neutral); its cleaned image
// and mask are copied back on the copy stream.  Progress is observed only by
// polling events: no call blocks on the device.  A server is used from one thread.
#include "api_internal.h"

#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <functional>
#include <thread>
#include <vector>

namespace crb {

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum ReqState { kWaiting, kActive, kDraining };

// Host copies between the caller's buffers and pinned staging, split over a few
// threads (a single core copies well below the host link's bandwidth).
class CopyPool {
  public:
    explicit CopyPool(unsigned n) {
        for (unsigned i = 0; i < n; ++i)
            threads_.emplace_back([this] { run(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : threads_)
            t.join();
    }
    void copy(void *dst, const void *src, size_t n) {
        const size_t chunk = (size_t)4 << 20;
        if (threads_.empty() || n <= chunk) {
            memcpy(dst, src, n);
            return;
        }
        const size_t parts = (n + chunk - 1) / chunk;
        std::atomic<size_t> next{0}, done{0};
        auto work = [&] {
            for (size_t p; (p = next.fetch_add(1)) < parts;) {
                const size_t off = p * chunk, len = off + chunk < n ? chunk : n - off;
                memcpy((char *)dst + off, (const char *)src + off, len);
                done.fetch_add(1);
            }
        };
        {
            std::lock_guard<std::mutex> g(mu_);
            job_ = work;
            ++gen_;
        }
        cv_.notify_all();
        work();                                   // the calling thread helps
        while (done.load() < parts)
            std::this_thread::yield();
        // retire the job and wait until no worker still holds it (it refers to this frame)
        std::unique_lock<std::mutex> g(mu_);
        job_ = nullptr;
        cv_done_.wait(g, [&] { return busy_ == 0; });
    }

  private:
    void run() {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> g(mu_);
        for (;;) {
            cv_.wait(g, [&] { return stop_ || gen_ != seen; });
            if (stop_)
                return;
            seen = gen_;
            if (!job_)
                continue;
            auto job = job_;
            ++busy_;
            g.unlock();
            job();
            g.lock();
            --busy_;
            cv_done_.notify_all();
        }
    }
    std::vector<std::thread> threads_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::condition_variable cv_done_;
    std::function<void()> job_;
    uint64_t gen_ = 0;
    int busy_ = 0;
    bool stop_ = false;
};

struct Request {
    int64_t id = 0;
    int32_t H = 0, W = 0;
    float gain = 0, readnoise = 0, sky = 0, sigclip = 0, sigfrac = 0, objlim = 0;
    int32_t niter = 0;
    const float *host_img = nullptr;   // caller's input, valid until completion
    bool direct = false;               // caller's buffers are pinned or on the device:
                                       // transferred without staging copies
    bool on_device = false;            // caller's buffers are device memory
    float *host_clean = nullptr;
    uint8_t *host_mask = nullptr;
    double t_submit = 0;
    size_t pin_bytes = 0, dev_bytes = 0;
    char *pin = nullptr;               // staging: image (4HW), then mask (HW)
    char *dev = nullptr;               // device: J (4HW) | mask (HW) | workspace
    DevFrame df;
    int k_next = 1;                    // next iteration to run
    ReqState state = kWaiting;
    hipEvent_t ev_h2d = nullptr;       // upload finished
    hipEvent_t ev_d2h = nullptr;       // download finished
    bool need_wait = false;            // next round must wait for ev_h2d
};

}  // namespace crb

using namespace crb;

struct crb_server {
    size_t budget = 0, in_use = 0, allocated = 0;
    int32_t max_slots = 0;
    int device = 0;
    hipStream_t compute = nullptr, copy = nullptr;
    int64_t next_id = 1;
    std::deque<Request *> waiting;
    std::vector<Request *> active;     // admitted, state kActive
    std::vector<Request *> draining;   // results being copied back
    // round in flight
    bool round_busy = false;
    std::vector<Request *> round_members;
    hipEvent_t ev_round = nullptr;
    // per-round tables: pinned host copies and device buffers
    size_t tab_cap = 0;                // bytes of each table buffer
    char *h_tab = nullptr, *d_tab = nullptr;
    // memory pools keyed by exact size
    std::multimap<size_t, char *> dev_free, pin_free;
    std::vector<hipEvent_t> event_pool;
    CopyPool *copies = nullptr;
};

namespace crb {

static crb_status get_event(crb_server *s, hipEvent_t *ev) {
    if (!s->event_pool.empty()) {
        *ev = s->event_pool.back();
        s->event_pool.pop_back();
        return CRB_OK;
    }
    return hip_status(hipEventCreateWithFlags(ev, hipEventDisableTiming), "hipEventCreate");
}

static void put_event(crb_server *s, hipEvent_t ev) {
    if (ev)
        s->event_pool.push_back(ev);
}

static crb_status pin_alloc(crb_server *s, size_t bytes, char **out) {
    auto it = s->pin_free.find(bytes);
    if (it != s->pin_free.end()) {
        *out = it->second;
        s->pin_free.erase(it);
        return CRB_OK;
    }
    hipError_t e = hipHostMalloc((void **)out, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
        return fail(CRB_ENOMEM, "pinned staging of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    return CRB_OK;
}

// device memory within the budget; pooled blocks of other sizes are released first
static crb_status dev_alloc(crb_server *s, size_t bytes, char **out) {
    auto it = s->dev_free.find(bytes);
    if (it != s->dev_free.end()) {
        *out = it->second;
        s->dev_free.erase(it);
        return CRB_OK;
    }
    while (s->allocated + bytes > s->budget && !s->dev_free.empty()) {
        auto victim = s->dev_free.begin();
        (void)hipFree(victim->second);
        s->allocated -= victim->first;
        s->dev_free.erase(victim);
    }
    if (s->allocated + bytes > s->budget)
        return CRB_EBUSY;
    hipError_t e = hipMalloc((void **)out, bytes);
    if (e != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
        return CRB_EBUSY;   // the device is fuller than the budget assumed: retry later
    }
    s->allocated += bytes;
    return CRB_OK;
}

// the kind of memory p points to: 0 pageable host memory (unknown to HIP), 1 page-locked
// host memory the device can read and write directly, 2 device memory of `device`,
// -1 another device's memory
static int memory_kind(const void *p, int device) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (a.type == hipMemoryTypeHost)
        return 1;
    if (a.type == hipMemoryTypeDevice)
        return a.device == device ? 2 : -1;
    return 0;
}

static size_t frame_dev_bytes(int32_t H, int32_t W) {
    const size_t n = (size_t)H * (size_t)W;
    const size_t img = (4 * n + 255) / 256 * 256;
    const size_t msk = (n + 255) / 256 * 256;
    return img + msk + ws_layout(H, W).total;
}

static void release_request(crb_server *s, Request *r) {
    if (r->dev) {
        s->dev_free.emplace(r->dev_bytes, r->dev);
        s->in_use -= r->dev_bytes;
        r->dev = nullptr;
    }
    if (r->pin) {
        s->pin_free.emplace(r->pin_bytes, r->pin);
        r->pin = nullptr;
    }
    put_event(s, r->ev_h2d);
    put_event(s, r->ev_d2h);
    delete r;
}

// Admit waiting requests (FIFO) while slots and budget allow, at most a few per
// call: staging an admitted frame is a host copy, and the next round should start
// while later frames are still being staged.
constexpr int kAdmitPerPoll = 4;

static crb_status admit(crb_server *s) {
    // a cap on staged admissions only: direct transfers cost the host nothing
    for (int staged = 0; !s->waiting.empty() && staged < kAdmitPerPoll;) {
        Request *r = s->waiting.front();
        const int held = (int)(s->active.size() + s->draining.size());
        if (held >= s->max_slots || s->in_use + r->dev_bytes > s->budget)
            return CRB_OK;
        char *dev = nullptr;
        crb_status st = dev_alloc(s, r->dev_bytes, &dev);
        if (st == CRB_EBUSY)
            return CRB_OK;
        if (st != CRB_OK)
            return st;
        if ((st = get_event(s, &r->ev_h2d)) != CRB_OK) {
            s->dev_free.emplace(r->dev_bytes, dev);
            return st;
        }
        if (!r->direct) {
            if ((st = pin_alloc(s, r->pin_bytes, &r->pin)) != CRB_OK) {
                s->dev_free.emplace(r->dev_bytes, dev);
                return st;
            }
            s->copies->copy(r->pin, r->host_img, 4 * (size_t)r->H * r->W);
            ++staged;
        }
        const size_t n = (size_t)r->H * (size_t)r->W;
        const size_t img = (4 * n + 255) / 256 * 256;
        const size_t msk = (n + 255) / 256 * 256;
        float *J = reinterpret_cast<float *>(dev);
        uint8_t *mask = reinterpret_cast<uint8_t *>(dev + img);
        r->dev = dev;
        s->in_use += r->dev_bytes;
        r->df = make_devframe(J, J, mask, dev + img + msk, ws_layout(r->H, r->W), r->H, r->W,
                              r->gain, r->readnoise, r->sky, r->sigclip, r->sigfrac, r->objlim,
                              r->niter, kFreshMask);
        hipError_t e = hipMemcpyAsync(J, r->direct ? (const void *)r->host_img : r->pin, 4 * n,
                                      r->on_device ? hipMemcpyDeviceToDevice
                                                   : hipMemcpyHostToDevice,
                                      s->copy);
        if (e == hipSuccess)
            e = hipEventRecord(r->ev_h2d, s->copy);
        if (e != hipSuccess)
            return hip_status(e, "upload");
        r->need_wait = true;
        r->k_next = 1;
        r->state = kActive;
        s->waiting.pop_front();
        s->active.push_back(r);
    }
    return CRB_OK;
}

static crb_status ensure_tables(crb_server *s, size_t bytes) {
    if (s->tab_cap >= bytes)
        return CRB_OK;
    size_t cap = s->tab_cap ? s->tab_cap : 1 << 16;
    while (cap < bytes)
        cap *= 2;
    if (s->h_tab)
        (void)hipHostFree(s->h_tab);
    if (s->d_tab)
        (void)hipFree(s->d_tab);
    s->h_tab = nullptr;
    s->d_tab = nullptr;
    s->tab_cap = 0;
    hipError_t e = hipHostMalloc((void **)&s->h_tab, cap, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipMalloc((void **)&s->d_tab, cap);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CRB_ENOMEM, "round tables of %zu bytes: %s", cap, hipGetErrorString(e));
    }
    s->tab_cap = cap;
    return CRB_OK;
}

// one iteration for every active frame, at its own iteration index
static crb_status launch_round(crb_server *s) {
    const int n = (int)s->active.size();
    if (n == 0)
        return CRB_OK;
    size_t ntd = 0, ntg = 0, pix = 0;
    for (Request *r : s->active) {
        ntd += (size_t)detect_tiles(r->H, r->W, kDetectTYDefault);
        ntg += (size_t)((r->H + kGrowTY - 1) / kGrowTY) * ((r->W + kGrowTX - 1) / kGrowTX);
        pix += (size_t)r->H * r->W;
    }
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o_fr = 0, o_td = al(n * sizeof(DevFrame)), o_tg = o_td + al(ntd * sizeof(TileRef));
    const size_t o_pre = o_tg + al(ntg * sizeof(TileRef));
    const size_t o_st = o_pre + al((n + 1) * sizeof(unsigned int));
    const size_t bytes = o_st + al(2 * n * sizeof(long long));
    crb_status st = ensure_tables(s, bytes);
    if (st != CRB_OK)
        return st;
    DevFrame *hf = reinterpret_cast<DevFrame *>(s->h_tab + o_fr);
    TileRef *htd = reinterpret_cast<TileRef *>(s->h_tab + o_td);
    TileRef *htg = reinterpret_cast<TileRef *>(s->h_tab + o_tg);
    size_t itd = 0, itg = 0;
    for (int i = 0; i < n; ++i) {
        Request *r = s->active[i];
        hf[i] = r->df;
        hf[i].k = r->k_next;
        for (int y = 0; y < r->H; y += kDetectTYDefault)
            for (int x = 0; x < r->W; x += kDetectTX)
                htd[itd++] = TileRef{i, y, x, 0};
        for (int y = 0; y < r->H; y += kGrowTY)
            for (int x = 0; x < r->W; x += kGrowTX)
                htg[itg++] = TileRef{i, y, x, 0};
        if (r->need_wait) {
            hipError_t e = hipStreamWaitEvent(s->compute, r->ev_h2d, 0);
            if (e != hipSuccess)
                return hip_status(e, "hipStreamWaitEvent");
            r->need_wait = false;
        }
    }
    const DevFrame *dfr = reinterpret_cast<const DevFrame *>(s->d_tab + o_fr);
    const TileRef *dtd = reinterpret_cast<const TileRef *>(s->d_tab + o_td);
    const TileRef *dtg = reinterpret_cast<const TileRef *>(s->d_tab + o_tg);
    unsigned int *dpre = reinterpret_cast<unsigned int *>(s->d_tab + o_pre);
    long long *dst = reinterpret_cast<long long *>(s->d_tab + o_st);
    DevFrame none;
    memset(&none, 0, sizeof(none));
    hipError_t e = hipMemcpyAsync(s->d_tab, s->h_tab, o_pre, hipMemcpyHostToDevice, s->compute);
    // rounds mix frames at different iterations: the default launch shapes (one block per
    // 32 x 64 detection tile, separate grow, list prefix and replacement)
    const LaunchCfg cfg;
    if (e == hipSuccess)
        e = launch_init(dfr, n, none, (size_t)kMaxIter, nullptr, 0, s->compute);
    if (e == hipSuccess)
        e = launch_detect(dfr, dtd, (int)ntd, none, 0, cfg, nullptr, s->compute);
    if (e == hipSuccess)
        e = launch_grow(dfr, dtg, (int)ntg, none, 0, false, cfg, s->compute);
    if (e == hipSuccess)
        e = launch_list_prefix(dfr, n, 0, dpre, s->compute);
    if (e == hipSuccess)
        e = launch_replace(dfr, n, dpre, none, 0, replace_grid(pix), s->compute);
    if (e == hipSuccess)
        e = launch_round_stats(dfr, n, dst, s->compute);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_tab + o_st, dst, 2 * n * sizeof(long long),
                           hipMemcpyDeviceToHost, s->compute);
    if (e == hipSuccess)
        e = hipEventRecord(s->ev_round, s->compute);
    if (e != hipSuccess)
        return hip_status(e, "round launch");
    s->round_members = s->active;
    s->round_busy = true;
    return CRB_OK;
}

// the round finished: advance frames, start downloads of finished ones
static crb_status finish_round(crb_server *s) {
    const int n = (int)s->round_members.size();
    size_t ntd = 0, ntg = 0;
    for (Request *r : s->round_members) {
        ntd += (size_t)detect_tiles(r->H, r->W, kDetectTYDefault);
        ntg += (size_t)((r->H + kGrowTY - 1) / kGrowTY) * ((r->W + kGrowTX - 1) / kGrowTX);
    }
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o_st = al(n * sizeof(DevFrame)) + al(ntd * sizeof(TileRef)) +
                        al(ntg * sizeof(TileRef)) + al((n + 1) * sizeof(unsigned int));
    const long long *stats = reinterpret_cast<const long long *>(s->h_tab + o_st);
    std::vector<Request *> still;
    for (int i = 0; i < n; ++i) {
        Request *r = s->round_members[i];
        const int k = r->k_next;
        const bool done = k >= r->niter || stats[2 * i] == 0;
        if (!done) {
            r->k_next = k + 1;
            still.push_back(r);
            continue;
        }
        // download the cleaned image and the mask once the round is complete
        crb_status st = get_event(s, &r->ev_d2h);
        if (st != CRB_OK)
            return st;
        const size_t npx = (size_t)r->H * r->W;
        hipError_t e = hipStreamWaitEvent(s->copy, s->ev_round, 0);
        void *dst_clean = r->direct ? (void *)r->host_clean : (void *)r->pin;
        void *dst_mask = r->direct ? (void *)r->host_mask : (void *)(r->pin + 4 * npx);
        const hipMemcpyKind kind = r->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst_clean, r->df.J, 4 * npx, kind, s->copy);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst_mask, r->df.mask, npx, kind, s->copy);
        if (e == hipSuccess)
            e = hipEventRecord(r->ev_d2h, s->copy);
        if (e != hipSuccess)
            return hip_status(e, "download");
        r->state = kDraining;
        s->draining.push_back(r);
    }
    // frames admitted while the round ran were appended after its members
    for (size_t i = s->round_members.size(); i < s->active.size(); ++i)
        still.push_back(s->active[i]);
    s->active.swap(still);
    s->round_members.clear();
    s->round_busy = false;
    return CRB_OK;
}

}  // namespace crb

extern "C" {

crb_status crb_server_create(size_t hbm_budget, int32_t max_slots, crb_server **out) {
    if (!out)
        return fail(CRB_EINVAL, "null out");
    *out = nullptr;
    if (hbm_budget == 0 || max_slots < 1)
        return fail(CRB_EINVAL, "budget must be > 0 and max_slots >= 1");
    crb_server *s = new (std::nothrow) crb_server();
    if (!s)
        return fail(CRB_ENOMEM, "host allocation failed");
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    {
        unsigned hw = std::thread::hardware_concurrency();
        unsigned n = hw > 1 ? (hw < 9 ? hw - 1 : 7) : 0;
        s->copies = new (std::nothrow) CopyPool(n);
        if (!s->copies) {
            delete s;
            return fail(CRB_ENOMEM, "host allocation failed");
        }
    }
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&s->ev_round, hipEventDisableTiming);
    if (e != hipSuccess) {
        crb_server_destroy(s);
        return hip_status(e, "server setup");
    }
    *out = s;
    return ok();
}

crb_status crb_server_submit(crb_server *s, const float *host_img, int32_t H, int32_t W,
                             float gain, float readnoise, float sky, float sigclip, float sigfrac,
                             float objlim, int32_t niter, float *host_clean, uint8_t *host_mask,
                             int64_t *out_id) {
    const double t0 = now_s();
    if (!s || !host_img || !host_clean || !host_mask || !out_id)
        return fail(CRB_EINVAL, "null argument");
    crb_status st = check_frame_args(H, W, gain, readnoise, sky, sigclip, sigfrac, objlim, niter);
    if (st != CRB_OK)
        return st;
    const size_t npx = (size_t)H * (size_t)W;
    Request *r = new (std::nothrow) Request();
    if (!r)
        return fail(CRB_ENOMEM, "host allocation failed");
    r->H = H;
    r->W = W;
    r->gain = gain;
    r->readnoise = readnoise;
    r->sky = sky;
    r->sigclip = sigclip;
    r->sigfrac = sigfrac;
    r->objlim = objlim;
    r->niter = niter;
    r->host_clean = host_clean;
    r->host_mask = host_mask;
    r->t_submit = t0;
    r->dev_bytes = frame_dev_bytes(H, W);
    if (r->dev_bytes > s->budget) {
        delete r;
        return fail(CRB_EBUSY, "frame needs %zu bytes of device memory, budget is %zu",
                    frame_dev_bytes(H, W), s->budget);
    }
    r->pin_bytes = 5 * npx;
    r->host_img = host_img;
    const int ki = memory_kind(host_img, s->device), kc = memory_kind(host_clean, s->device),
              km = memory_kind(host_mask, s->device);
    if (ki < 0 || kc < 0 || km < 0 || (ki == 2) != (kc == 2) || (ki == 2) != (km == 2)) {
        delete r;
        return fail(CRB_EINVAL, "the image and both outputs must all be host memory or all "
                                "device memory of the server's device");
    }
    r->on_device = ki == 2;
    r->direct = ki > 0 && kc > 0 && km > 0;
    if (niter == 0 && r->on_device) {
        // nothing to compute: the result is the input, copied on the device
        hipError_t e = hipMemcpyAsync(host_clean, host_img, 4 * npx, hipMemcpyDeviceToDevice,
                                      s->copy);
        if (e == hipSuccess)
            e = hipMemsetAsync(host_mask, 0, npx, s->copy);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s->copy);
        if (e != hipSuccess) {
            delete r;
            return hip_status(e, "niter 0 copy");
        }
    } else if (niter == 0) {       // nothing to compute: the result is the input
        memcpy(host_clean, host_img, 4 * npx);
        memset(host_mask, 0, npx);
    }
    r->id = s->next_id++;
    *out_id = r->id;
    s->waiting.push_back(r);
    return ok();
}

crb_status crb_server_poll(crb_server *s, int64_t *done_ids, double *done_latency,
                           int32_t max_done, int32_t *n_done) {
    if (!s || !n_done || max_done < 0 || (max_done > 0 && (!done_ids || !done_latency)))
        return fail(CRB_EINVAL, "bad arguments");
    *n_done = 0;
    crb_status st;
    // requests with niter == 0 complete at once
    for (auto it = s->waiting.begin(); it != s->waiting.end();) {
        Request *r = *it;
        if (r->niter == 0 && *n_done < max_done) {
            done_ids[*n_done] = r->id;
            done_latency[*n_done] = now_s() - r->t_submit;
            ++*n_done;
            it = s->waiting.erase(it);
            release_request(s, r);
        } else {
            ++it;
        }
    }
    // finished downloads
    for (size_t i = 0; i < s->draining.size() && *n_done < max_done;) {
        Request *r = s->draining[i];
        hipError_t q = hipEventQuery(r->ev_d2h);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        if (q != hipSuccess)
            return hip_status(q, "download event");
        const size_t npx = (size_t)r->H * r->W;
        if (!r->direct) {
            s->copies->copy(r->host_clean, r->pin, 4 * npx);
            s->copies->copy(r->host_mask, r->pin + 4 * npx, npx);
        }
        done_ids[*n_done] = r->id;
        done_latency[*n_done] = now_s() - r->t_submit;
        ++*n_done;
        s->draining.erase(s->draining.begin() + i);
        release_request(s, r);
    }
    // the round in flight
    if (s->round_busy) {
        hipError_t q = hipEventQuery(s->ev_round);
        if (q == hipErrorNotReady) {
            if ((st = admit(s)) != CRB_OK)     // uploads overlap the running round
                return st;
            return ok();
        }
        if (q != hipSuccess)
            return hip_status(q, "round event");
        if ((st = finish_round(s)) != CRB_OK)
            return st;
    }
    if ((st = admit(s)) != CRB_OK)
        return st;
    if ((st = launch_round(s)) != CRB_OK)
        return st;
    return ok();
}

int32_t crb_server_pending(crb_server *s) {
    if (!s)
        return 0;
    return (int32_t)(s->waiting.size() + s->active.size() + s->draining.size());
}

void crb_server_destroy(crb_server *s) {
    if (!s)
        return;
    if (s->compute)
        (void)hipStreamSynchronize(s->compute);
    if (s->copy)
        (void)hipStreamSynchronize(s->copy);
    for (Request *r : s->waiting)
        release_request(s, r);
    for (Request *r : s->active)
        release_request(s, r);
    for (Request *r : s->draining)
        release_request(s, r);
    for (auto &kv : s->dev_free)
        (void)hipFree(kv.second);
    for (auto &kv : s->pin_free)
        (void)hipHostFree(kv.second);
    for (hipEvent_t ev : s->event_pool)
        (void)hipEventDestroy(ev);
    if (s->ev_round)
        (void)hipEventDestroy(s->ev_round);
    if (s->h_tab)
        (void)hipHostFree(s->h_tab);
    if (s->d_tab)
        (void)hipFree(s->d_tab);
    if (s->compute)
        (void)hipStreamDestroy(s->compute);
    if (s->copy)
        (void)hipStreamDestroy(s->copy);
    delete s->copies;
    delete s;
}

}  // extern "C"
