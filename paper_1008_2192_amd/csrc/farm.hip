// Tile farm of libcrb (gfx950) and its work functions: POISSON and WAITER, the
// paper's framework probes (Section 6.3), and SOURCES, its example of a work
// function whose actors return structures (peak positions and aperture sums) rather
// than subimages (Section 7).  The contract between the farm and a work function is
// stated in farm.h.
#include "farm.h"

#include <math.h>

namespace crb {

// ---------------------------------------------------------------------------
// POISSON: Knuth's multiplication method on a counter-based generator
// ---------------------------------------------------------------------------

// Philox4x32-10 counter-based generator (Salmon et al., SC 2011): ten rounds of
// two 32x32->64-bit products with the multipliers 0xD2511F53 and 0xCD9E8D57; the
// key advances by 0x9E3779B9 and 0xBB67AE85 after each round.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// e^-x for 0 <= x <= 500: split x by ln 2 (Cody-Waite: a short high part of ln 2
// makes k * ln2_hi exact), degree-13 Taylor series of e^r by Horner's rule, then an
// exact power-of-two scale.  Only correctly rounded operations in a fixed order.
__device__ __forceinline__ double exp_neg(double x) {
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    const double inv_ln2 = 1.44269504088896338700e+00;
    const double y = -x;
    const double kf = floor(y * inv_ln2 + 0.5);
    const double r = (y - kf * ln2_hi) - kf * ln2_lo;
    const double inv_fact[14] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0,
                                 1.0 / 720.0, 1.0 / 5040.0, 1.0 / 40320.0, 1.0 / 362880.0,
                                 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0,
                                 1.0 / 6227020800.0};
    double p = inv_fact[13];
#pragma unroll
    for (int n = 12; n >= 0; --n)
        p = p * r + inv_fact[n];
    return ldexp(p, (int)kf);
}

// Poisson deviate with mean `mean` by multiplying uniforms until the product drops
// to e^-mean (Knuth's method); uniform j of pixel i comes from word j%4 of the
// generator at counter (i_lo, i_hi, j/4, 0).
__device__ __forceinline__ float poisson_deviate(float mean_f, size_t i, uint32_t k0,
                                                 uint32_t k1) {
    double mean = (double)mean_f;
    if (!(mean > 0.0))
        mean = 0.0;
    if (mean > 500.0)
        mean = 500.0;
    const double limit = exp_neg(mean);
    double prod = 1.0;
    unsigned int k = 0;
    for (uint32_t blk = 0;; ++blk) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), blk, 0u), k0, k1);
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            prod = prod * (((double)words[q] + 0.5) * (1.0 / 4294967296.0));
            if (!(prod > limit))
                return (float)k;
            ++k;
        }
    }
}

// Where a work function finds its pixel: the frame in global memory, and for
// staged kinds the LDS copy of the tile with its apron.
struct FarmCtx {
    const float *in;      // frame, H x W
    const float *tile;    // staged tile (row length pitch), null for unstaged kinds
    int pitch;
    int ly, lx;           // the pixel's position in the staged tile (apron included)
    int y, x, H, W;       // the pixel's frame coordinates, frame size
};

struct WorkPoisson {
    static constexpr bool kList = false, kStaged = false;
    __host__ __device__ static int radius(const WorkArgs &) { return 0; }
    __device__ static float pixel(const FarmCtx &c, const WorkArgs &a) {
        const size_t i = (size_t)c.y * c.W + c.x;
        return poisson_deviate(c.in[i], i, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    }
};

// WAITER: wait in[i] microseconds (clamped to [0, 1e6]), then copy the pixel.
struct WorkWaiter {
    static constexpr bool kList = false, kStaged = false;
    __host__ __device__ static int radius(const WorkArgs &) { return 0; }
    __device__ static float pixel(const FarmCtx &c, const WorkArgs &a) {
        const float v = c.in[(size_t)c.y * c.W + c.x];
        float us = v;
        if (!(us > 0.0f))
            us = 0.0f;
        if (us > 1.0e6f)
            us = 1.0e6f;
        const long long ticks = (long long)((double)us * (double)a.wall_khz / 1000.0);
        const long long t0 = (long long)wall_clock64();
        while ((long long)wall_clock64() - t0 < ticks)
            __builtin_amdgcn_s_sleep(1);
        return v;
    }
};

// SOURCES: a pixel is a source when it exceeds the threshold and every other pixel
// of the frame within Chebyshev distance r is smaller, or equal and later in raster
// order (a plateau reports its first pixel).  Out-of-frame apron positions hold
// -inf, which every candidate beats, so the peak test needs no bounds checks.  The
// record's sums run over the in-frame pixels of the (2a+1)^2 box, row by row, in
// binary64 (no contraction), which fixes their rounding.
struct WorkSources {
    static constexpr bool kList = true, kStaged = true;
    static constexpr float kOutside = -INFINITY;
    __host__ __device__ static int radius(const WorkArgs &a) { return a.r > a.a ? a.r : a.a; }
    __device__ static bool find(const FarmCtx &c, const WorkArgs &a, SourceRec &rec) {
        const float *t = c.tile + c.ly * c.pitch + c.lx;
        const float v = t[0];
        if (!(v > a.threshold))
            return false;
        for (int dy = -a.r; dy <= a.r; ++dy) {
            const float *row = t + dy * c.pitch;
            for (int dx = -a.r; dx <= a.r; ++dx) {
                const float q = row[dx];
                const bool later = dy > 0 || (dy == 0 && dx > 0);
                if (!(q < v) && !(later && q == v) && (dy != 0 || dx != 0))
                    return false;
            }
        }
        rec.y = c.y;
        rec.x = c.x;
        rec.peak = v;
        int npix = 0;
        double flux = 0.0, sy = 0.0, sx = 0.0;
        const double sky = (double)a.sky;
        for (int dy = -a.a; dy <= a.a; ++dy) {
            if (c.y + dy < 0 || c.y + dy >= c.H)
                continue;
            const float *row = t + dy * c.pitch;
            for (int dx = -a.a; dx <= a.a; ++dx) {
                if (c.x + dx < 0 || c.x + dx >= c.W)
                    continue;
                const double d = (double)row[dx] - sky;
                flux = flux + d;
                sy = sy + (double)dy * d;
                sx = sx + (double)dx * d;
                ++npix;
            }
        }
        rec.npix = npix;
        rec.flux = flux;
        rec.sy = sy;
        rec.sx = sx;
        return true;
    }
};

__global__ void k_farm_reset(unsigned int *tickets, unsigned long long *count) {
    if (threadIdx.x < kFarmQueues)
        tickets[threadIdx.x] = 0u;
    if (threadIdx.x == 0 && count)
        *count = 0ull;
}

// Moves the records buffered in LDS to the caller's list: one atomic on the counter
// reserves their slots, then the block copies them as 8-byte words.  Block-wide.
__device__ __forceinline__ void flush_records(SourceRec *__restrict__ sRec, unsigned int *sN,
                                              unsigned long long *sBase,
                                              SourceRec *__restrict__ out_list,
                                              long long capacity,
                                              unsigned long long *__restrict__ count) {
    constexpr int kT = 256, kWords = (int)(sizeof(SourceRec) / 8);
    const unsigned int n = *sN;
    if (threadIdx.x == 0)
        *sBase = atomicAdd(count, (unsigned long long)n);
    __syncthreads();
    const unsigned long long base = *sBase;
    const unsigned long long *src = reinterpret_cast<const unsigned long long *>(sRec);
    unsigned long long *dst = reinterpret_cast<unsigned long long *>(out_list);
    for (unsigned int i = threadIdx.x; i < n * kWords; i += kT) {
        const unsigned long long slot = base + i / kWords;
        if (slot < (unsigned long long)capacity)
            dst[base * kWords + i] = src[i];
    }
    __syncthreads();
    if (threadIdx.x == 0)
        *sN = 0u;
    __syncthreads();
}

// The persistent farm.  Tiles are numbered row-major and split into kFarmQueues
// contiguous ranges, one ticket counter each; a workgroup starts on queue
// blockIdx % kFarmQueues (workgroups are dealt round-robin to the XCDs, so a queue's
// tiles stay in one XCD's L2) and, when that range is exhausted, moves on to the
// next.  A ticket is a run of `chunk` consecutive tiles, so counters see few atomics.
// Each tile is staged (with its apron) if the work function reads neighbours, and
// the function runs on every pixel of it; positions within a tile advance by whole
// rows of the thread count, so no per-pixel division is needed.  List outputs are
// buffered in LDS (wave ballot, one LDS atomic per wave) and moved to the caller's
// list when the buffer could not take another pass, and at the end.
template <class WF>
__global__ __launch_bounds__(256) void k_farm(const float *__restrict__ in, int H, int W,
                                              WorkArgs args, int tile_h, int tile_w, int chunk,
                                              float *__restrict__ out_img,
                                              SourceRec *__restrict__ out_list,
                                              long long capacity,
                                              unsigned long long *__restrict__ count,
                                              unsigned int *__restrict__ tickets) {
    constexpr int kT = 256;
    extern __shared__ float sTile[];
    __shared__ long long sTicket, sEnd;
    __shared__ SourceRec sRec[WF::kList ? kFarmRecords : 1];
    __shared__ unsigned int sN;
    __shared__ unsigned long long sBase;
    const int R = WF::kStaged ? WF::radius(args) : 0;
    const int ntx = (W - 1) / tile_w + 1;
    const long long ntiles = (long long)ntx * ((H - 1) / tile_h + 1);
    if (WF::kList && threadIdx.x == 0)
        sN = 0u;
    int queue = blockIdx.x % kFarmQueues;
    for (;;) {
        if (threadIdx.x < 64) {
            // the first wave: lane 0 takes a ticket from the current queue; once that
            // range is exhausted, lanes 0..7 read all counters at once and the wave
            // moves to the next queue (in cyclic order) that still has tiles
            long long t = -1, end = 0;
            for (;;) {
                long long got = 0;
                const long long q0 = ntiles * queue / kFarmQueues;
                const long long q1 = ntiles * (queue + 1) / kFarmQueues;
                if (threadIdx.x == 0)
                    got = (long long)atomicAdd(&tickets[queue], (unsigned int)chunk);
                got = __shfl((int)got, 0);
                if (q0 + got < q1) {
                    t = q0 + got;
                    end = min(q1, t + chunk);
                    break;
                }
                bool open = false;
                if (threadIdx.x < kFarmQueues) {
                    const long long a = ntiles * threadIdx.x / kFarmQueues;
                    const long long b = ntiles * (threadIdx.x + 1) / kFarmQueues;
                    const unsigned int seen = __hip_atomic_load(&tickets[threadIdx.x],
                                                                __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                    open = a + (long long)seen < b;
                }
                const unsigned long long m = __ballot(open) & ((1ull << kFarmQueues) - 1ull);
                if (!m)
                    break;
                // next open queue after the current one, cyclically
                const unsigned long long after = m & ~((2ull << queue) - 1ull);
                queue = __ffsll((long long)(after ? after : m)) - 1;
            }
            if (threadIdx.x == 0) {
                sTicket = t;
                sEnd = end;
            }
        }
        __syncthreads();
        const long long t0 = sTicket, t1 = sEnd;
        __syncthreads();
        if (t0 < 0)
            break;
        for (long long t = t0; t < t1; ++t) {
            const int y0 = (int)(t / ntx) * tile_h, x0 = (int)(t % ntx) * tile_w;
            const int th = min(tile_h, H - y0), tw = min(tile_w, W - x0);
            FarmCtx c;
            c.in = in;
            c.tile = nullptr;
            c.pitch = 0;
            c.H = H;
            c.W = W;
            if constexpr (WF::kStaged) {
                // batches of kStageBatch elements per thread: a batch's loads are all
                // issued before its LDS stores, so their latencies overlap
                constexpr int kStageBatch = 8;
                const int pitch = tw + 2 * R, n = (th + 2 * R) * pitch;
                const int q = kT / pitch, rem = kT - q * pitch;
                int ly = threadIdx.x / pitch, lx = threadIdx.x - ly * pitch;
                for (int base = threadIdx.x; base < n; base += kStageBatch * kT) {
                    float v[kStageBatch];
#pragma unroll
                    for (int b = 0; b < kStageBatch; ++b) {
                        const int gy = y0 - R + ly, gx = x0 - R + lx;
                        v[b] = WF::kOutside;
                        if (base + b * kT < n && gy >= 0 && gy < H && gx >= 0 && gx < W)
                            v[b] = in[(size_t)gy * W + gx];
                        ly += q;
                        lx += rem;
                        if (lx >= pitch) {
                            lx -= pitch;
                            ++ly;
                        }
                    }
#pragma unroll
                    for (int b = 0; b < kStageBatch; ++b)
                        if (base + b * kT < n)
                            sTile[base + b * kT] = v[b];
                }
                c.tile = sTile;
                c.pitch = pitch;
                __syncthreads();
            }
            const long long n = (long long)th * tw;
            const int q = kT / tw, rem = kT - q * tw;
            int ly = threadIdx.x / tw, lx = threadIdx.x - ly * tw;
            for (long long j0 = 0; j0 < n; j0 += kT) {
                const bool valid = j0 + (long long)threadIdx.x < n;
                c.y = y0 + ly;
                c.x = x0 + lx;
                c.ly = ly + R;
                c.lx = lx + R;
                if constexpr (WF::kList) {
                    SourceRec rec;
                    const bool hit = valid && WF::find(c, args, rec);
                    const unsigned long long m = __ballot(hit);
                    if (m) {
                        const int lane = __lane_id();
                        const int leader = __ffsll((long long)m) - 1;
                        unsigned int base = 0u;
                        if (lane == leader)
                            base = atomicAdd(&sN, (unsigned int)__popcll(m));
                        base = __shfl(base, leader);
                        if (hit)
                            sRec[base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull))] = rec;
                    }
                    __syncthreads();
                    if (sN > (unsigned int)(kFarmRecords - kT))
                        flush_records(sRec, &sN, &sBase, out_list, capacity, count);
                } else {
                    if (valid)
                        out_img[(size_t)c.y * W + c.x] = WF::pixel(c, args);
                }
                ly += q;
                lx += rem;
                if (lx >= tw) {
                    lx -= tw;
                    ++ly;
                }
            }
            __syncthreads();    // the staged tile is reused by the next tile
        }
    }
    if constexpr (WF::kList) {
        if (sN)
            flush_records(sRec, &sN, &sBase, out_list, capacity, count);
    }
}

template <class WF>
hipError_t launch_kind(const WorkArgs &args, const float *in, int H, int W, int workers,
                       int tile_h, int tile_w, float *out_img, SourceRec *out_list,
                       long long capacity, unsigned long long *count, unsigned int *tickets,
                       hipStream_t s) {
    size_t lds = 0;
    if (WF::kStaged) {
        const int R = WF::radius(args);
        lds = (size_t)(tile_h + 2 * R) * (size_t)(tile_w + 2 * R) * sizeof(float);
    }
    // tickets of `chunk` tiles: about 8 per workgroup, so the dynamic balance keeps
    // a fine grain while the counters take few atomics
    const long long ntiles = (long long)((W - 1) / tile_w + 1) * ((H - 1) / tile_h + 1);
    long long chunk = ntiles / ((long long)workers * 8);
    chunk = chunk < 1 ? 1 : (chunk > 64 ? 64 : chunk);
    k_farm<WF><<<workers, 256, lds, s>>>(in, H, W, args, tile_h, tile_w, (int)chunk, out_img,
                                        out_list, capacity, count, tickets);
    return hipGetLastError();
}

int work_radius(int kind, const WorkArgs &a, int niter) {
    switch (kind) {
    case kWorkLacosmic:
        return 8 * niter;     // per iteration: detection 4, two grows 1 each, replacement 2
    case kWorkPoisson:
        return WorkPoisson::radius(a);
    case kWorkWaiter:
        return WorkWaiter::radius(a);
    case kWorkSources:
        return WorkSources::radius(a);
    default:
        return -1;
    }
}

size_t farm_lds_bytes(int kind, const WorkArgs &a, int tile_h, int tile_w) {
    if (kind != kWorkSources)
        return 0;
    const int R = WorkSources::radius(a);
    return (size_t)(tile_h + 2 * R) * (size_t)(tile_w + 2 * R) * sizeof(float) +
           kFarmRecords * sizeof(SourceRec);
}

hipError_t launch_farm_reset(unsigned int *tickets, unsigned long long *count, hipStream_t s) {
    k_farm_reset<<<1, 64, 0, s>>>(tickets, count);
    return hipGetLastError();
}

hipError_t launch_farm(int kind, const WorkArgs &args, const float *in, int H, int W,
                       int workers, int tile_h, int tile_w, float *out_img,
                       SourceRec *out_list, long long capacity, unsigned long long *count,
                       unsigned int *tickets, hipStream_t s) {
    switch (kind) {
    case kWorkPoisson:
        return launch_kind<WorkPoisson>(args, in, H, W, workers, tile_h, tile_w, out_img,
                                        out_list, capacity, count, tickets, s);
    case kWorkWaiter:
        return launch_kind<WorkWaiter>(args, in, H, W, workers, tile_h, tile_w, out_img,
                                       out_list, capacity, count, tickets, s);
    case kWorkSources:
        return launch_kind<WorkSources>(args, in, H, W, workers, tile_h, tile_w, out_img,
                                        out_list, capacity, count, tickets, s);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace crb
