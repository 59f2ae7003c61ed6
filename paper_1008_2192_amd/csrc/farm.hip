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

// A float in the global address space: loads through it are global (not flat) loads.
typedef __attribute__((address_space(1))) const float GFloat;
// Fourth word of a raw buffer resource on gfx9-family GPUs: 32-bit data format,
// range-checked against the byte count given with the base.
constexpr int kBufWord3 = 0x00020000;

// Where a work function finds its pixel: the frame (resident in HBM; neighbours are
// read through the caches, never beyond the declared radius) and the position.
struct FarmCtx {
    const float *in;      // frame, H x W
    int y, x, H, W;       // the pixel's frame coordinates, frame size
};

struct WorkPoisson {
    static constexpr bool kList = false;
    static constexpr bool kNeighbours = false;
    __host__ __device__ static int radius(const WorkArgs &) { return 0; }
    __device__ static float pixel(const FarmCtx &c, const WorkArgs &a) {
        const size_t i = (size_t)c.y * c.W + c.x;
        return poisson_deviate(c.in[i], i, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    }
};

// WAITER: wait in[i] microseconds (clamped to [0, 1e6]), then copy the pixel.
struct WorkWaiter {
    static constexpr bool kList = false;
    static constexpr bool kNeighbours = false;
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
// order (a plateau reports its first pixel).  The record's sums run over the
// in-frame pixels of the (2a+1)^2 box, row by row, in binary64 (no contraction),
// which fixes their rounding.  candidate() is the cheap test every pixel takes;
// find() runs on the candidates only.  The window is read row by row with 2R+1
// loads per row at clamped columns (R = max(r, a) <= 4, a compile-time bound chosen
// by a uniform switch), all rows unrolled, so the loads of a candidate overlap instead
// of each waiting for the one before.
template <int R>
__device__ __forceinline__ bool sources_find(const FarmCtx &c, const WorkArgs &a,
                                             SourceRec &rec) {
    constexpr int K = 2 * R + 1;
    const GFloat *in = (const GFloat *)c.in;
    const float v = in[(size_t)c.y * c.W + c.x];
    // away from the side edges a row's window is 2R+1 consecutive pixels: one address
    const bool inner = c.x >= R && c.x + R < c.W;
    bool peak = true;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
        const int yy = c.y + dy;
        if (dy < -a.r || dy > a.r || yy < 0 || yy >= c.H)
            continue;
        const GFloat *row = in + (size_t)yy * c.W;
        float q[K];
        if (inner) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                q[k] = row[c.x - R + k];
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k)
                q[k] = row[min(max(c.x - R + k, 0), c.W - 1)];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int dx = k - R, xx = c.x + dx;
            if (dx < -a.r || dx > a.r || xx < 0 || xx >= c.W || (dy == 0 && dx == 0))
                continue;
            const bool later = dy > 0 || (dy == 0 && dx > 0);
            if (!(q[k] < v) && !(later && q[k] == v))
                peak = false;
        }
    }
    if (!peak)
        return false;
    rec.y = c.y;
    rec.x = c.x;
    rec.peak = v;
    int npix = 0;
    double flux = 0.0, sy = 0.0, sx = 0.0;
    const double sky = (double)a.sky;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
        const int yy = c.y + dy;
        if (dy < -a.a || dy > a.a || yy < 0 || yy >= c.H)
            continue;
        const GFloat *row = in + (size_t)yy * c.W;
        float q[K];
        if (inner) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                q[k] = row[c.x - R + k];
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k)
                q[k] = row[min(max(c.x - R + k, 0), c.W - 1)];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int dx = k - R, xx = c.x + dx;
            if (dx < -a.a || dx > a.a || xx < 0 || xx >= c.W)
                continue;
            const double d = (double)q[k] - sky;
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

// The same test and sums with run-time loops, for radii above 4 (larger unrolled
// windows would not fit in registers).
__device__ __forceinline__ bool sources_find_loops(const FarmCtx &c, const WorkArgs &a,
                                                   SourceRec &rec) {
    const float *p = c.in + (size_t)c.y * c.W + c.x;
    const float v = p[0];
    const int ya = max(c.y - a.r, 0), yb = min(c.y + a.r, c.H - 1);
    const int xa = max(c.x - a.r, 0), xb = min(c.x + a.r, c.W - 1);
    for (int yy = ya; yy <= yb; ++yy) {
        const float *row = c.in + (size_t)yy * c.W;
        for (int xx = xa; xx <= xb; ++xx) {
            const float q = row[xx];
            const bool later = yy > c.y || (yy == c.y && xx > c.x);
            if (!(q < v) && !(later && q == v) && (yy != c.y || xx != c.x))
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
        const float *row = p + (ptrdiff_t)dy * c.W;
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

struct WorkSources {
    static constexpr bool kList = true;
    static constexpr bool kNeighbours = true;
    __host__ __device__ static int radius(const WorkArgs &a) { return a.r > a.a ? a.r : a.a; }
    __device__ static bool candidate(float v, const WorkArgs &a) { return v > a.threshold; }
    // Necessary for a source when r >= 1: the direct neighbours above and to the left
    // (earlier in raster order) are smaller, those below and to the right are not
    // larger.  A neighbour the scan does not know, or that lies outside the frame,
    // comes as -inf and passes.
    __device__ static bool neighbours(float v, float up, float dn, float lf, float rt,
                                      const WorkArgs &a) {
        return a.r < 1 || (up < v && lf < v && !(dn > v) && !(rt > v));
    }
    __device__ static bool find(const FarmCtx &c, const WorkArgs &a, SourceRec &rec) {
        switch (radius(a)) {
        case 1: return sources_find<1>(c, a, rec);
        case 2: return sources_find<2>(c, a, rec);
        case 3: return sources_find<3>(c, a, rec);
        case 4: return sources_find<4>(c, a, rec);
        default: return sources_find_loops(c, a, rec);
        }
    }
};

__global__ void k_farm_reset(unsigned int *tickets, unsigned long long *count) {
    if (threadIdx.x < kFarmQueues)
        tickets[threadIdx.x] = 0u;
    if (threadIdx.x == 0 && count)
        *count = 0ull;
}

// The next run of tiles for the calling wave, or t0 = -1 when every queue is drained.
// Lane 0 takes a ticket from the wave's current queue; once that range is exhausted,
// lanes 0..kFarmQueues-1 read all counters at once and the wave moves to the next
// queue (in cyclic order) that still has tiles.
__device__ __forceinline__ void next_tiles(unsigned int *__restrict__ tickets, long long ntiles,
                                           int chunk, int &queue, long long &t0, long long &t1) {
    const int lane = __lane_id();
    for (;;) {
        const long long q0 = ntiles * queue / kFarmQueues;
        const long long q1 = ntiles * (queue + 1) / kFarmQueues;
        int got = 0;
        if (lane == 0)
            got = (int)atomicAdd(&tickets[queue], (unsigned int)chunk);
        got = __shfl(got, 0);
        if (q0 + got < q1) {
            t0 = q0 + got;
            t1 = min(q1, t0 + chunk);
            return;
        }
        bool open = false;
        if (lane < kFarmQueues) {
            const long long a = ntiles * lane / kFarmQueues;
            const long long b = ntiles * (lane + 1) / kFarmQueues;
            const unsigned int seen = __hip_atomic_load(&tickets[lane], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            open = a + (long long)seen < b;
        }
        const unsigned long long m = __ballot(open) & ((1ull << kFarmQueues) - 1ull);
        if (!m) {
            t0 = t1 = -1;
            return;
        }
        const unsigned long long after = m & ~((2ull << queue) - 1ull);
        queue = __ffsll((long long)(after ? after : m)) - 1;
    }
}

// Moves a wave's buffered records to the caller's list: one atomic on the counter
// reserves their slots, then the wave copies them as 8-byte words.
__device__ __forceinline__ void flush_records(const SourceRec *__restrict__ buf, int n,
                                              SourceRec *__restrict__ out_list,
                                              long long capacity,
                                              unsigned long long *__restrict__ count) {
    constexpr int kWords = (int)(sizeof(SourceRec) / 8);
    const int lane = __lane_id();
    unsigned long long base = 0ull;
    if (lane == 0)
        base = atomicAdd(count, (unsigned long long)n);
    const unsigned int lo = __shfl((unsigned int)base, 0);
    const unsigned int hi = __shfl((unsigned int)(base >> 32), 0);
    base = ((unsigned long long)hi << 32) | lo;
    const unsigned long long *src = reinterpret_cast<const unsigned long long *>(buf);
    unsigned long long *dst = reinterpret_cast<unsigned long long *>(out_list);
    for (int i = lane; i < n * kWords; i += 64)
        if (base + (unsigned long long)(i / kWords) < (unsigned long long)capacity)
            dst[base * kWords + i] = src[i];
}

// The farm.  Every wave is an actor: it takes runs of `chunk` tiles from the tickets
// (tiles numbered row-major, split into kFarmQueues contiguous ranges; a wave starts
// on the queue of its global wave index modulo kFarmQueues -- workgroups are dealt
// round-robin to the XCDs, so a queue's tiles mostly stay in one XCD's L2) and works
// through each tile 64 pixels at a time, with no workgroup barrier.
//   Image work functions compute every pixel of the tile.
//   List work functions first scan the tile with a batch of loads in flight per lane
//   and compact the pixels that pass candidate() (and, for a function that declares
//   kNeighbours, neighbours() on the direct neighbours the batch holds) into a
//   per-wave LDS list; all lanes then run find() on the list (one candidate per lane)
//   and buffer the records they find per wave, moving them to the caller's list when
//   the buffer could not take another pass and at the end.  When tile_w is a multiple
//   of 64 (at most 256, with at most 256 rows) a batch is 16 rows of 64 pixels read by
//   buffer loads with a uniform row offset, and a tile's candidates gather in one list
//   (16-bit positions) so that find() runs on full passes.
template <class WF>
__global__ __launch_bounds__(256) void k_farm(const float *__restrict__ in, int H, int W,
                                              WorkArgs args, int tile_h, int tile_w, int chunk,
                                              int waves, float *__restrict__ out_img,
                                              SourceRec *__restrict__ out_list,
                                              long long capacity,
                                              unsigned long long *__restrict__ count,
                                              unsigned int *__restrict__ tickets) {
    constexpr int kScanBatch = 16;
    constexpr int kBufBatch = 16;   // rows of 64 pixels per batch of the buffer scan
    __shared__ int sCand[WF::kList ? 4 * kFarmCandidates : 1];
    __shared__ SourceRec sRec[WF::kList ? 4 * kFarmWaveRecords : 1];
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    const int gwave = blockIdx.x * 4 + wave;
    if (gwave >= waves)
        return;
    int *cand = sCand + (WF::kList ? wave * kFarmCandidates : 0);
    SourceRec *rbuf = sRec + (WF::kList ? wave * kFarmWaveRecords : 0);
    int nrec = 0;
    const int ntx = (W - 1) / tile_w + 1;
    const long long ntiles = (long long)ntx * ((H - 1) / tile_h + 1);
    int queue = gwave % kFarmQueues;
    FarmCtx c;
    c.in = in;
    c.H = H;
    c.W = W;
    for (;;) {
        long long t0, t1;
        next_tiles(tickets, ntiles, chunk, queue, t0, t1);
        if (t0 < 0)
            break;
        for (long long t = t0; t < t1; ++t) {
            const int y0 = (int)(t / ntx) * tile_h, x0 = (int)(t % ntx) * tile_w;
            const int th = min(tile_h, H - y0), tw = min(tile_w, W - x0);
            const long long n = (long long)th * tw;
            const int q = 64 / tw, rem = 64 - q * tw;
            int ly = lane / tw, lx = lane - ly * tw;
            if constexpr (!WF::kList) {
                for (long long j0 = 0; j0 < n; j0 += 64) {
                    if (j0 + lane < n) {
                        c.y = y0 + ly;
                        c.x = x0 + lx;
                        out_img[(size_t)c.y * W + c.x] = WF::pixel(c, args);
                    }
                    ly += q;
                    lx += rem;
                    if (lx >= tw) {
                        lx -= tw;
                        ++ly;
                    }
                }
            } else {
                // candidates run on one lane each; the find pass over the list
                uint16_t *const cand16 = reinterpret_cast<uint16_t *>(cand);
                auto run_candidates = [&](int ncand, bool packed) {
                    for (int i0 = 0; i0 < ncand; i0 += 64) {
                        SourceRec rec;
                        bool found = false;
                        if (i0 + lane < ncand) {
                            const int p = packed ? (int)cand16[i0 + lane] : cand[i0 + lane];
                            c.y = y0 + (packed ? (p >> 8) : p / tw);
                            c.x = x0 + (packed ? (p & 0xFF) : p % tw);
                            found = WF::find(c, args, rec);
                        }
                        const unsigned long long m = __ballot(found);
                        if (found)
                            rbuf[nrec + __popcll(m & ((1ull << lane) - 1ull))] = rec;
                        nrec += __popcll(m);
                        if (nrec > kFarmWaveRecords - 64) {
                            flush_records(rbuf, nrec, out_list, capacity, count);
                            nrec = 0;
                        }
                    }
                };
                int ncand = 0;
                if ((tile_w & 63) == 0 && tile_w <= 256 && th <= 256 &&
                    (long long)(th - 1) * W + tw < (1ll << 29)) {
                    // rows of whole 64-pixel segments: buffer loads over the tile's rows
                    // with the lane's byte offset and a uniform segment offset, so a load
                    // costs no vector instruction; candidates packed in 16 bits as
                    // (row << 8) | col, so twice as many wait for a full pass
                    const int nseg = tile_w >> 6;
                    const long long steps = (long long)th * nseg;
                    const __amdgpu_buffer_rsrc_t rows = __builtin_amdgcn_make_buffer_rsrc(
                        (void *)(in + (size_t)y0 * W + x0), (short)0,
                        (int)(((long long)(th - 1) * W + tw) * 4), kBufWord3);
                    float carry = -INFINITY;        // the row above a batch (nseg == 1)
                    // batch s0: rows of 64 pixels s0 .. s0+kBufBatch-1 in segment order
                    auto load_batch = [&](float (&v)[kBufBatch], long long s0) {
                        int row = (int)(s0 / nseg), seg = (int)(s0 - (long long)row * nseg);
#pragma unroll
                        for (int b = 0; b < kBufBatch; ++b) {
                            v[b] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                                rows, lane * 4, s0 + b < steps ? (row * W + seg * 64) * 4 : 0,
                                0));
                            if (++seg == nseg) {
                                seg = 0;
                                ++row;
                            }
                        }
                    };
                    for (long long s0 = 0; s0 < steps; s0 += kBufBatch) {
                        float v[kBufBatch];
                        load_batch(v, s0);
                        int row = (int)(s0 / nseg), seg = (int)(s0 - (long long)row * nseg);
#pragma unroll
                        for (int b = 0; b < kBufBatch; ++b) {
                            const int col = seg * 64 + lane;
                            bool hit = s0 + b < steps && col < tw && WF::candidate(v[b], args);
                            if constexpr (WF::kNeighbours) {
                                // direct neighbours this batch holds (same row: adjacent
                                // lanes; rows above and below: adjacent batch entries
                                // when a row is one segment)
                                const float lf = __shfl_up(v[b], 1), rt = __shfl_down(v[b], 1);
                                float up = -INFINITY, dn = -INFINITY;
                                if (nseg == 1) {
                                    up = b > 0 ? v[b > 0 ? b - 1 : 0] : carry;
                                    if (b + 1 < kBufBatch && s0 + b + 1 < steps)
                                        dn = v[b + 1 < kBufBatch ? b + 1 : b];
                                }
                                hit = hit && WF::neighbours(v[b], up, dn,
                                                           lane > 0 ? lf : -INFINITY,
                                                           lane < 63 && col + 1 < tw
                                                               ? rt : -INFINITY, args);
                            }
                            const unsigned long long m = __ballot(hit);
                            if (hit)
                                cand16[ncand + __popcll(m & ((1ull << lane) - 1ull))] =
                                    (uint16_t)((row << 8) | col);
                            ncand += __popcll(m);
                            if (++seg == nseg) {
                                seg = 0;
                                ++row;
                            }
                        }
                        carry = v[kBufBatch - 1];
                        if (ncand > 2 * kFarmCandidates - kBufBatch * 64 ||
                            s0 + kBufBatch >= steps) {
                            run_candidates(ncand, true);
                            ncand = 0;
                        }
                    }
                } else {
                long long j0 = 0;
                while (j0 < n) {
                    // scan up to kScanBatch passes, all loads first
                    float v[kScanBatch];
                    int pos[kScanBatch];
#pragma unroll
                    for (int b = 0; b < kScanBatch; ++b) {
                        // unconditional loads (a lane past the tile's end rereads the
                        // tile's first pixel and ignores it), so none waits for another
                        const bool in_tile = j0 + b * 64 + lane < n;
                        const int yy = in_tile ? y0 + ly : y0, xx = in_tile ? x0 + lx : x0;
                        v[b] = in[(size_t)yy * W + xx];
                        pos[b] = in_tile ? ly * tw + lx : -1;
                        ly += q;
                        lx += rem;
                        if (lx >= tw) {
                            lx -= tw;
                            ++ly;
                        }
                    }
#pragma unroll
                    for (int b = 0; b < kScanBatch; ++b) {
                        const bool hit = pos[b] >= 0 && WF::candidate(v[b], args);
                        const unsigned long long m = __ballot(hit);
                        if (hit)
                            cand[ncand + __popcll(m & ((1ull << lane) - 1ull))] = pos[b];
                        ncand += __popcll(m);
                    }
                    j0 += kScanBatch * 64;
                    // run the candidates when the list could not take another batch,
                    // and at the end of the tile
                    if (ncand > kFarmCandidates - kScanBatch * 64 || j0 >= n) {
                        run_candidates(ncand, false);
                        ncand = 0;
                    }
                }
                }
            }
        }
    }
    if constexpr (WF::kList) {
        if (nrec)
            flush_records(rbuf, nrec, out_list, capacity, count);
    }
}

template <class WF>
hipError_t launch_kind(const WorkArgs &args, const float *in, int H, int W, int workers,
                       int tile_h, int tile_w, float *out_img, SourceRec *out_list,
                       long long capacity, unsigned long long *count, unsigned int *tickets,
                       hipStream_t s) {
    // tickets of `chunk` tiles: about 2 per wave; atomics on a ticket counter serialise
    // in its L2, so few and spread over kFarmQueues counters keep them off the path
    const long long ntiles = (long long)((W - 1) / tile_w + 1) * ((H - 1) / tile_h + 1);
    long long chunk = ntiles / ((long long)workers * 2);
    chunk = chunk < 1 ? 1 : (chunk > 64 ? 64 : chunk);
    const int blocks = (workers + 3) / 4;
    k_farm<WF><<<blocks, 256, 0, s>>>(in, H, W, args, tile_h, tile_w, (int)chunk, workers,
                                      out_img, out_list, capacity, count, tickets);
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
