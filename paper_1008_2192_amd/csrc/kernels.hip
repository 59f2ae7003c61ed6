// HIP kernels of libcrb for gfx950 (MI355X): one L.A.Cosmic iteration as three
// launches -- detection (detect.hip), grow/count, replacement -- plus init, stats,
// subimage and parity-test helpers.
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
#include "device_common.h"

#include <math.h>

namespace crb {

#include "medtile.inc"     // sort25 for the replacement

// ---------------------------------------------------------------------------
// grow + count + cumulative mask + flagged list
// ---------------------------------------------------------------------------
//
// Word-parallel: a lane holds the codes of 16 horizontally adjacent pixels in four
// dwords (byte j of dword d = pixel 4d + j), so a 3-wide dilation is byte shifts
// inside the lane plus the edge bytes of the neighbouring lanes.  A wave covers 62
// such groups (992 pixels) of a strip of kGrowTY rows; lanes 0 and 63 hold the
// groups just outside the strip, whose inner edge bytes the dilation needs.  Rows
// stream through a delay line: codes of row y give the horizontal dilation of the
// first selection at y, then G1 at y-1 (vertical OR of three rows, gated by
// S' > sigclip), then G2 at y-2 (gated by S' > sigfrac*sigclip).  No LDS and no
// block barrier.  The flagged list is written row by row across the wave, so
// consecutive entries are neighbours in a row.  Iteration 1 lists the whole mask; later
// iterations append their new flags only.  A strip with no first selection within reach
// returns at once (at iteration 1 only where detection has cleared the mask; after it A
// is rare, since the flagged pixels have been replaced).

constexpr uint32_t kByteLsb = 0x01010101u;

struct Px16 {
    uint32_t d[4];
};

__device__ __forceinline__ uint32_t shfl_prev(uint32_t v) {   // value of lane-1
    return (uint32_t)__shfl_up((int)v, 1);
}
__device__ __forceinline__ uint32_t shfl_next(uint32_t v) {   // value of lane+1
    return (uint32_t)__shfl_down((int)v, 1);
}
// 3-wide horizontal OR of byte flags (one flag in bit 0 of each byte)
__device__ __forceinline__ Px16 hdilate(const Px16 &v) {
    const uint32_t left = shfl_prev(v.d[3]) >> 24;          // pixel just left of this lane
    const uint32_t right = shfl_next(v.d[0]) << 24;         // pixel just right of this lane
    Px16 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t lo = q == 0 ? left : (v.d[q - 1] >> 24);
        const uint32_t hi = q == 3 ? right : (v.d[q + 1] << 24);
        o.d[q] = v.d[q] | (v.d[q] << 8) | (v.d[q] >> 8) | lo | hi;
    }
    return o;
}

// 16 bytes of row y starting at pixel x (x multiple of 16); bytes outside read 0
__device__ __forceinline__ Px16 load16(const uint8_t *__restrict__ p, int y, int x, int H, int W,
                                       bool aligned) {
    Px16 v = {{0u, 0u, 0u, 0u}};
    if (y < 0 || y >= H || x + 16 <= 0 || x >= W)
        return v;
    const uint8_t *row = p + (size_t)y * W;
    if (aligned && x >= 0) {
        const uint4 q = *reinterpret_cast<const uint4 *>(row + x);
        v.d[0] = q.x; v.d[1] = q.y; v.d[2] = q.z; v.d[3] = q.w;
        return v;
    }
#pragma unroll
    for (int b = 0; b < 16; ++b)
        if (x + b >= 0 && x + b < W)
            v.d[b >> 2] |= (uint32_t)row[x + b] << (8 * (b & 3));
    return v;
}

__device__ __forceinline__ void store16(uint8_t *__restrict__ p, int y, int x, int W,
                                        bool aligned, const Px16 &v) {
    uint8_t *row = p + (size_t)y * W;
    if (aligned) {
        *reinterpret_cast<uint4 *>(row + x) = make_uint4(v.d[0], v.d[1], v.d[2], v.d[3]);
        return;
    }
#pragma unroll
    for (int b = 0; b < 16; ++b)
        if (x + b < W)
            row[x + b] = (uint8_t)(v.d[b >> 2] >> (8 * (b & 3)));
}

// bits 0, 8, 16, 24 of v -> bits 0..3 (the four products land on bits 21..24 without carries)
__device__ __forceinline__ uint32_t squeeze4(uint32_t v) { return ((v * 0x00204081u) >> 21) & 0xFu; }

__device__ __forceinline__ unsigned int wave_incl_scan(unsigned int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned int u = (unsigned int)__shfl_up((int)v, o);
        if (lane >= o)
            v += u;
    }
    return v;
}

// 16 bytes of row y at pixel x (x a multiple of 16) from a plane whose width is a
// multiple of 16, with no branch: an out-of-frame group reads an in-frame one and is
// zeroed, so the load can be issued early (groups are wholly inside or outside).
__device__ __forceinline__ Px16 load16_aligned(const uint8_t *__restrict__ p, int y, int x,
                                               int H, int W) {
    const bool ok = y >= 0 && y < H && x >= 0 && x < W;
    const int yy = clampi(y, H), xx = min(max(x, 0), W - 16);
    const uint4 q = *reinterpret_cast<const uint4 *>(p + (size_t)yy * W + xx);
    const uint32_t m = ok ? 0xFFFFFFFFu : 0u;
    return Px16{{q.x & m, q.y & m, q.z & m, q.w & m}};
}

// Whether a strip of rows y0 .. y0+TYG-1 and columns x0 .. x0+kGrowTX-1 can gain a
// flag: G2 lies within 2 pixels of A (two 3x3 dilations), so with no A in the detection
// tiles within that reach the strip keeps its mask.  A tile that the reach enters by
// its first or last two rows only is judged by those rows.  Called by a whole wave.
template <int TYG>
__device__ __forceinline__ bool strip_near_first(const DevFrame &f, int y0, int x0, int lane) {
    // a strip lies in one row of detection tiles, so its reach touches at most three
    static_assert(kDetectTY % TYG == 0 && 3 * ((kGrowTX + 3) / kDetectTX + 2) <= 64,
                  "one lane per detection tile within reach");
    const int H = f.H, W = f.W;
    const int ylo = max(y0 - 2, 0), yhi = min(y0 + TYG + 1, H - 1);
    const int xlo = max(x0 - 2, 0), xhi = min(x0 + kGrowTX + 1, W - 1);
    const int r0 = ylo / kDetectTY, c0 = xlo / kDetectTX;
    const int ncol = xhi / kDetectTX - c0 + 1;
    bool hit = false;
    if (lane < (yhi / kDetectTY - r0 + 1) * ncol) {
        const int r = r0 + lane / ncol, c = c0 + lane % ncol, top = r * kDetectTY;
        const unsigned int need = ylo >= top + kDetectTY - 2 ? 4u : (yhi < top + 2 ? 2u : 1u);
        const uint32_t q = reinterpret_cast<const uint32_t *>(f.tile_first)
                               [r * ((W + kDetectTX - 1) / kDetectTX) + c];
        hit = ((q | q >> 8 | q >> 16 | q >> 24) & need) != 0u;   // the tile's four waves
    }
    return __ballot(hit) != 0ull;
}

// One wave's strip: rows y0 .. y0+TYG-1 of the 992-pixel column group at x0.  With
// ALIGNED (the width a multiple of 16) every load is branch-free and the code and mask
// rows are fetched kAhead rows before their use, so several are in flight at once.
template <int TYG, bool ALIGNED>
__device__ __forceinline__ void grow_strip(const DevFrame &f, int y0, int x0, int k, int lane) {
    constexpr int kAhead = 4;
    const int H = f.H, W = f.W;
    // iteration 1 on a mask that detection has just cleared: nothing to read
    const bool fresh = k == 1 && (f.flags & kFreshMask);
    const int px = x0 - 16 + 16 * lane;                // first pixel of this lane's group
    const bool owner = lane >= 1 && lane <= kGrowTX / 16 && px < W;
    // from iteration 2 on the list already holds M_{k-1} and takes only the new flags
    const bool list_new = k >= 2;
    if ((list_new || fresh) && !f.g2 && f.tile_first &&
        !strip_near_first<TYG>(f, y0, x0, lane))
        return;

    Px16 hA0 = {}, hA1 = {};          // dilated first selection, rows y-2, y-1
    Px16 hi1 = {};                    // [S' > sigclip] at row y-1
    Px16 lo1 = {}, lo2 = {};          // [S' > low] at rows y-1, y-2
    Px16 hG0 = {}, hG1 = {};          // dilated G1 at rows y-3, y-2
    uint32_t mbits[TYG / 2];          // listed bits of the strip, 16 per row
    unsigned int nnew = 0, nm = 0;    // new flags, listed flags
    bool lane_new = false;
    Px16 cring[kAhead], mring[kAhead];
    if constexpr (ALIGNED) {
#pragma unroll
        for (int t = 0; t < kAhead; ++t) {
            cring[t] = load16_aligned(f.codes, y0 - 2 + t, px, H, W);
            mring[t] = load16_aligned(f.mask, y0 + t, px, H, W);
        }
    }
#pragma unroll
    for (int t = 0; t < TYG + 4; ++t) {
        const int y = y0 - 2 + t;
        Px16 c;
        if constexpr (ALIGNED) {
            c = cring[t % kAhead];
            if (t + kAhead < TYG + 4)
                cring[t % kAhead] = load16_aligned(f.codes, y + kAhead, px, H, W);
        } else {
            c = load16(f.codes, y, px, H, W, false);
        }
        Px16 a, hi2, lo0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a.d[q] = c.d[q] & kByteLsb;
            hi2.d[q] = (c.d[q] >> 1) & kByteLsb;
            lo0.d[q] = (c.d[q] >> 2) & kByteLsb;
        }
        const Px16 hA2 = hdilate(a);
        Px16 g1;                                      // G1 at row y-1 (zero outside the image)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            g1.d[q] = (hA0.d[q] | hA1.d[q] | hA2.d[q]) & hi1.d[q];
        const Px16 hG2 = hdilate(g1);
        if (t >= 4) {
            const int r = t - 4;                     // output row y0 + r == y - 2
            Px16 g2;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                g2.d[q] = (hG0.d[q] | hG1.d[q] | hG2.d[q]) & lo2.d[q];
            Px16 mp;
            if constexpr (ALIGNED) {
                mp = mring[r % kAhead];
                if (r + kAhead < TYG)
                    mring[r % kAhead] = load16_aligned(f.mask, y0 + r + kAhead, px, H, W);
                if (fresh)
                    mp = Px16{};
            }
            uint32_t m16 = 0;                        // listed flags of the row
            if (owner && y - 2 < H) {
                if constexpr (!ALIGNED)
                    mp = fresh ? Px16{} : load16(f.mask, y - 2, px, H, W, false);
                Px16 m;
                uint32_t anynew = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t nw = g2.d[q] & ~mp.d[q];
                    m.d[q] = mp.d[q] | g2.d[q];
                    anynew |= nw;
                    nnew += (unsigned int)__popc(nw);
                    m16 |= squeeze4(list_new ? nw : m.d[q]) << (4 * q);
                }
                if (anynew)
                    store16(f.mask, y - 2, px, W, ALIGNED, m);
                if (f.g2)
                    store16(f.g2, y - 2, px, W, ALIGNED, g2);
                lane_new |= anynew != 0u;
                nm += (unsigned int)__popc(m16);
            }
            if (r & 1)
                mbits[r >> 1] |= m16 << 16;
            else
                mbits[r >> 1] = m16;
        }
        hA0 = hA1; hA1 = hA2;
        lo2 = lo1; lo1 = lo0;
        hi1 = hi2;
        hG0 = hG1; hG1 = hG2;
    }
    // the strip lies in one row of detection tiles, and a lane's 16 pixels in one tile
    if (lane_new && f.tile_new)
        f.tile_new[(y0 / kDetectTY) * ((W + kDetectTX - 1) / kDetectTX) + px / kDetectTX] =
            (unsigned int)k;
    // one atomic per wave for the count and one for the list space; one scan of the
    // lanes' counts places each lane's entries (its rows in order) in the wave's space
    const unsigned int tn = __ockl_wfred_add_u32(nnew);
    const unsigned int incl = wave_incl_scan(nm, lane);
    const unsigned int total = (unsigned int)__builtin_amdgcn_readlane((int)incl, 63);
    if (!total) {
        if (tn && lane == 0)
            atomicAdd(&f.nnew[k - 1], (unsigned long long)tn);
        return;
    }
    unsigned int base = 0;
    if (lane == 0) {
        if (tn)
            atomicAdd(&f.nnew[k - 1], (unsigned long long)tn);
        base = atomicAdd(&f.listlen[0], total);
    }
    unsigned int off = (unsigned int)__builtin_amdgcn_readfirstlane((int)base) + incl - nm;
#pragma unroll
    for (int r = 0; r < TYG; ++r) {
        uint32_t m16 = (mbits[r >> 1] >> (16 * (r & 1))) & 0xFFFFu;
        while (m16) {
            const int b = __ffs(m16) - 1;
            f.list[off++] = (uint32_t)(y0 + r) * (uint32_t)W + (uint32_t)(px + b);
            m16 &= m16 - 1;
        }
    }
}

template <int TYG>
// 3 waves per SIMD: at most 168 VGPRs (the 32-row strip needs about that many)
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_grow(
    const DevFrame *__restrict__ frames, const TileRef *__restrict__ tiles, DevFrame single,
    int kiter, int ntiles) {
    const int lane = threadIdx.x & 63;
    const int wt = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);   // wave tile index
    if (wt >= ntiles)
        return;
    DevFrame f;
    int y0, x0;
    if (tiles) {
        // a listed strip of kGrowTY rows is split over kGrowTY / TYG waves
        constexpr int kSub = kGrowTY / TYG;
        const TileRef t = tiles[wt / kSub];
        f = frames[t.frame];
        y0 = t.y0;
        x0 = t.x0;
        if constexpr (kSub > 1) {
            y0 += (wt % kSub) * TYG;
            if (y0 >= f.H)
                return;
        }
    } else {
        f = single;
        const int ntx = (f.W + kGrowTX - 1) / kGrowTX;
        y0 = (wt / ntx) * TYG;
        x0 = (wt % ntx) * kGrowTX;
    }
    const int k = kiter ? kiter : f.k;
    if (frame_skips(f, k))
        return;
    if ((f.W & 15) == 0)
        grow_strip<TYG, true>(f, y0, x0, k, lane);
    else
        grow_strip<TYG, false>(f, y0, x0, k, lane);
}

// ---------------------------------------------------------------------------
// replacement
// ---------------------------------------------------------------------------

// Unflagged pixels are never written and flagged ones are never used as values, so
// the update in place is correct within the launch.  All 25 mask bytes and all 25 J
// values of the window are loaded unconditionally (clamped addresses are always
// valid), so the 50 loads are in flight together; a flagged neighbour's J may be
// rewritten meanwhile by another thread, and that value is discarded.
__device__ __forceinline__ void replace_one(const DevFrame &f, uint32_t p, int k) {
    const int W = f.W, H = f.H;
    const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * (uint32_t)W);
    // From iteration 2 on, J differs from the input only at pixels of M_{k-1}, whose
    // values the previous replacement took from the unflagged input pixels of their
    // windows.  A pixel of M_{k-1} with no new flag within 2 pixels has the same
    // unflagged window now, so it keeps its value: a tile with no new flag of this
    // iteration (its stamp is not k) within reach means nothing to do.
    if (k >= 2 && f.tile_new) {
        const int tx = (W + kDetectTX - 1) / kDetectTX;
        const int r0 = max(y - 2, 0) / kDetectTY, r1 = min(y + 2, H - 1) / kDetectTY;
        const int c0 = max(x - 2, 0) / kDetectTX, c1 = min(x + 2, W - 1) / kDetectTX;
        const unsigned int *t = f.tile_new, uk = (unsigned int)k;
        if (t[r0 * tx + c0] != uk && t[r0 * tx + c1] != uk && t[r1 * tx + c0] != uk &&
            t[r1 * tx + c1] != uk)
            return;
    }
    float v[25];
    uint8_t mk[25];
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy) {
        const size_t row = (size_t)clampi(y + dy, H) * W;
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            const size_t q = row + clampi(x + dx, W);
            mk[(dy + 2) * 5 + dx + 2] = f.mask[q];
            v[(dy + 2) * 5 + dx + 2] = f.J[q];
        }
    }
    const float old = v[12];
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < 25; ++j) {
        const bool m = mk[j] != 0;
        v[j] = m ? INFINITY : v[j];
        cnt += m ? 0 : 1;
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
    const float nv = (ia == ib) ? a : (float)(((double)a + (double)b) * 0.5);
    f.J[p] = nv;
    // incremental detection: a new value dirties every detection tile within
    // Chebyshev distance 4 (the reach of a code into J)
    if ((f.flags & kIncremental) && __float_as_uint(nv) != __float_as_uint(old)) {
        const int tx = (W + kDetectTX - 1) / kDetectTX;
        const int ty0 = max(y - 4, 0) / kDetectTY, ty1 = min(y + 4, H - 1) / kDetectTY;
        const int tx0 = max(x - 4, 0) / kDetectTX, tx1 = min(x + 4, W - 1) / kDetectTX;
        for (int a = ty0; a <= ty1; ++a)
            for (int b = tx0; b <= tx1; ++b)
                f.dirty[a * tx + b] = 1;
    }
}

__global__ __launch_bounds__(kThreads) void k_list_prefix(const DevFrame *__restrict__ frames,
                                                          int nframes, int kiter,
                                                          unsigned int *__restrict__ prefix) {
    __shared__ unsigned int sPart[kThreads];
    __shared__ unsigned int sCarry;
    if (threadIdx.x == 0)
        sCarry = 0;
    __syncthreads();
    for (int base = 0; base < nframes; base += kThreads) {
        const int i = base + threadIdx.x;
        unsigned int len = 0;
        if (i < nframes) {
            const DevFrame &f = frames[i];
            const int k = kiter ? kiter : f.k;
            len = frame_skips(f, k) ? 0u : f.listlen[0];
        }
        sPart[threadIdx.x] = len;
        __syncthreads();
        for (int o = 1; o < kThreads; o <<= 1) {      // inclusive scan
            const unsigned int v = threadIdx.x >= o ? sPart[threadIdx.x - o] : 0u;
            __syncthreads();
            sPart[threadIdx.x] += v;
            __syncthreads();
        }
        if (i < nframes)
            prefix[i] = sCarry + sPart[threadIdx.x] - len;
        __syncthreads();
        if (threadIdx.x == kThreads - 1)
            sCarry += sPart[kThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        prefix[nframes] = sCarry;
}

__global__ __launch_bounds__(kThreads) void k_replace(const DevFrame *__restrict__ frames,
                                                      int nframes,
                                                      const unsigned int *__restrict__ prefix,
                                                      DevFrame single, int kiter) {
    const unsigned int stride = gridDim.x * kThreads;
    unsigned int i = blockIdx.x * kThreads + threadIdx.x;
    if (!frames) {
        const int k = kiter ? kiter : single.k;
        if (frame_skips(single, k))
            return;
        const unsigned int n = single.listlen[0];
        for (; i < n; i += stride)
            replace_one(single, single.list[i], k);
        return;
    }
    const unsigned int total = prefix[nframes];
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD one
    // contiguous slice of the list (neighbouring pixels share cache lines in its L2).
    unsigned int end = total, step = stride;
    if ((gridDim.x & 7) == 0) {
        const unsigned int slice = (total + 7) >> 3;
        const unsigned int first = (blockIdx.x & 7) * slice;
        end = min(total, first + slice);
        i = first + (blockIdx.x >> 3) * kThreads + threadIdx.x;
        step = (gridDim.x >> 3) * kThreads;
    }
    // the frame holding item i: found once by bisection, then advanced as i grows
    int lo = 0;
    if (i < end) {
        int hi = nframes - 1;                          // last frame with prefix <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
    }
    for (; i < end; i += step) {
        while (prefix[lo + 1] <= i)
            ++lo;
        const DevFrame &f = frames[lo];
        replace_one(f, f.list[i - prefix[lo]], kiter ? kiter : f.k);
    }
}

// ---------------------------------------------------------------------------
// init and stats
// ---------------------------------------------------------------------------

// Grid rows (blockIdx.y) take the frames in turn.
__global__ __launch_bounds__(kThreads) void k_init(const DevFrame *__restrict__ frames,
                                                   int nframes, DevFrame single) {
    const size_t gid = (size_t)blockIdx.x * kThreads + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * kThreads;
    const int nf = frames ? nframes : 1;
    for (int fi = blockIdx.y; fi < nf; fi += gridDim.y) {
        const DevFrame f = frames ? frames[fi] : single;
        if (f.niter == 0) {
            const size_t n = (size_t)f.H * (size_t)f.W;
            for (size_t i = gid; i < n; i += stride) {
                if (f.img != f.J)
                    f.J[i] = f.img[i];
                f.mask[i] = 0;
            }
        }
        // counters restart at a frame's first iteration (f.k is 0 outside serving)
        if (f.nnew && f.k <= 1 && gid < (size_t)kMaxIter) {
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

__global__ void k_round_stats(const DevFrame *__restrict__ frames, int nframes,
                              long long *__restrict__ stats) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nframes)
        return;
    const DevFrame f = frames[i];
    long long total = 0;
    for (int k = 1; k <= f.k; ++k)
        total += (long long)f.nnew[k - 1];
    stats[2 * i] = (long long)f.nnew[f.k - 1];
    stats[2 * i + 1] = total;
}

// ---------------------------------------------------------------------------
// subimage partition (the paper's 2-D split with a border, Section 6.2)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_extract(const float *__restrict__ img, int W,
                                                      const SubRect *__restrict__ subs) {
    const SubRect r = subs[blockIdx.y];
    const size_t n = (size_t)r.h * r.w;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kThreads) {
        const int y = (int)(i / r.w), x = (int)(i - (size_t)y * r.w);
        r.sub_img[i] = img[(size_t)(r.a0 + y) * W + r.b0 + x];
    }
}

__global__ __launch_bounds__(kThreads) void k_stitch(float *__restrict__ out_clean,
                                                     uint8_t *__restrict__ out_mask, int W,
                                                     const SubRect *__restrict__ subs) {
    const SubRect r = subs[blockIdx.y];
    const int ih = r.y1 - r.y0, iw = r.x1 - r.x0;
    const size_t n = (size_t)ih * iw;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kThreads) {
        const int y = r.y0 + (int)(i / iw), x = r.x0 + (int)(i % iw);
        const size_t q = (size_t)(y - r.a0) * r.w + (x - r.b0);
        out_clean[(size_t)y * W + x] = r.sub_clean[q];
        out_mask[(size_t)y * W + x] = r.sub_mask[q];
    }
}

// ---------------------------------------------------------------------------
// parity-test kernels: the median networks alone, binary64 sqrt and division
// ---------------------------------------------------------------------------

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
                       size_t max_pixels, hipStream_t s) {
    const int rows = d_frames ? (nframes < 65535 ? nframes : 65535) : 1;
    const unsigned int cap = 4096u / (unsigned int)rows > 16u ? 4096u / (unsigned int)rows : 16u;
    const unsigned int gx = grid_for(max_pixels > (size_t)kMaxIter ? max_pixels : kMaxIter, cap);
    k_init<<<dim3(gx, rows), kThreads, 0, s>>>(d_frames, nframes, single);
    return hipGetLastError();
}

hipError_t launch_list_prefix(const DevFrame *d_frames, int nframes, int k,
                              unsigned int *d_prefix, hipStream_t s) {
    k_list_prefix<<<1, kThreads, 0, s>>>(d_frames, nframes, k, d_prefix);
    return hipGetLastError();
}

hipError_t launch_grow(const DevFrame *d_frames, const TileRef *d_tiles, int ntiles,
                       const DevFrame &single, int k, hipStream_t s) {
    constexpr int wpb = kThreads / 64;
    if (d_tiles) {
        if (ntiles <= 0)
            return hipSuccess;
        if (k >= 2) {
            // after iteration 1 few strips are near A and each runs alone: a wave per
            // 8-row part of a listed strip shortens the row chain it waits on
            const int n = ntiles * (kGrowTY / kGrowTYSmall);
            k_grow<kGrowTYSmall><<<(n + wpb - 1) / wpb, kThreads, 0, s>>>(d_frames, d_tiles,
                                                                           single, k, n);
        } else {
            k_grow<kGrowTY><<<(ntiles + wpb - 1) / wpb, kThreads, 0, s>>>(d_frames, d_tiles,
                                                                           single, k, ntiles);
        }
        return hipGetLastError();
    }
    // a single frame: short strips when the frame is small, so more waves share it, and
    // after iteration 1
    const bool small = k >= 2 || (size_t)single.H * single.W < ((size_t)1 << 22);
    const int ty = small ? kGrowTYSmall : kGrowTY;
    ntiles = ((single.W + kGrowTX - 1) / kGrowTX) * ((single.H + ty - 1) / ty);
    if (small)
        k_grow<kGrowTYSmall><<<(ntiles + wpb - 1) / wpb, kThreads, 0, s>>>(nullptr, nullptr,
                                                                            single, k, ntiles);
    else
        k_grow<kGrowTY><<<(ntiles + wpb - 1) / wpb, kThreads, 0, s>>>(nullptr, nullptr, single,
                                                                       k, ntiles);
    return hipGetLastError();
}

hipError_t launch_replace(const DevFrame *d_frames, int nframes, const unsigned int *d_prefix,
                          const DevFrame &single, int k, int grid, hipStream_t s) {
    k_replace<<<grid < 1 ? 1 : grid, kThreads, 0, s>>>(d_frames, nframes, d_prefix, single, k);
    return hipGetLastError();
}

hipError_t launch_stats(const DevFrame *d_frames, int nframes, long long *d_stats,
                        hipStream_t s) {
    k_stats<<<(nframes + 63) / 64, 64, 0, s>>>(d_frames, nframes, d_stats);
    return hipGetLastError();
}

hipError_t launch_round_stats(const DevFrame *d_frames, int nframes, long long *d_stats,
                              hipStream_t s) {
    k_round_stats<<<(nframes + 63) / 64, 64, 0, s>>>(d_frames, nframes, d_stats);
    return hipGetLastError();
}

hipError_t launch_extract(const float *img, int W, const SubRect *d_subs, int nsub,
                          size_t max_pixels, hipStream_t s) {
    dim3 grid(grid_for(max_pixels, 1024), nsub);
    k_extract<<<grid, kThreads, 0, s>>>(img, W, d_subs);
    return hipGetLastError();
}

hipError_t launch_stitch(float *out_clean, uint8_t *out_mask, int W, const SubRect *d_subs,
                         int nsub, size_t max_pixels, hipStream_t s) {
    dim3 grid(grid_for(max_pixels, 1024), nsub);
    k_stitch<<<grid, kThreads, 0, s>>>(out_clean, out_mask, W, d_subs);
    return hipGetLastError();
}

hipError_t launch_debug_fp64(const double *x, const double *y, int n, double *out_sqrt,
                             double *out_div, hipStream_t s) {
    k_debug_fp64<<<(n + kThreads - 1) / kThreads, kThreads, 0, s>>>(x, y, n, out_sqrt, out_div);
    return hipGetLastError();
}

}  // namespace crb
