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
// Numerics: medians are exact selections by min/max networks.  The replacement's
// median is an exact FP32 selection (the mean of two middle values is formed in
// binary64 and rounded once).  Every detection decision is the one the binary64
// definition takes (detect.hip: an FP32 estimate of S decides only where its proven
// error bound settles the comparison, binary64 in the definition's operation order
// elsewhere; no contraction: built with -ffp-contract=off), so a decision on a given
// J is independent of the tiling and of the launch shape.
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
    // a strip lies in one row of summary tiles, so its reach touches at most three
    static_assert(kSumTY % TYG == 0 && 3 * ((kGrowTX + 3) / kSumTX + 2) <= 64,
                  "one lane per summary tile within reach");
    const int H = f.H, W = f.W;
    const int ylo = max(y0 - 2, 0), yhi = min(y0 + TYG + 1, H - 1);
    const int xlo = max(x0 - 2, 0), xhi = min(x0 + kGrowTX + 1, W - 1);
    const int r0 = ylo / kSumTY, c0 = xlo / kSumTX;
    const int ncol = xhi / kSumTX - c0 + 1;
    bool hit = false;
    if (lane < (yhi / kSumTY - r0 + 1) * ncol) {
        const int r = r0 + lane / ncol, c = c0 + lane % ncol, top = r * kSumTY;
        const unsigned int need = ylo >= top + kSumTY - 2 ? 4u : (yhi < top + 2 ? 2u : 1u);
        const uint32_t q = reinterpret_cast<const uint32_t *>(f.tile_first)
                               [r * ((W + kSumTX - 1) / kSumTX) + c];
        hit = ((q | q >> 8 | q >> 16 | q >> 24) & need) != 0u;   // the tile's four waves
    }
    return __ballot(hit) != 0ull;
}

// One wave's strip: rows y0 .. y0+TYG-1 of the 992-pixel column group at x0.  With
// ALIGNED (the width a multiple of 16) every load is branch-free and the code and mask
// rows are fetched kAhead rows before their use, so several are in flight at once.
// FRESH: known to be iteration 1 on a mask that detection has just cleared, whose rows
// are then not read at all; other strips test for a fresh mask at run time and still
// load the mask rows (so that the one variant keeps its registers unspilled).
template <int TYG, bool ALIGNED, bool FRESH>
__device__ __forceinline__ void grow_strip(const DevFrame &f, int y0, int x0, int k, int lane) {
    constexpr int kAhead = 4;
    const int H = f.H, W = f.W;
    // iteration 1 on a mask that detection has just cleared: nothing to read
    const bool fresh = FRESH || (k == 1 && (f.flags & kFreshMask));
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
            if constexpr (!FRESH)
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
            if constexpr (ALIGNED && FRESH) {
                mp = Px16{};
            } else if constexpr (ALIGNED) {
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
    // the strip lies in one row of summary tiles, and a lane's 16 pixels in one tile
    if (lane_new && f.tile_new)
        f.tile_new[(y0 / kSumTY) * ((W + kSumTX - 1) / kSumTX) + px / kSumTX] = (unsigned int)k;
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

// FRESH: iteration 1, and every frame of the launch has a mask that detection has just
// cleared (a kernel of its own: with both aligned variants in one kernel the 32-row
// strip spills).
template <int TYG, bool FRESH>
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
        grow_strip<TYG, true, FRESH>(f, y0, x0, k, lane);
    else
        grow_strip<TYG, false, false>(f, y0, x0, k, lane);
}

// ---------------------------------------------------------------------------
// replacement
// ---------------------------------------------------------------------------

// The replacement of pixel (y, x) from its clamped 5 x 5 window: v holds J_k there and
// bit j of fl is set where the window's pixel j is flagged (M_k).  The median of the
// unflagged values (an even count: the mean of the two middle ones, formed in binary64
// and rounded once) is written to J; with no unflagged value J keeps its value.
__device__ __forceinline__ void replace_from_window(const DevFrame &f, int y, int x,
                                                    float (&v)[25], uint32_t fl, int k) {
    const int W = f.W, H = f.H;
    const float old = v[12];
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < 25; ++j) {
        const bool m = (fl >> j) & 1u;
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
    f.J[(size_t)y * W + x] = nv;
    // incremental detection: a new value stamps every summary tile within Chebyshev
    // distance 4 (the reach of a code into J) with this iteration; the next detection
    // re-evaluates the tiles meeting a summary tile with that stamp
    if ((f.flags & kIncremental) && __float_as_uint(nv) != __float_as_uint(old)) {
        const int tx = (W + kSumTX - 1) / kSumTX;
        const int ty0 = max(y - 4, 0) / kSumTY, ty1 = min(y + 4, H - 1) / kSumTY;
        const int tx0 = max(x - 4, 0) / kSumTX, tx1 = min(x + 4, W - 1) / kSumTX;
        for (int a2 = ty0; a2 <= ty1; ++a2)
            for (int b2 = tx0; b2 <= tx1; ++b2)
                f.dirty[a2 * tx + b2] = (uint8_t)k;
    }
}

// Values off .. off + 4 (off in 0..3) of the 8-value block (lo, hi): shifted by 2 when
// bit 1 of off is set, then by 1 when bit 0 is (selects of named values: an array here
// would be indexed through scratch memory).
__device__ __forceinline__ void window_row(float4 lo, float4 hi, int off, float &o0, float &o1,
                                           float &o2, float &o3, float &o4) {
    const bool s2 = (off & 2) != 0, s1 = (off & 1) != 0;
    const float h0 = s2 ? lo.z : lo.x, h1 = s2 ? lo.w : lo.y, h2 = s2 ? hi.x : lo.z;
    const float h3 = s2 ? hi.y : lo.w, h4 = s2 ? hi.z : hi.x, h5 = s2 ? hi.w : hi.y;
    o0 = s1 ? h1 : h0;
    o1 = s1 ? h2 : h1;
    o2 = s1 ? h3 : h2;
    o3 = s1 ? h4 : h3;
    o4 = s1 ? h5 : h4;
}

// Whether the 5x5 window of (y, x) can be read as aligned 8-pixel blocks, one per
// window row: at least 2 columns from either edge, the block of the bottom window row
// (the largest index: rows are clamped into the frame) ends within the frame buffer, and
// J starts on a 16-byte boundary.
__device__ __forceinline__ bool window_blocks_ok(const DevFrame &f, int y, int x) {
    const int W = f.W, H = f.H;
    if (x < 2 || x + 2 >= W || ((uintptr_t)f.J & 15u) != 0u)
        return false;
    const size_t last = (((size_t)min(y + 2, H - 1) * W + (size_t)(x - 2)) & ~(size_t)3) + 8;
    return last <= (size_t)H * (size_t)W;
}

// Index of the first pixel (column x - 2) of window row i (0..4) of (y, x); that row's
// block starts at the multiple of 4 at or below it.
__device__ __forceinline__ size_t window_row_start(const DevFrame &f, int y, int x, int i) {
    return (size_t)clampi(y + i - 2, f.H) * f.W + (size_t)(x - 2);
}

// J over the window of (y, x) (window_blocks_ok): two 16-byte loads a row.
__device__ __forceinline__ void load_window_j_blocks(const DevFrame &f, int y, int x,
                                                     float (&v)[25]) {
    float4 jb[5][2];
    int off[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const size_t s0 = window_row_start(f, y, x, i), a = s0 & ~(size_t)3;
        off[i] = (int)(s0 - a);
        const float4 *jp = reinterpret_cast<const float4 *>(f.J + a);
        jb[i][0] = jp[0];
        jb[i][1] = jp[1];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i)
        window_row(jb[i][0], jb[i][1], off[i], v[i * 5], v[i * 5 + 1], v[i * 5 + 2],
                   v[i * 5 + 3], v[i * 5 + 4]);
}

// Unflagged pixels are never written and flagged ones are never used as values, so
// the update in place is correct within the launch.  All mask bytes and J values of the
// window are loaded unconditionally (clamped addresses are always valid), so the loads
// are in flight together; a flagged neighbour's J may be rewritten meanwhile by another
// thread, and that value is discarded.  A pixel at least 2 columns from either edge
// whose window rows lie within the frame buffer as 8-pixel blocks takes each window row
// as the 8 values and 8 mask bytes at the 4-pixel boundary at or below x - 2 (two
// 16-byte and two 4-byte loads, not five of each): the pixels of a wave lie far apart,
// and every load instruction costs the cache an access per distinct line it meets.
// Other pixels load the 25 clamped positions one by one.
__device__ __forceinline__ void replace_one(const DevFrame &f, uint32_t p, int k) {
    const int W = f.W, H = f.H;
    const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * (uint32_t)W);
    // From iteration 2 on, J differs from the input only at pixels of M_{k-1}, whose
    // values the previous replacement took from the unflagged input pixels of their
    // windows.  A pixel of M_{k-1} with no new flag within 2 pixels has the same
    // unflagged window now, so it keeps its value: a tile with no new flag of this
    // iteration (its stamp is not k) within reach means nothing to do.
    if (k >= 2 && f.tile_new) {
        const int tx = (W + kSumTX - 1) / kSumTX;
        const int r0 = max(y - 2, 0) / kSumTY, r1 = min(y + 2, H - 1) / kSumTY;
        const int c0 = max(x - 2, 0) / kSumTX, c1 = min(x + 2, W - 1) / kSumTX;
        const unsigned int *t = f.tile_new, uk = (unsigned int)k;
        if (t[r0 * tx + c0] != uk && t[r0 * tx + c1] != uk && t[r1 * tx + c0] != uk &&
            t[r1 * tx + c1] != uk)
            return;
    }
    float v[25];
    uint32_t fl = 0u;
    if (window_blocks_ok(f, y, x) && ((uintptr_t)f.mask & 3u) == 0u) {
        // the mask bytes by the same blocks: one 8-byte load a row
        uint32_t mb[5][2];
        int off[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const size_t s0 = window_row_start(f, y, x, i), a = s0 & ~(size_t)3;
            off[i] = (int)(s0 - a);
            const uint32_t *mp = reinterpret_cast<const uint32_t *>(f.mask + a);
            mb[i][0] = mp[0];
            mb[i][1] = mp[1];
        }
        load_window_j_blocks(f, y, x, v);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const unsigned long long m =
                (((unsigned long long)mb[i][1] << 32) | mb[i][0]) >> (8 * off[i]);
#pragma unroll
            for (int j = 0; j < 5; ++j)
                fl |= ((m >> (8 * j)) & 0xFFull) != 0ull ? 1u << (i * 5 + j) : 0u;
        }
    } else {
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
#pragma unroll
        for (int j = 0; j < 25; ++j)
            fl |= mk[j] != 0 ? 1u << j : 0u;
    }
    replace_from_window(f, y, x, v, fl, k);
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
// fused grow + count + replacement (one launch per iteration)
// ---------------------------------------------------------------------------
//
// A wave takes a strip of TYG rows and 992 columns, as the grow does, and also computes
// G2 and M_k on the two rows above and the two below it (its mask halo, owned and written
// by the neighbouring strips): the codes it reads reach 4 rows beyond the strip, the
// mask 2.  M_k and G2 of those TYG + 4 rows go to the wave's part of the LDS as 16 bits
// per lane and row.  The wave then replaces the pixels of its own rows that need it, 64 at
// a time from a compacted list: at iteration 1 every pixel of M_k; later the pixels of M_k
// with a pixel of G2 within Chebyshev distance 2 (a superset of those with a new flag
// within 2, the only ones whose replacement can differ from the value they hold).
// No flagged list, list prefix or separate replacement launch is needed.
//
// The halo's mask may be read while its owner writes it: a halo pixel q has M_k(q) =
// M_{k-1}(q) | G2(q), and the owner only adds G2(q) to M_{k-1}(q), so whether the wave
// reads M_{k-1}(q) or M_k(q) the OR is M_k(q).  The replacement reads J only at pixels
// outside M_k, which no wave writes in this launch.

constexpr int kFusedList = 128;      // candidates per round of a wave's replacement

// Whether a strip of rows y0 .. y0+TYG-1 and columns x0 .. x0+kGrowTX-1 has a pixel of A
// within Chebyshev distance R (R <= 4), from the detection's summary bytes (8 rows each;
// a reach that meets a summary tile only in its first or last two rows tests those).
// Called by a whole wave.
template <int TYG, int R>
__device__ __forceinline__ bool strip_near_first_r(const DevFrame &f, int y0, int x0, int lane) {
    static_assert(R <= 4 && TYG <= kSumTY && kSumTY % TYG == 0 &&
                      3 * ((kGrowTX + 2 * R - 1) / kSumTX + 2) <= 64,
                  "one lane per summary tile within reach");
    const int H = f.H, W = f.W;
    const int ylo = max(y0 - R, 0), yhi = min(y0 + TYG - 1 + R, H - 1);
    const int xlo = max(x0 - R, 0), xhi = min(x0 + kGrowTX - 1 + R, W - 1);
    const int r0 = ylo / kSumTY, c0 = xlo / kSumTX;
    const int ncol = xhi / kSumTX - c0 + 1;
    bool hit = false;
    if (lane < (yhi / kSumTY - r0 + 1) * ncol) {
        const int r = r0 + lane / ncol, c = c0 + lane % ncol, top = r * kSumTY;
        const int lo = max(ylo, top) - top, hi = min(yhi, top + kSumTY - 1) - top;
        const uint32_t q = reinterpret_cast<const uint32_t *>(f.tile_first)
                               [r * ((W + kSumTX - 1) / kSumTX) + c];
        if (hi <= 1)
            hit = ((q & 0xFFu) & 2u) != 0u;                 // rows 0-1 of the tile
        else if (lo >= kSumTY - 2)
            hit = (((q >> 24) & 0xFFu) & 4u) != 0u;         // rows 30-31
        else
            for (int b = lo >> 3; b <= hi >> 3; ++b)       // bytes of 8 rows
                hit |= ((q >> (8 * b)) & 1u) != 0u;
    }
    return __ballot(hit) != 0ull;
}

// LDS of one wave of the fused kernel: M_k and G2 for rows y0-2 .. y0+TYG+1, 16 bits per
// lane and row (bit b of lane l: pixel x0 - 16 + 16 l + b), and the candidate list.
template <int TYG>
struct FusedLds {
    uint16_t m[(TYG + 4) * 64];
    uint16_t g[(TYG + 4) * 64];
    uint32_t list[kFusedList];
};

// The wave's LDS writes visible to all of its lanes before they are read.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// 16 flag bytes (bit 0 of each) -> 16 bits
__device__ __forceinline__ uint32_t squeeze16(const Px16 &v) {
    return squeeze4(v.d[0]) | (squeeze4(v.d[1]) << 4) | (squeeze4(v.d[2]) << 8) |
           (squeeze4(v.d[3]) << 12);
}

template <int TYG, bool ALIGNED>
__device__ __forceinline__ void grow_replace_strip(const DevFrame &f, int y0, int x0, int k,
                                                   int lane, FusedLds<TYG> &sh) {
    constexpr int kAhead = 4;
    constexpr int NR = TYG + 8;                 // code rows streamed: y0-4 .. y0+TYG+3
    const int H = f.H, W = f.W;
    const bool fresh = k == 1 && (f.flags & kFreshMask);
    const int px = x0 - 16 + 16 * lane;
    const bool owner = lane >= 1 && lane <= kGrowTX / 16 && px < W;
    // a candidate needs a pixel of G2 within 2 pixels (or, at iteration 1, is one), and
    // G2 lies within 2 of A: no A within 4 of the strip means nothing to do
    if ((k >= 2 || fresh) && f.tile_first && !strip_near_first_r<TYG, 4>(f, y0, x0, lane))
        return;

    Px16 hA0 = {}, hA1 = {}, hi1 = {}, lo1 = {}, lo2 = {}, hG0 = {}, hG1 = {};
    unsigned int nnew = 0;
    Px16 cring[kAhead];
    if constexpr (ALIGNED) {
#pragma unroll
        for (int t = 0; t < kAhead; ++t)
            cring[t] = load16_aligned(f.codes, y0 - 4 + t, px, H, W);
    }
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        const int y = y0 - 4 + t;
        Px16 c;
        if constexpr (ALIGNED) {
            c = cring[t % kAhead];
            if (t + kAhead < NR)
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
        Px16 g1;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            g1.d[q] = (hA0.d[q] | hA1.d[q] | hA2.d[q]) & hi1.d[q];
        const Px16 hG2 = hdilate(g1);
        if (t >= 4) {
            const int r = t - 6;                        // output row y0 + r == y - 2
            const int yr = y - 2;
            Px16 g2;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                g2.d[q] = (hG0.d[q] | hG1.d[q] | hG2.d[q]) & lo2.d[q];
            Px16 mp = {};
            if (!fresh) {
                if constexpr (ALIGNED)
                    mp = load16_aligned(f.mask, yr, px, H, W);
                else
                    mp = load16(f.mask, yr, px, H, W, false);
            }
            Px16 m;
            uint32_t anynew = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t nw = g2.d[q] & ~mp.d[q];
                m.d[q] = mp.d[q] | g2.d[q];
                anynew |= nw;
                if (r >= 0 && r < TYG)
                    nnew += owner && yr < H ? (unsigned int)__popc(nw) : 0u;
            }
            if (r >= 0 && r < TYG && owner && yr < H && anynew)
                store16(f.mask, yr, px, W, ALIGNED, m);
            sh.m[(r + 2) * 64 + lane] = (uint16_t)squeeze16(m);
            sh.g[(r + 2) * 64 + lane] = (uint16_t)squeeze16(g2);
        }
        hA0 = hA1; hA1 = hA2;
        lo2 = lo1; lo1 = lo0;
        hi1 = hi2;
        hG0 = hG1; hG1 = hG2;
    }
    const unsigned int tn = __ockl_wfred_add_u32(nnew);
    if (tn && lane == 0)
        atomicAdd(&f.nnew[k - 1], (unsigned long long)tn);
    wave_lds_sync();

    // candidates of the owned rows, 16 bits per lane and row
    uint32_t cbits[(TYG + 1) / 2];
    unsigned int ncand = 0;
#pragma unroll
    for (int r = 0; r < TYG; ++r) {
        uint32_t c16 = owner && y0 + r < H ? (uint32_t)sh.m[(r + 2) * 64 + lane] : 0u;
        if (k >= 2) {
            uint32_t v = 0u, vp = 0u, vn = 0u;           // G2 of rows r-2 .. r+2
#pragma unroll
            for (int d = 0; d <= 4; ++d) {
                v |= sh.g[(r + d) * 64 + lane];
                vp |= sh.g[(r + d) * 64 + (lane > 0 ? lane - 1 : 0)];
                vn |= sh.g[(r + d) * 64 + (lane < 63 ? lane + 1 : 63)];
            }
            const uint32_t d5 = (v | (v << 1) | (v << 2) | (v >> 1) | (v >> 2) | (vp >> 14) |
                                 (vp >> 15) | (vn << 15) | (vn << 14)) & 0xFFFFu;
            c16 &= d5;
        }
        if (r & 1)
            cbits[r >> 1] |= c16 << 16;
        else
            cbits[r >> 1] = c16;
        ncand += (unsigned int)__popc(c16);
    }
    const unsigned int incl = wave_incl_scan(ncand, lane);
    const unsigned int total = (unsigned int)__builtin_amdgcn_readlane((int)incl, 63);
    const unsigned int excl = incl - ncand;
    for (unsigned int base = 0; base < total; base += kFusedList) {
        // this round's candidates: the lanes' entries base .. base + kFusedList - 1
        unsigned int at = excl;
#pragma unroll
        for (int r = 0; r < TYG; ++r) {
            uint32_t c16 = (cbits[r >> 1] >> (16 * (r & 1))) & 0xFFFFu;
            while (c16) {
                const int b = __ffs(c16) - 1;
                if (at >= base && at < base + kFusedList)
                    sh.list[at - base] = ((uint32_t)r << 10) | (uint32_t)(16 * lane + b);
                ++at;
                c16 &= c16 - 1u;
            }
        }
        wave_lds_sync();
        const unsigned int nround = min(total - base, (unsigned int)kFusedList);
        for (unsigned int e = (unsigned int)lane; e < nround; e += 64) {
            const uint32_t ent = sh.list[e];
            const int r = (int)(ent >> 10), cx = (int)(ent & 1023u);
            const int y = y0 + r, x = x0 - 16 + cx;
            float v[25];
            uint32_t fl = 0u;
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
                const int yy = clampi(y + dy, H);
                const uint16_t *mrow = &sh.m[(yy - y0 + 2) * 64];
                const size_t row = (size_t)yy * W;
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx) {
                    const int xx = clampi(x + dx, W);
                    const int c = xx - (x0 - 16);
                    v[(dy + 2) * 5 + dx + 2] = f.J[row + xx];
                    fl |= ((mrow[c >> 4] >> (c & 15)) & 1u) << ((dy + 2) * 5 + dx + 2);
                }
            }
            replace_from_window(f, y, x, v, fl, k);
        }
        wave_lds_sync();       // the list is rewritten in the next round
    }
}

template <int TYG>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_grow_replace(
    const DevFrame *__restrict__ frames, const TileRef *__restrict__ tiles, DevFrame single,
    int kiter, int ntiles) {
    __shared__ FusedLds<TYG> sLds[kThreads / 64];
    const int lane = threadIdx.x & 63;
    const int wt = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (wt >= ntiles)
        return;
    DevFrame f;
    int y0, x0;
    if (tiles) {
        constexpr int kSub = kGrowTY / TYG;
        const TileRef t = tiles[wt / kSub];
        f = frames[t.frame];
        y0 = t.y0 + (wt % kSub) * TYG;
        x0 = t.x0;
        if (y0 >= f.H)
            return;
    } else {
        f = single;
        const int ntx = (f.W + kGrowTX - 1) / kGrowTX;
        y0 = (wt / ntx) * TYG;
        x0 = (wt % ntx) * kGrowTX;
    }
    const int k = kiter ? kiter : f.k;
    if (frame_skips(f, k))
        return;
    FusedLds<TYG> &sh = sLds[threadIdx.x >> 6];
    if ((f.W & 15) == 0)
        grow_replace_strip<TYG, true>(f, y0, x0, k, lane, sh);
    else
        grow_replace_strip<TYG, false>(f, y0, x0, k, lane, sh);
}

// ---------------------------------------------------------------------------
// init and stats
// ---------------------------------------------------------------------------

// Grid rows (blockIdx.y) take the frames in turn.
__global__ __launch_bounds__(kThreads) void k_init(const DevFrame *__restrict__ frames,
                                                   int nframes, DevFrame single,
                                                   unsigned int *__restrict__ tickets,
                                                   int nticket) {
    const size_t gid = (size_t)blockIdx.x * kThreads + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * kThreads;
    // the persistent launches' ticket counters start at zero on every run
    if (tickets && blockIdx.y == 0)
        for (size_t i = gid; i < (size_t)nticket; i += stride)
            tickets[i] = 0u;
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

// A copy by 4-byte buffer loads and stores, one element per lane in consecutive order
// (the detection stages J with the same 4-byte buffer loads): its HBM counter readings
// against its known byte count calibrate the counters for that access width.  Blocks
// take 2^20-element chunks (each within one buffer resource, below 2^32 bytes).
__global__ __launch_bounds__(kThreads) void k_debug_copy_b32(const float *__restrict__ src,
                                                             float *__restrict__ dst,
                                                             long long n) {
    constexpr long long kChunk = 1ll << 20;
    const long long nchunks = (n + kChunk - 1) / kChunk;
    for (long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const long long base = c * kChunk;
        const long long len = n - base < kChunk ? n - base : kChunk;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(src + base), (short)0, (int)(len * 4), 0x00020000);
        const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(dst + base), (short)0, (int)(len * 4), 0x00020000);
        for (int i = threadIdx.x; i < (int)len; i += kThreads) {
            const unsigned int v = __builtin_amdgcn_raw_buffer_load_b32(rs, i * 4, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(v, rd, i * 4, 0, 0);
        }
    }
}

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
                       size_t max_pixels, unsigned int *tickets, int nticket, hipStream_t s) {
    const int rows = d_frames ? (nframes < 65535 ? nframes : 65535) : 1;
    const unsigned int cap = 4096u / (unsigned int)rows > 16u ? 4096u / (unsigned int)rows : 16u;
    size_t items = max_pixels > (size_t)kMaxIter ? max_pixels : (size_t)kMaxIter;
    items = items > (size_t)nticket ? items : (size_t)nticket;
    const unsigned int gx = grid_for(items, cap);
    k_init<<<dim3(gx, rows), kThreads, 0, s>>>(d_frames, nframes, single, tickets, nticket);
    return hipGetLastError();
}

hipError_t launch_list_prefix(const DevFrame *d_frames, int nframes, int k,
                              unsigned int *d_prefix, hipStream_t s) {
    k_list_prefix<<<1, kThreads, 0, s>>>(d_frames, nframes, k, d_prefix);
    return hipGetLastError();
}

// Strip height of a grow launch: the configured first-iteration height (default: 32 rows
// for batches and frames of 2^22 pixels or more, 8 below), 8 rows after iteration 1,
// where few strips are near A and each runs alone, so a shorter row chain is waited on.
static int grow_height(bool batch, const DevFrame &single, int k, const LaunchCfg &cfg) {
    if (k >= 2)
        return kGrowTYSmall;
    if (cfg.grow_h)
        return cfg.grow_h;
    if (batch)
        return kGrowTY;
    return (size_t)single.H * single.W < ((size_t)1 << 22) ? kGrowTYSmall : kGrowTY;
}

hipError_t launch_grow(const DevFrame *d_frames, const TileRef *d_tiles, int ntiles,
                       const DevFrame &single, int k, bool fresh, const LaunchCfg &cfg,
                       hipStream_t s) {
    constexpr int wpb = kThreads / 64;
    if (d_tiles && ntiles <= 0)
        return hipSuccess;
    // serving launches (k == 0) mix iterations: the first-iteration height for all.  The
    // fused kernel runs 8-row strips (taller ones would hold their rows in registers
    // beyond the 168 a wave may have at 3 waves per SIMD).
    const bool fused = cfg.fused && !single.g2;
    const int ty = fused ? kGrowTYSmall : grow_height(d_tiles != nullptr, single, k, cfg);
    int n;
    if (d_tiles)
        n = ntiles * (kGrowTY / ty);          // a listed 32-row strip splits into kGrowTY / ty
    else
        n = ((single.W + kGrowTX - 1) / kGrowTX) * ((single.H + ty - 1) / ty);
    const unsigned int grid = (unsigned int)((n + wpb - 1) / wpb);
    if (fused) {
        k_grow_replace<kGrowTYSmall><<<grid, kThreads, 0, s>>>(d_frames, d_tiles, single, k, n);
    } else {
        fresh = fresh && k == 1;
        switch (ty) {
        case 8:
            if (fresh)
                k_grow<8, true><<<grid, kThreads, 0, s>>>(d_frames, d_tiles, single, k, n);
            else
                k_grow<8, false><<<grid, kThreads, 0, s>>>(d_frames, d_tiles, single, k, n);
            break;
        case 16:
            if (fresh)
                k_grow<16, true><<<grid, kThreads, 0, s>>>(d_frames, d_tiles, single, k, n);
            else
                k_grow<16, false><<<grid, kThreads, 0, s>>>(d_frames, d_tiles, single, k, n);
            break;
        case 32:
            if (fresh)
                k_grow<32, true><<<grid, kThreads, 0, s>>>(d_frames, d_tiles, single, k, n);
            else
                k_grow<32, false><<<grid, kThreads, 0, s>>>(d_frames, d_tiles, single, k, n);
            break;
        default:
            return hipErrorInvalidValue;
        }
    }
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

hipError_t launch_debug_copy_b32(const float *src, float *dst, long long n, hipStream_t s) {
    if (n <= 0)
        return hipSuccess;
    const long long nchunks = (n + (1ll << 20) - 1) >> 20;
    k_debug_copy_b32<<<(unsigned int)(nchunks < 4096 ? nchunks : 4096), kThreads, 0, s>>>(src,
                                                                                        dst, n);
    return hipGetLastError();
}

hipError_t launch_debug_fp64(const double *x, const double *y, int n, double *out_sqrt,
                             double *out_div, hipStream_t s) {
    k_debug_fp64<<<(n + kThreads - 1) / kThreads, kThreads, 0, s>>>(x, y, n, out_sqrt, out_div);
    return hipGetLastError();
}

}  // namespace crb
