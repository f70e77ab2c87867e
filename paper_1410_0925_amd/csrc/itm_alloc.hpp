// Allocation (section "Allocation", stages one and two) and the visible list
// (stage three): device code of the fused per-frame kernel in itm_integrate.hip.
//
// One thread per pixel, 16x16 pixel tiles per workgroup so that the lanes of a
// wave walk neighbouring rays and hit the same buckets.  Per valid pixel:
// binary64 band-segment end points, binary32 walk over the blocks the segment
// crosses, each block's key claimed in the workgroup's LDS set, and for every key
// the workgroup claims first, a lookup or a lock-free insertion by that one lane:
//   * bucket slots are claimed with a 64-bit compare-and-swap of the key word, so
//     two lanes inserting the same block agree on one slot and a key can never
//     land in a slot once an earlier slot of its bucket holds it;
//   * when both slots hold other keys, the block is claimed in a per-frame set
//     (compare-and-swap, open addressing); only the claimant takes an excess entry
//     and links it at the end of the bucket's chain with a compare-and-swap on
//     the last `next` field, so no excess entry is wasted on a block several lanes
//     race for and no lane ever waits on another;
//   * a block whose excess claim finds the list exhausted is dropped and counted
//     once per frame.
// The paper's stage two (reserve a voxel block) is implicit: every entry owns the
// voxel block at its own index, so a winning claim is the whole insertion.  For
// stage three the workgroup stamps each block of its LDS set with the frame
// number (an atomic exchange: the first workgroup to stamp a block owns it for
// the frame).
#pragma once

#include "itm_internal.hpp"

namespace itm {

// Housekeeping of the kernel that opens a frame (the allocation, or a volume
// import), every workgroup its share: the other parity's counters and list
// counters, the next frame's claim count, the previous frame's claim slots (su
// of them, read from *a.set_used_prev by the caller) and, with the search range
// on, the other parity's bin counts are cleared.  Nothing the frame's kernel
// itself uses is cleared, so the stores may go out at any point of it.
__device__ inline void frame_housekeeping(const FuseArgs &a, int su)
{
    if (blockIdx.x == 0) {
        if (threadIdx.x < kStripes) {
            a.cnt->upd[a.parity ^ 1][threadIdx.x][0] = 0;
            a.cnt->vis[a.parity ^ 1][threadIdx.x][0] = 0;
        }
        if (threadIdx.x == 0) a.cnt->unbinned[a.parity ^ 1][0] = 0;
        if (threadIdx.x < kListSegs) a.list_clear[32 * threadIdx.x] = 0;
        if (threadIdx.x == 0) *a.set_used_next = 0;
    }
    const int gt = blockIdx.x * blockDim.x + threadIdx.x, gs = gridDim.x * blockDim.x;
    for (int i = gt; i < su; i += gs) a.set_prev[a.set_list_prev[i]] = 0ull;
    if (a.rb_clear)
        for (int i = gt; i < a.n_clear; i += gs) a.rb_clear[i] = 0;
}

// one visited block: find it, or insert it; return the entry id to list, or -1
__device__ inline int32_t find_or_insert(const FuseArgs &a, int bx, int by, int bz)
{
    const HashView &h = a.h;
    const unsigned long long key = pack_key(bx, by, bz);
    const uint32_t b = hash_index(bx, by, bz, h.mask);
    Bucket *B = h.buckets + b;
    // fast path: plain reads; keys are never changed once written, so a match is
    // final, and a stale empty slot is corrected by the compare-and-swap below
    const ulonglong2 k2 = *reinterpret_cast<const ulonglong2 *>(B->key);
    if (k2.x == key) return 2 * (int32_t)b;
    if (k2.y == key) return 2 * (int32_t)b + 1;
    if (k2.x != 0ull && k2.y != 0ull) {
        int32_t x = __hip_atomic_load(&h.head[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (x >= 0) {
            const Excess *E = h.excess + x;
            if (__hip_atomic_load(&E->key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == key) return 2 * h.n_buckets + x;
            x = __hip_atomic_load(&E->next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // insertion into the ordered part
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const unsigned long long old = atomicCAS(&B->key[i], 0ull, key);
        if (old == 0ull) {
            atomicAdd(&a.cnt->vba_next, 1);   // the block is the entry's own (count only)
            if (i == 0) atomicOr(&h.occ[b >> 5], 1u << (b & 31));  // slot 0 fills first
            const uint32_t m = macro_index(bx, by, bz);
            atomicOr(&h.macro[m >> 5], 1u << (m & 31));
            return 2 * (int32_t)b + i;
        }
        if (old == key) return 2 * (int32_t)b + i;
    }
    // the bucket holds two other blocks: claim this block for the excess list
    uint32_t slot = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 32) & a.set_mask;
    for (uint32_t probe = 0;; probe++) {
        if (probe > a.set_mask) {  // claim set full (more distinct claims in one frame
                                   // than it holds): dropped, counted per lane
            atomicAdd(&a.cnt->dropped_total, 1ull);
            return -1;
        }
        const unsigned long long old = atomicCAS(&a.set[slot], 0ull, key);
        if (old == 0ull) break;
        if (old == key) return -1;  // claimed by another lane, which flags it
        slot = (slot + 1) & a.set_mask;
    }
    a.set_list[atomicAdd(a.set_used, 1)] = (int32_t)slot;
    // Earlier frames' chain entries were all seen by the walk above; entries
    // linked during this frame belong to other claimed blocks.  So the block is
    // absent: take an excess entry.
    const int32_t x = atomicAdd(&a.cnt->excess_next, 1);
    if (x >= h.n_excess) {
        atomicAdd(&a.cnt->dropped_total, 1ull);
        return -1;
    }
    Excess *E = h.excess + x;
    E->key = key;
    atomicAdd(&a.cnt->vba_next, 1);
    {
        const uint32_t m = macro_index(bx, by, bz);
        atomicOr(&h.macro[m >> 5], 1u << (m & 31));
    }
    // link at the end of the chain; every failed compare-and-swap means another
    // claimant linked first, so the walk moves on and terminates
    int32_t *loc = &h.head[b];
    for (;;) {
        const int32_t old = atomicCAS(loc, -1, x);
        if (old == -1) break;
        loc = &h.excess[old].next;
    }
    return 2 * h.n_buckets + x;
}

constexpr int kSet = 2048;   // LDS set of the blocks one workgroup visits (8 slots per thread)

// Claim a block key in the workgroup's set: the slot, and whether this lane put
// the key there (its owner: the one lane that probes the hash table for it);
// -1 when the set is full.  Empty slots hold key 0 (no valid key is 0).
__device__ __forceinline__ int set_claim(unsigned long long *s_k, unsigned long long key, bool &owner)
{
    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 53);   // 11 bits: kSet slots
#pragma unroll 1
    for (int probe = 0; probe < kSet; probe++, h = (h + 1) & (kSet - 1)) {
        const unsigned long long old = atomicCAS(&s_k[h], 0ull, key);
        if (old == 0ull || old == key) {
            owner = old == 0ull;
            return (int)h;
        }
    }
    owner = false;
    return -1;
}

// Expected-depth rectangles of the workgroup's n listed blocks at the frame's
// pose, appended to the bins of the tiles they overlap.  8 lanes per block make
// its rectangle (block_rect8), 32 blocks per pass.  The blocks a workgroup lists
// come from its own pixels, so their rectangles share tiles: the (block, tile)
// pairs are first counted per tile in an LDS table, one global atomic per
// distinct tile reserves the tile's slots, and the pairs then take consecutive
// slots (a tile that finds the table full reserves pair by pair).  tab: LDS,
// 4 * kBinTab ints (tile, pairs, cursor, base); n is uniform.  mid() runs on every
// thread between the projections and the reservations, before a barrier.
constexpr int kBinTab = 256;

__device__ __forceinline__ int bin_tab_slot(int32_t *tab, int tile, bool insert)
{
    uint32_t h = ((uint32_t)tile * 2654435761u) >> 24;   // 8 bits: kBinTab slots
#pragma unroll 1
    for (int probe = 0; probe < kBinTab; probe++, h = (h + 1) & (kBinTab - 1)) {
        const int32_t cur = insert ? atomicCAS(&tab[4 * h], -1, tile) : tab[4 * h];
        if (cur == tile || (insert && cur == -1)) return (int)h;
        if (cur == -1) return -1;   // lookup: not in the table
    }
    return -1;
}

template <typename Mid>
__device__ inline void bin_blocks(const FrameGeom &g, const RangeBins &rb, const unsigned long long *keys, int n,
                                  int32_t *tab, Mid mid)
{
    const int corner = threadIdx.x & 7;
    for (int i = threadIdx.x; i < kBinTab; i += blockDim.x) {
        tab[4 * i] = -1;
        tab[4 * i + 1] = 0;
        tab[4 * i + 2] = 0;
    }
    __syncthreads();
    // 1. rectangles; pairs counted per tile (the first pass's rectangle is kept)
    RangeRect r0;
    bool ok0 = false;
    for (int base = 0; base < n; base += 32) {   // uniform
        const int j = base + (int)(threadIdx.x >> 3);
        RangeRect r;
        const bool ok = block_rect8(g, j < n, j < n ? keys[j] : 0ull, r);
        if (base == 0) {
            r0 = r;
            ok0 = ok;
        }
        if (!ok) continue;
        int tx0, ty0, ntx, n_tiles;
        rect_tiles(r, tx0, ty0, ntx, n_tiles);
        for (int t = corner; t < n_tiles; t += 8) {
            const int slot = bin_tab_slot(tab, (ty0 + t / ntx) * rb.tw + tx0 + t % ntx, true);
            if (slot >= 0) atomicAdd(&tab[4 * slot + 1], 1);
        }
    }
    mid();
    __syncthreads();
    // 2. one reservation per distinct tile
    for (int i = threadIdx.x; i < kBinTab; i += blockDim.x) {
        const int tile = tab[4 * i];
        if (tile >= 0) tab[4 * i + 3] = atomicAdd(&rb.cnt[tile], tab[4 * i + 1]);
    }
    __syncthreads();
    // 3. the pairs take their slots
    for (int base = 0; base < n; base += 32) {   // uniform
        const int j = base + (int)(threadIdx.x >> 3);
        RangeRect r = r0;
        bool ok = ok0;
        if (base > 0) ok = block_rect8(g, j < n, j < n ? keys[j] : 0ull, r);
        if (!ok) continue;
        int tx0, ty0, ntx, n_tiles;
        rect_tiles(r, tx0, ty0, ntx, n_tiles);
        for (int t = corner; t < n_tiles; t += 8) {
            const int tile = (ty0 + t / ntx) * rb.tw + tx0 + t % ntx;
            const int slot = bin_tab_slot(tab, tile, false);
            const int pos = slot >= 0 ? tab[4 * slot + 3] + atomicAdd(&tab[4 * slot + 2], 1)
                                      : atomicAdd(&rb.cnt[tile], 1);
            if (pos < rb.cap) rb.rect[(int64_t)tile * rb.cap + pos] = r;
        }
    }
}

// one valid pixel: the blocks its band segment crosses, found or inserted,
// recorded in the workgroup's set (or, when the set is full, listed directly)
// Swapping (section "Swapping"): the one lane that lists a block in this frame
// gives it a device voxel block from the pool when it has none (a new block, or
// one whose data is on the host); with the pool empty it stays without one this
// frame (not integrated, counted).  Without swapping the entry is the block.
__device__ __forceinline__ void device_block(const FuseArgs &a, int32_t e)
{
    if (!a.pool.stack) return;
    if (a.h.blk[e] >= 0) return;
    const int32_t top = atomicSub(a.pool.top, 1) - 1;
    if (top >= 0) a.h.blk[e] = a.pool.stack[top];
    else atomicAdd(a.pool.no_block, 1ull);
}

__device__ inline void alloc_pixel(const FuseArgs &a, int u, int v, float depth, int32_t *s_e,
                            unsigned long long *s_k)
{
    const FrameGeom &g = a.fg;
    // band segment end points in block units (binary64, fixed order, no fusion)
    const double d = (double)depth;
    double z0 = d - g.mu;
    if (z0 < 0.0) z0 = 0.0;
    const double z1 = d + g.mu;
    const double rx = ((double)u - g.cxd) * g.inv_fx;
    const double ry = ((double)v - g.cyd) * g.inv_fy;
    float P0[3], P1[3];
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const double z = k ? z1 : z0;
        const double q0 = z * rx, q1 = z * ry, q2 = z;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            double w = g.Rwc[3 * c + 0] * q0;
            w = w + g.Rwc[3 * c + 1] * q1;
            w = w + g.Rwc[3 * c + 2] * q2;
            w = w + g.twc[c];
            const float P = (float)(w * g.inv_bs);
            if (!(P >= -32767.0f && P < 32767.0f)) return;
            if (k) P1[c] = P; else P0[c] = P;
        }
    }

    // blocks crossed by the segment (binary32): start at floor(P0), cross the
    // axis with the smallest next-boundary parameter (ties x, y, z), recompute
    // that axis' parameter from its new boundary
    int b[3], n[3], st[3];
    float D[3], t[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int b0 = (int)floorf(P0[c]);
        const int b1 = (int)floorf(P1[c]);
        b[c] = b0;
        n[c] = b1 > b0 ? b1 - b0 : b0 - b1;
        st[c] = b1 > b0 ? 1 : (b1 < b0 ? -1 : 0);
        D[c] = P1[c] - P0[c];
        t[c] = n[c] > 0 ? ((float)(b0 + (st[c] > 0 ? 1 : 0)) - P0[c]) / D[c] : 0.0f;
    }
    // The walk in batches of 4 blocks: the batch's bucket records are loaded
    // together (one memory round), then matched; a block not found in its bucket
    // takes the full path (chain walk, insertion).
    bool done = false;
    while (!done) {
        int cx[4], cy[4], cz[4];
        bool valid[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            valid[q] = !done;
            cx[q] = b[0];
            cy[q] = b[1];
            cz[q] = b[2];
            if (done) continue;
            if (n[0] + n[1] + n[2] == 0) {
                done = true;
                continue;
            }
            int c = -1;
#pragma unroll
            for (int r = 0; r < 3; r++)
                if (n[r] > 0 && (c < 0 || t[r] < t[c])) c = r;
            b[c] += st[c];
            n[c]--;
            if (n[c] > 0) t[c] = ((float)(b[c] + (st[c] > 0 ? 1 : 0)) - P0[c]) / D[c];
        }
        // The workgroup's pixels cross the same few blocks: each key is claimed in
        // the LDS set first, and only its owner probes the hash table and records
        // the entry in the set (a key that finds the set full is probed, stamped
        // and listed by its own lane).
        int slot4[4];
        uint32_t probe = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            slot4[q] = -1;
            if (!valid[q]) continue;
            bool owner;
            slot4[q] = set_claim(s_k, pack_key(cx[q], cy[q], cz[q]), owner);
            if (owner || slot4[q] < 0) probe |= 1u << q;
        }
        // Every lane reads its four buckets (any block's bucket is a valid
        // address; a lane that does not probe a block reads a line its owner
        // reads too) and keeps the records it probes: read under a branch, the
        // first record was waited for before the other three were issued.
        ulonglong2 k2[4];
#pragma unroll
        for (int q = 0; q < 4; q++)
            k2[q] = *reinterpret_cast<const ulonglong2 *>(a.h.buckets[hash_index(cx[q], cy[q], cz[q], a.h.mask)].key);
#pragma unroll
        for (int q = 0; q < 4; q++)
            if (!(probe & (1u << q))) k2[q] = make_ulonglong2(0ull, 0ull);   // no valid key is 0
        int32_t e4[4];
        uint32_t slow = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const unsigned long long key = pack_key(cx[q], cy[q], cz[q]);
            const int32_t bi = 2 * (int32_t)hash_index(cx[q], cy[q], cz[q], a.h.mask);
            e4[q] = k2[q].x == key ? bi : k2[q].y == key ? bi + 1 : -1;
            if ((probe & (1u << q)) && e4[q] < 0) slow |= 1u << q;
        }
        // the full path, from one call site (register selects, no indexed arrays)
        while (slow) {
            const int q = __builtin_ctz(slow);
            slow &= slow - 1;
            const int x = q == 0 ? cx[0] : q == 1 ? cx[1] : q == 2 ? cx[2] : cx[3];
            const int y = q == 0 ? cy[0] : q == 1 ? cy[1] : q == 2 ? cy[2] : cy[3];
            const int z = q == 0 ? cz[0] : q == 1 ? cz[1] : q == 2 ? cz[2] : cz[3];
            const int32_t e = find_or_insert(a, x, y, z);
#pragma unroll
            for (int r = 0; r < 4; r++)
                if (r == q) e4[r] = e;
        }
        // The batch's stamp exchanges, all issued before any is waited for: their
        // results are hidden from the compiler until all four are out, as it
        // would otherwise compare each result, and wait for it, before issuing
        // the next.  The first workgroup to stamp a block lists it.
        uint32_t old4[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            old4[q] = a.stamp_now;
            if ((probe & (1u << q)) && e4[q] >= 0) old4[q] = atomicExch(&a.stamp[e4[q]], a.stamp_now);
        }
        asm volatile("" : "+v"(old4[0]), "+v"(old4[1]), "+v"(old4[2]), "+v"(old4[3]));
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (!(probe & (1u << q))) continue;
            const int32_t e = e4[q];
            if (slot4[q] >= 0) {
                // stamped while other lanes still probe; -1 (dropped, or listed by
                // another workgroup) leaves the slot out of the list
                const bool first = e >= 0 && old4[q] != a.stamp_now;
                s_e[slot4[q]] = first ? e : -1;
                if (first) device_block(a, e);
            } else if (e >= 0 && old4[q] != a.stamp_now) {
                // the workgroup's set is full: list the block on its own; its
                // expected-depth rectangle is not binned, so the frame's bins are
                // marked incomplete (every tile then computes its range exactly
                // from the visible list)
                device_block(a, e);
                VisRec r;
                r.key = pack_key(cx[q & 3], cy[q & 3], cz[q & 3]);
                r.e = e;
                r.pad = 0;
                a.list.rec[(int64_t)32 * a.list.cap + atomicAdd(&a.list.cnt[32 * 32], 1)] = r;
                if (a.rb.unbinned) *a.rb.unbinned = 1;
            }
        }
    }
}

}  // namespace itm
