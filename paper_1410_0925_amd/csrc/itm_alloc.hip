// Allocation (section "Allocation", stages one to three) and scene initialisation.
//
// k_alloc: one thread per pixel, 16x16 pixel tiles per workgroup so that the
// lanes of a wave walk neighbouring rays and hit the same buckets.  Per valid
// pixel: binary64 band-segment end points, binary32 walk over the blocks the
// segment crosses, and for every block a lookup or a lock-free insertion:
//   * bucket slots are claimed with a 64-bit compare-and-swap of the key word, so
//     two lanes inserting the same block agree on one slot and a key can never
//     land in a slot once an earlier slot of its bucket holds it;
//   * when both slots hold other keys, the block is claimed in a per-frame set
//     (compare-and-swap, open addressing); only the claimant takes an excess entry
//     and a voxel block and links the entry at the end of the bucket's chain with
//     a compare-and-swap on the last `next` field, so no excess entry is wasted on
//     a block several lanes race for and no lane ever waits on another;
//   * a block whose excess claim finds the list exhausted is dropped and counted
//     once per frame.
// The paper's stages two (reserve a voxel block) and three (visible list) are the
// atomic pop at a winning claim and the flag scan at the start of k_integrate.
#include "itm_internal.hpp"

namespace itm {

// one visited block: find it, or insert it; return the entry id to flag, or -1
__device__ static int32_t find_or_insert(const AllocArgs &a, int bx, int by, int bz)
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
        int32_t x = __hip_atomic_load(&B->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
            B->ptr[i] = atomicAdd(&a.cnt->vba_next, 1);
            if (i == 0) atomicOr(&h.occ[b >> 5], 1u << (b & 31));  // slot 0 fills first
            const uint32_t m = macro_index(bx, by, bz);
            atomicOr(&h.macro[m >> 5], 1u << (m & 31));
            const uint32_t f = bfilt_index(bx, by, bz);
            atomicOr(&h.bfilt[f >> 5], 1u << (f & 31));
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
    a.set_list[atomicAdd(&a.cnt->set_used[a.parity], 1)] = (int32_t)slot;
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
    E->ptr = atomicAdd(&a.cnt->vba_next, 1);
    {
        const uint32_t m = macro_index(bx, by, bz);
        atomicOr(&h.macro[m >> 5], 1u << (m & 31));
        const uint32_t f = bfilt_index(bx, by, bz);
        atomicOr(&h.bfilt[f >> 5], 1u << (f & 31));
    }
    // link at the end of the chain; every failed compare-and-swap means another
    // claimant linked first, so the walk moves on and terminates
    int32_t *loc = &B->head;
    for (;;) {
        const int32_t old = atomicCAS(loc, -1, x);
        if (old == -1) break;
        loc = &h.excess[old].next;
    }
    return 2 * h.n_buckets + x;
}

__global__ __launch_bounds__(256) void k_alloc(AllocArgs a)
{
    const FrameGeom &g = a.fg;
    if (blockIdx.x == 0) {
        // per-frame counters, filled by k_integrate
        if (threadIdx.x < kStripes) {
            a.cnt->upd[0][threadIdx.x][0] = 0;
            a.cnt->vis[0][threadIdx.x][0] = 0;
        }
    }
    int tx, ty;
    if (!xcd_tile((g.W + 15) / 16, (g.H + 15) / 16, tx, ty)) return;
    const int u = tx * 16 + (threadIdx.x & 15);
    const int v = ty * 16 + (threadIdx.x >> 4);
    if (u >= g.W || v >= g.H) return;
    const float depth = a.depth[(int64_t)v * g.W + u];
    if (!(depth > 0.0f) || isinf(depth)) return;

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
    for (;;) {
        const int32_t e = find_or_insert(a, b[0], b[1], b[2]);
        if (e >= 0) a.vis[e] = 1;
        if (n[0] + n[1] + n[2] == 0) break;
        int c = -1;
#pragma unroll
        for (int q = 0; q < 3; q++)
            if (n[q] > 0 && (c < 0 || t[q] < t[c])) c = q;
        b[c] += st[c];
        n[c]--;
        if (n[c] > 0) t[c] = ((float)(b[c] + (st[c] > 0 ? 1 : 0)) - P0[c]) / D[c];
    }
}

hipError_t launch_alloc(const AllocArgs &a, hipStream_t st)
{
    k_alloc<<<xcd_grid(((a.fg.W + 15) / 16) * ((a.fg.H + 15) / 16)), 256, 0, st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// initialisation: empty hash entries, zero flags and counters, fresh voxels
// (F = 1, W = 0 -- the paper's initial voxel value)
// ---------------------------------------------------------------------------
template <int FMT>
__global__ void k_init_vba(typename Vox<FMT>::S *sdf, typename Vox<FMT>::Wt *w, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const auto one = Vox<FMT>::from_f(1.0f);
    const auto zero = Vox<FMT>::w_from_f(0.0f);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        sdf[i] = one;
        w[i] = zero;
    }
}

__global__ void k_init_hash(Bucket *b, int64_t nb, Excess *x, int64_t nx, uint8_t *vis, int64_t nvis,
                            unsigned long long *set, int64_t nset, uint32_t *occ, int64_t nocc,
                            Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < nb; i += stride) {
        b[i].key[0] = b[i].key[1] = 0ull;
        b[i].ptr[0] = b[i].ptr[1] = -2;
        b[i].head = -1;
        b[i].pad = 0;
    }
    for (int64_t i = t0; i < nx; i += stride) {
        x[i].key = 0ull;
        x[i].ptr = -2;
        x[i].next = -1;
    }
    for (int64_t i = t0; i < nvis; i += stride) vis[i] = 0;
    for (int64_t i = t0; i < nset; i += stride) set[i] = 0ull;
    for (int64_t i = t0; i < nocc; i += stride) occ[i] = 0u;
    if (t0 == 0) {
        Counters z = {};
        *cnt = z;
    }
}

hipError_t launch_init(Bucket *b, int64_t nb, Excess *x, int64_t nx, uint8_t *vis, int64_t nvis,
                       unsigned long long *set, int64_t nset, uint32_t *occ, int64_t nocc,
                       Counters *cnt, int fmt, void *sdf, void *w, int64_t n_vox, hipStream_t st)
{
    k_init_hash<<<2048, 256, 0, st>>>(b, nb, x, nx, vis, nvis, set, nset, occ, nocc, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (fmt) {
    case ITM_VOX_F32:
        k_init_vba<ITM_VOX_F32><<<8192, 256, 0, st>>>((float *)sdf, (float *)w, n_vox);
        break;
    case ITM_VOX_F16:
        k_init_vba<ITM_VOX_F16><<<8192, 256, 0, st>>>((__half *)sdf, (__half *)w, n_vox);
        break;
    default:
        k_init_vba<ITM_VOX_S16U8><<<8192, 256, 0, st>>>((int16_t *)sdf, (uint8_t *)w, n_vox);
        break;
    }
    return hipGetLastError();
}

}  // namespace itm
