// Swapping (section "Swapping"): the device keeps a pool of voxel blocks
// smaller than the map; blocks that leave the view move to the host, and a host
// copy comes back into the device block a block takes when it is visible again,
// merged with what the device fused into it meanwhile (the secondary
// integration).  The host decides which blocks move (fixed transfer sizes, in
// key order); these kernels find the candidates, move the voxels through the
// device side of the transfer buffers and keep the pool.
#include <algorithm>

#include "itm_internal.hpp"

namespace itm {

// One thread per hash entry: the candidates of this frame's transfers.
//   swap in:  entries holding a device block and a host copy not yet merged;
//   swap out: entries holding a device block, nothing to merge, not listed in
//             this frame (stamp != stamp_now).
// Each list gets (entry, key) records; counts in cnt[0] (in) and cnt[1] (out).
// Thread 0 also resets a pool top that the allocation ran below zero.
__global__ __launch_bounds__(256) void k_swap_scan(SwapScanArgs a)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && *a.pool.top < 0) *a.pool.top = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.n_entries; e += stride) {
        const int32_t b = a.h.blk[e];
        if (b < 0) continue;
        const bool on_host = a.onhost[e] != 0;
        if (!on_host && a.stamp[e] == a.stamp_now) continue;   // visible, nothing to merge
        const unsigned long long key = entry_key(a.h, (int32_t)e);
        const int which = on_host ? 0 : 1;
        const int32_t pos = atomicAdd(&a.cnt[which], 1);
        SwapRec r;
        r.key = key;
        r.e = (int32_t)e;
        r.pad = 0;
        (which ? a.out_list : a.in_list)[pos] = r;
    }
}

hipError_t launch_swap_scan(const SwapScanArgs &a, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>((a.n_entries + 255) / 256, 8192);
    k_swap_scan<<<std::max(grid, 1), 256, 0, st>>>(a);
    return hipGetLastError();
}

// Swap in: one workgroup per block; the host copy (storage form, in the
// transfer buffer) merges into the entry's device block:
//   W = W_d + W_h; F = (W_d F_d + W_h F_h) / W, W = min(W, max_w)
// (unchanged when both weights are 0); the entry has nothing left to merge.
template <int FMT>
__global__ __launch_bounds__(256) void k_swap_merge(SwapMoveArgs a)
{
    using V = Vox<FMT>;
    auto *sdf = (typename V::S *)a.sdf;
    auto *w = (typename V::Wt *)a.w;
    const auto *ts = (const typename V::S *)a.xfer_sdf;
    const auto *tw = (const typename V::Wt *)a.xfer_w;
    for (int i = blockIdx.x; i < a.n; i += gridDim.x) {
        const int32_t e = a.entries[i];
        const int32_t b = a.h.blk[e];
        for (int l = threadIdx.x; l < kBlockVox; l += blockDim.x) {
            const int64_t d = (int64_t)b * kBlockVox + l, x = (int64_t)i * kBlockVox + l;
            const float Fd = V::to_f(sdf[d]), Wd = V::w_to_f(w[d]);
            const float Fh = V::to_f(ts[x]), Wh = V::w_to_f(tw[x]);
            const float Wn = Wd + Wh;
            if (Wn > 0.0f) {
                sdf[d] = V::from_f((Wd * Fd + Wh * Fh) / Wn);
                w[d] = V::w_from_f(fminf(Wn, a.max_w));
            }
        }
        if (threadIdx.x == 0) a.onhost[e] = 0;
    }
}

// Swap out: one workgroup per block; the device block's voxels go to the
// transfer buffer, the block is reset (F = 1, W = 0) and returned to the pool,
// and the entry now has its data on the host only.
template <int FMT>
__global__ __launch_bounds__(256) void k_swap_out(SwapMoveArgs a)
{
    using V = Vox<FMT>;
    auto *sdf = (typename V::S *)a.sdf;
    auto *w = (typename V::Wt *)a.w;
    auto *ts = (typename V::S *)a.xfer_sdf;
    auto *tw = (typename V::Wt *)a.xfer_w;
    const auto one = V::from_f(1.0f);
    const auto zero = V::w_from_f(0.0f);
    for (int i = blockIdx.x; i < a.n; i += gridDim.x) {
        const int32_t e = a.entries[i];
        const int32_t b = a.h.blk[e];
        for (int l = threadIdx.x; l < kBlockVox; l += blockDim.x) {
            const int64_t d = (int64_t)b * kBlockVox + l, x = (int64_t)i * kBlockVox + l;
            ts[x] = sdf[d];
            tw[x] = w[d];
            sdf[d] = one;
            w[d] = zero;
        }
        __syncthreads();   // the block's voxels are read and reset before it is handed out
        if (threadIdx.x == 0) {
            a.pool.stack[atomicAdd(a.pool.top, 1)] = b;
            a.h.blk[e] = -1;
            a.onhost[e] = 1;
        }
    }
}

hipError_t launch_swap_move(int fmt, bool out, const SwapMoveArgs &a, hipStream_t st)
{
    const int grid = std::max(1, std::min(a.n, 4096));
    if (a.n <= 0) return hipSuccess;
    switch (fmt * 2 + (out ? 1 : 0)) {
    case 2 * ITM_VOX_F32: k_swap_merge<ITM_VOX_F32><<<grid, 256, 0, st>>>(a); break;
    case 2 * ITM_VOX_F32 + 1: k_swap_out<ITM_VOX_F32><<<grid, 256, 0, st>>>(a); break;
    case 2 * ITM_VOX_F16: k_swap_merge<ITM_VOX_F16><<<grid, 256, 0, st>>>(a); break;
    case 2 * ITM_VOX_F16 + 1: k_swap_out<ITM_VOX_F16><<<grid, 256, 0, st>>>(a); break;
    case 2 * ITM_VOX_S16U8: k_swap_merge<ITM_VOX_S16U8><<<grid, 256, 0, st>>>(a); break;
    default: k_swap_out<ITM_VOX_S16U8><<<grid, 256, 0, st>>>(a); break;
    }
    return hipGetLastError();
}

// pool initialisation: every device block free, no entry holding one
__global__ void k_swap_init(int32_t *stack, int32_t n_blocks, int32_t *top, int32_t *blk, uint8_t *onhost,
                            int64_t n_entries)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < n_blocks; i += stride) stack[i] = (int32_t)i;
    for (int64_t i = t0; i < n_entries; i += stride) {
        blk[i] = -1;
        onhost[i] = 0;
    }
    if (t0 == 0) *top = n_blocks;
}

hipError_t launch_swap_init(int32_t *stack, int32_t n_blocks, int32_t *top, int32_t *blk, uint8_t *onhost,
                            int64_t n_entries, hipStream_t st)
{
    k_swap_init<<<2048, 256, 0, st>>>(stack, n_blocks, top, blk, onhost, n_entries);
    return hipGetLastError();
}

}  // namespace itm
