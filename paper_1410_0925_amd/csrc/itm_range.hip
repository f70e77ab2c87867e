// Expected depth ranges (section "Raycast", the search range; the paper's
// CreateExpectedDepths): the visible blocks are forward-projected and each
// pixel gets the min and max camera depth of the block boxes covering it.
//
// The paper splits this into a fragment list (16 x 16 pixel pieces of every
// block's bounding box, counted with a prefix sum) and a render pass that
// updates per-pixel min / max with atomics.  Here every block's rectangle is
// appended to the bin of each 16 x 16 tile it overlaps (one atomic per block
// and tile, no per-pixel atomics), and the raycast's workgroup for a tile --
// which covers exactly those 16 x 16 pixels -- takes the min / max over its bin
// in registers, so the range image itself never goes through memory.  The
// allocation kernel bins at the frame's own pose as it lists each visible block;
// k_range_bin does it for a raycast at any other pose, from the visible list.
#include <algorithm>

#include "itm_internal.hpp"

namespace itm {

__global__ __launch_bounds__(256) void k_range_clear(int32_t *cnt, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) cnt[i] = 0;
}

// one thread per visible block (grid-strided over the visible list)
__global__ __launch_bounds__(256) void k_range_bin(FrameGeom g, VisList list, RangeBins rb)
{
    __shared__ int s_pre[kListSegs + 1];
    if (threadIdx.x < kWave) {
        const VisPrefix p = vis_prefix(list, threadIdx.x);
        if (threadIdx.x < kListSegs) s_pre[threadIdx.x + 1] = p.incl;
        if (threadIdx.x == 0) s_pre[0] = 0;
    }
    __syncthreads();
    const int total = s_pre[kListSegs];
    // 32 blocks per workgroup pass, 8 lanes each
    for (int base = blockIdx.x * 32; base < total; base += gridDim.x * 32) {   // uniform
        const int j = base + (int)(threadIdx.x >> 3);
        bin_block8(g, rb, j < total, j < total ? vis_item_at(list, s_pre, j).key : 0ull);
    }
}

// the range image: one workgroup per tile, row-major pixels within it
__global__ __launch_bounds__(256) void k_range_image(FrameGeom g, VisList list, RangeBins rb, float2 *zr)
{
    __shared__ RangeLds L;
    const int tx = blockIdx.x % rb.tw, ty = blockIdx.x / rb.tw;
    const int u = tx * kTile + (threadIdx.x & (kTile - 1)), v = ty * kTile + threadIdx.x / kTile;
    float zlo, zhi;
    const TileBin bin = tile_bin(rb, tx, ty);
    tile_range(g, list, rb, tx, ty, bin, u, v, L, zlo, zhi);
    if (u < g.W && v < g.H) zr[(int64_t)v * g.W + u] = make_float2(zlo, zhi);
}

hipError_t launch_range_clear(int32_t *cnt, int n, hipStream_t st)
{
    k_range_clear<<<std::max(1, std::min((n + 255) / 256, 1024)), 256, 0, st>>>(cnt, n);
    return hipGetLastError();
}

hipError_t launch_range_bin(const FrameGeom &g, const VisList &list, const RangeBins &rb, hipStream_t st)
{
    k_range_bin<<<256, 256, 0, st>>>(g, list, rb);
    return hipGetLastError();
}

hipError_t launch_range_image(const FrameGeom &g, const VisList &list, const RangeBins &rb, float2 *zr,
                              hipStream_t st)
{
    k_range_image<<<rb.tw * rb.th, 256, 0, st>>>(g, list, rb, zr);
    return hipGetLastError();
}

}  // namespace itm
