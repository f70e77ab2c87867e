// Scene initialisation (empty hash table, zero counters, fresh voxels) and the
// export gather.  The allocation itself is device code in itm_alloc.hpp, run by
// the fused per-frame kernel of itm_integrate.hip.
#include <algorithm>

#include "itm_internal.hpp"

namespace itm {

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

__global__ void k_init_hash(Bucket *b, int32_t *head, int64_t nb, Excess *x, int64_t nx, uint32_t *stamp,
                            int64_t nstamp, unsigned long long *set, int64_t nset, uint32_t *occ, int64_t nocc,
                            Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < nb; i += stride) {
        b[i].key[0] = b[i].key[1] = 0ull;
        head[i] = -1;
    }
    for (int64_t i = t0; i < nx; i += stride) {
        x[i].key = 0ull;
        x[i].next = -1;
        x[i].pad = 0;
    }
    for (int64_t i = t0; i < nstamp; i += stride) stamp[i] = 0u;
    for (int64_t i = t0; i < nset; i += stride) set[i] = 0ull;
    for (int64_t i = t0; i < nocc; i += stride) occ[i] = 0u;
    if (t0 == 0) {
        Counters z = {};
        *cnt = z;
    }
}

// export: the voxels of the listed blocks, packed in list order
template <int FMT>
__global__ __launch_bounds__(256) void k_export_gather(const typename Vox<FMT>::S *sdf,
                                                       const typename Vox<FMT>::Wt *w, const int32_t *blocks,
                                                       int64_t n, typename Vox<FMT>::S *out_sdf,
                                                       typename Vox<FMT>::Wt *out_w)
{
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t src = (int64_t)blocks[i] * kBlockVox, dst = i * kBlockVox;
        for (int l = threadIdx.x; l < kBlockVox; l += blockDim.x) {
            if (out_sdf) out_sdf[dst + l] = sdf[src + l];
            if (out_w) out_w[dst + l] = w[src + l];
        }
    }
}

hipError_t launch_export_gather(int fmt, const void *sdf, const void *w, const int32_t *blocks, int64_t n,
                                void *out_sdf, void *out_w, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(n, 1), 4096);
    switch (fmt) {
    case ITM_VOX_F32:
        k_export_gather<ITM_VOX_F32><<<grid, 256, 0, st>>>((const float *)sdf, (const float *)w, blocks, n,
                                                            (float *)out_sdf, (float *)out_w);
        break;
    case ITM_VOX_F16:
        k_export_gather<ITM_VOX_F16><<<grid, 256, 0, st>>>((const __half *)sdf, (const __half *)w, blocks, n,
                                                            (__half *)out_sdf, (__half *)out_w);
        break;
    default:
        k_export_gather<ITM_VOX_S16U8><<<grid, 256, 0, st>>>((const int16_t *)sdf, (const uint8_t *)w, blocks,
                                                              n, (int16_t *)out_sdf, (uint8_t *)out_w);
        break;
    }
    return hipGetLastError();
}

// import: the given blocks' voxels (float32 F and W, export layout) into their
// voxel blocks, converted to the storage form; one workgroup per block
template <int FMT>
__global__ __launch_bounds__(256) void k_import_voxels(const int32_t *entry, const float *in_sdf, const float *in_w,
                                                       int64_t n, typename Vox<FMT>::S *sdf,
                                                       typename Vox<FMT>::Wt *w, uchar4 *clr)
{
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int32_t e = entry[i];
        if (e < 0) continue;   // dropped
        const int64_t dst = (int64_t)e * kBlockVox, src = i * kBlockVox;
        for (int l = threadIdx.x; l < kBlockVox; l += blockDim.x) {
            sdf[dst + l] = Vox<FMT>::from_f(in_sdf[src + l]);
            w[dst + l] = Vox<FMT>::w_from_f(in_w[src + l]);
            if (clr) clr[dst + l] = make_uchar4(0, 0, 0, 0);
        }
    }
}

hipError_t launch_import_voxels(int fmt, const int32_t *entry, const float *in_sdf, const float *in_w, int64_t n,
                                void *sdf, void *w, uchar4 *clr, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(n, 1), 4096);
    switch (fmt) {
    case ITM_VOX_F32:
        k_import_voxels<ITM_VOX_F32><<<grid, 256, 0, st>>>(entry, in_sdf, in_w, n, (float *)sdf, (float *)w, clr);
        break;
    case ITM_VOX_F16:
        k_import_voxels<ITM_VOX_F16><<<grid, 256, 0, st>>>(entry, in_sdf, in_w, n, (__half *)sdf, (__half *)w, clr);
        break;
    default:
        k_import_voxels<ITM_VOX_S16U8><<<grid, 256, 0, st>>>(entry, in_sdf, in_w, n, (int16_t *)sdf, (uint8_t *)w,
                                                              clr);
        break;
    }
    return hipGetLastError();
}

// export of colour voxels: the listed blocks' 512 x 4 bytes, packed in list order
__global__ __launch_bounds__(256) void k_export_colour(const uchar4 *clr, const int32_t *blocks, int64_t n,
                                                       uchar4 *out)
{
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t src = (int64_t)blocks[i] * kBlockVox, dst = i * kBlockVox;
        for (int l = threadIdx.x; l < kBlockVox; l += blockDim.x) out[dst + l] = clr[src + l];
    }
}

hipError_t launch_export_colour(const uchar4 *clr, const int32_t *blocks, int64_t n, uchar4 *out, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(n, 1), 4096);
    k_export_colour<<<grid, 256, 0, st>>>(clr, blocks, n, out);
    return hipGetLastError();
}

hipError_t launch_init(Bucket *b, int32_t *head, int64_t nb, Excess *x, int64_t nx, uint32_t *stamp,
                       int64_t nstamp, unsigned long long *set, int64_t nset, uint32_t *occ, int64_t nocc,
                       Counters *cnt, int fmt, void *sdf, void *w, int64_t n_vox, hipStream_t st)
{
    k_init_hash<<<2048, 256, 0, st>>>(b, head, nb, x, nx, stamp, nstamp, set, nset, occ, nocc, cnt);
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
