// Integration (section "Integration", computeUpdatedVoxelDepthInfo) over the
// voxels of the frame's visible blocks.
//
// One wave per visible block (the workgroups find their blocks by scanning the
// visibility flags, so no count is read back).  Lane l owns voxels 4l..4l+3 and
// 256+4l..256+4l+3 of the block,
// so every voxel load or store instruction of a wave covers one contiguous range
// (16 B per lane in the float form).  A lane reads its 8 voxels, decides for
// each whether it is updated -- that needs only the voxel's position and the
// depth image -- and writes back a group of 4 voxels only when one of them is.
//
// Decisions follow a fixed binary32 evaluation order (so that they can be
// reproduced exactly): the block origin's camera coordinates are formed in binary64
// once per block and split into a binary32 pair hi + lo; the in-block offset
// (lx g_x + ly g_y) + lz g_z is added to lo first.  The value eta = d - p_z is
// formed as (d - hi_z) - (lo_z + offset_z), accurate to ~1e-8 m at room scale.
#include "itm_internal.hpp"

namespace itm {

template <int FMT>
struct Group4;  // 4 consecutive voxels of one storage form

template <>
struct Group4<ITM_VOX_F32> {
    float4 s, w;
    __device__ void load(const void *sdf, const void *wt, int64_t i)
    {
        s = *reinterpret_cast<const float4 *>((const float *)sdf + i);
        w = *reinterpret_cast<const float4 *>((const float *)wt + i);
    }
    __device__ void store(void *sdf, void *wt, int64_t i) const
    {
        *reinterpret_cast<float4 *>((float *)sdf + i) = s;
        *reinterpret_cast<float4 *>((float *)wt + i) = w;
    }
    __device__ float F(int j) const { return j == 0 ? s.x : j == 1 ? s.y : j == 2 ? s.z : s.w; }
    __device__ float Wv(int j) const { return j == 0 ? w.x : j == 1 ? w.y : j == 2 ? w.z : w.w; }
    __device__ void set(int j, float f, float wv)
    {
        if (j == 0) { s.x = f; w.x = wv; }
        else if (j == 1) { s.y = f; w.y = wv; }
        else if (j == 2) { s.z = f; w.z = wv; }
        else { s.w = f; w.w = wv; }
    }
};

template <>
struct Group4<ITM_VOX_F16> {
    __half s[4], w[4];
    __device__ void load(const void *sdf, const void *wt, int64_t i)
    {
        const uint2 a = *reinterpret_cast<const uint2 *>((const __half *)sdf + i);
        const uint2 b = *reinterpret_cast<const uint2 *>((const __half *)wt + i);
        __builtin_memcpy(s, &a, 8);
        __builtin_memcpy(w, &b, 8);
    }
    __device__ void store(void *sdf, void *wt, int64_t i) const
    {
        uint2 a, b;
        __builtin_memcpy(&a, s, 8);
        __builtin_memcpy(&b, w, 8);
        *reinterpret_cast<uint2 *>((__half *)sdf + i) = a;
        *reinterpret_cast<uint2 *>((__half *)wt + i) = b;
    }
    __device__ float F(int j) const { return __half2float(s[j]); }
    __device__ float Wv(int j) const { return __half2float(w[j]); }
    __device__ void set(int j, float f, float wv)
    {
        s[j] = __float2half_rn(f);
        w[j] = __float2half_rn(wv);
    }
};

template <>
struct Group4<ITM_VOX_S16U8> {
    int16_t s[4];
    uint8_t w[4];
    __device__ void load(const void *sdf, const void *wt, int64_t i)
    {
        const uint2 a = *reinterpret_cast<const uint2 *>((const int16_t *)sdf + i);
        const uint32_t b = *reinterpret_cast<const uint32_t *>((const uint8_t *)wt + i);
        __builtin_memcpy(s, &a, 8);
        __builtin_memcpy(w, &b, 4);
    }
    __device__ void store(void *sdf, void *wt, int64_t i) const
    {
        uint2 a;
        uint32_t b;
        __builtin_memcpy(&a, s, 8);
        __builtin_memcpy(&b, w, 4);
        *reinterpret_cast<uint2 *>((int16_t *)sdf + i) = a;
        *reinterpret_cast<uint32_t *>((uint8_t *)wt + i) = b;
    }
    __device__ float F(int j) const { return Vox<ITM_VOX_S16U8>::to_f(s[j]); }
    __device__ float Wv(int j) const { return (float)w[j]; }
    __device__ void set(int j, float f, float wv)
    {
        s[j] = Vox<ITM_VOX_S16U8>::from_f(f);
        w[j] = (uint8_t)wv;
    }
};

// one visible block (entry e) by one wave; returns the lane's updated voxels
template <int FMT>
__device__ uint32_t integrate_block(const IntegrateArgs &a, int32_t e, int lane, unsigned long long &key_out)
{
    const FrameGeom &g = a.fg;
    unsigned long long key;
    int32_t ptr;
    entry_at(a.h, e, key, ptr);
    key_out = key;
    if (ptr < 0) return 0;  // cannot happen: every flagged entry owns a block
    int kx, ky, kz;
    unpack_key(key, kx, ky, kz);
    // block origin in camera coordinates, binary64 -> binary32 pair
    const double o0 = (double)(8 * kx) * g.s, o1 = (double)(8 * ky) * g.s, o2 = (double)(8 * kz) * g.s;
    float hi[3], lo[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        double w = g.Rcw[3 * c + 0] * o0;
        w = w + g.Rcw[3 * c + 1] * o1;
        w = w + g.Rcw[3 * c + 2] * o2;
        w = w + g.tcw[c];
        hi[c] = (float)w;
        lo[c] = (float)(w - (double)hi[c]);
    }
    const float mu = g.mu_f, inv_mu = 1.0f / mu;
    const int64_t vbase = (int64_t)ptr * kBlockVox;
    // The voxels are loaded together with the depth reads instead of after
    // them (the update decision needs only the depth image): one dependent
    // memory round less, for about 6% more voxel bytes read (whole 128-byte
    // lines are touched anyway).
    Group4<FMT> vg[2];
    vg[0].load(a.sdf, a.w, vbase + 4 * lane);
    vg[1].load(a.sdf, a.w, vbase + 4 * lane + 256);
    uint32_t n_upd = 0;
#pragma unroll
    for (int grp = 0; grp < 2; grp++) {
        const int li0 = 4 * lane + 256 * grp;
        const float fy_ = (float)((li0 >> 3) & 7), fz_ = (float)(li0 >> 6);
        float eta[4];
        uint32_t upd = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const float fx_ = (float)((li0 & 7) + j);
            float p[3], dl2 = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                float t = fx_ * g.g[0][c];
                t = t + fy_ * g.g[1][c];
                t = t + fz_ * g.g[2][c];
                p[c] = hi[c] + (lo[c] + t);
                if (c == 2) dl2 = t;
            }
            eta[j] = 0.0f;
            if (p[2] <= 0.0f) continue;
            const float x = g.fx * p[0] / p[2] + g.cx;
            const float y = g.fy * p[1] / p[2] + g.cy;
            if (x < 1.0f || x > (float)(g.W - 2) || y < 1.0f || y > (float)(g.H - 2)) continue;
            const float d = a.depth[(int)(x + 0.5f) + (int)(y + 0.5f) * g.W];
            if (!(d > 0.0f) || isinf(d)) continue;
            const float e32 = (d - hi[2]) - (lo[2] + dl2);
            if (e32 < -mu) continue;
            eta[j] = e32;
            upd |= 1u << j;
        }
        if (upd) {
            Group4<FMT> &v = vg[grp];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (!(upd & (1u << j))) continue;
                const float f = fminf(1.0f, eta[j] * inv_mu);
                const float F = v.F(j), W = v.Wv(j);
                const float Wn = W + 1.0f;
                // running average F <- (W F + f) / (W + 1), in incremental form
                const float Fn = F + (f - F) / Wn;
                v.set(j, Fn, fminf(Wn, g.max_w_f));
            }
            v.store(a.sdf, a.w, vbase + li0);
            n_upd += __builtin_popcount(upd);
        }
    }
    return n_upd;
}

constexpr int kScanThreads = 256;
constexpr int kScanEntries = kScanThreads * 8;   // flag bytes per workgroup
static_assert(kScanEntries == kSegEntries, "one visible-list segment per workgroup");

// Expected-depth rectangles of the workgroup's n visible blocks at the frame's
// pose, appended to the bins of the tiles they overlap.  8 lanes per block take
// its 8 box corners and merge them with a butterfly; 32 blocks per pass.  A
// phase of its own after the integration, so that its binary64 temporaries do
// not add to the integration's registers.
__device__ void bin_blocks(const IntegrateArgs &a, const unsigned long long *keys, int n)
{
    const FrameGeom &g = a.fg;
    const int grp = threadIdx.x >> 3, corner = threadIdx.x & 7;
    for (int base = 0; base < n; base += kScanThreads / 8) {   // uniform
        const int j = base + grp;
        BoxAcc b;
        if (j < n) {
            int kx, ky, kz;
            unpack_key(keys[j], kx, ky, kz);
            box_corner(g, kx, ky, kz, corner, b);
        } else {
            b.zlo = b.xlo = b.ylo = INFINITY;
            b.zhi = b.xhi = b.yhi = -INFINITY;
            b.behind = false;
        }
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
            BoxAcc c;
            c.zlo = __shfl_xor(b.zlo, o, kWave);
            c.zhi = __shfl_xor(b.zhi, o, kWave);
            c.xlo = __shfl_xor(b.xlo, o, kWave);
            c.xhi = __shfl_xor(b.xhi, o, kWave);
            c.ylo = __shfl_xor(b.ylo, o, kWave);
            c.yhi = __shfl_xor(b.yhi, o, kWave);
            c.behind = __shfl_xor((int)b.behind, o, kWave) != 0;
            box_merge(b, c);
        }
        RangeRect r;
        if (j < n && box_rect(g, b, r)) {
            int tx0, ty0, ntx, n_tiles;
            rect_tiles(r, tx0, ty0, ntx, n_tiles);
            for (int t = corner; t < n_tiles; t += 8) {
                const int tile = (ty0 + t / ntx) * a.rb.tw + tx0 + t % ntx;
                const int slot = atomicAdd(&a.rb.cnt[tile], 1);
                if (slot < a.rb.cap) a.rb.rect[(int64_t)tile * a.rb.cap + slot] = r;
            }
        }
    }
}

__device__ __forceinline__ int bytes_set(uint32_t x) { return (int)((x * 0x01010101u) >> 24); }


// Stage three of the allocation (the visible list) fused with the integration:
// workgroup b scans flag bytes [2048 b, 2048 b + 2048), clears them, compacts
// the set ones into an LDS list (wave prefix sums) -- also written out as
// segment b of the visible list -- and its 4 waves integrate those blocks.  The hash spreads blocks uniformly over the entries, so every
// workgroup gets about the same share (about 4 blocks at VGA).  The same pass
// clears the allocation's claim-set slots.
template <int FMT>
__global__ __launch_bounds__(kScanThreads) void k_integrate(IntegrateArgs a)
{
    __shared__ int32_t s_list[kScanEntries];
    __shared__ unsigned long long s_key[kScanEntries];   // block keys, for the range bins
    __shared__ int s_wave[kScanThreads / kWave];
    __shared__ int s_n;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int nwaves = kScanThreads / kWave;
    // scan and clear 8 flags per thread
    const int64_t w8 = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    uint2 f = make_uint2(0u, 0u);
    if (w8 < a.n_words8) f = a.vis8[w8];
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt->set_used[a.parity ^ 1] = 0;  // next frame's counter
    {
        const int su = a.cnt->set_used[a.parity];
        for (int i = blockIdx.x * kScanThreads + threadIdx.x; i < su; i += gridDim.x * kScanThreads)
            a.set[a.set_list[i]] = 0ull;
    }
    if (a.rb.cnt) {   // the next frame's bins
        for (int i = blockIdx.x * kScanThreads + threadIdx.x; i < a.n_clear; i += gridDim.x * kScanThreads)
            a.rb_clear[i] = 0;
    }
    const int c = bytes_set(f.x) + bytes_set(f.y);
    if (c) a.vis8[w8] = make_uint2(0u, 0u);
    int incl = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < nwaves; w++) {
            const int x = s_wave[w];
            s_wave[w] = t;
            t += x;
        }
        s_n = t;
        a.seg.cnt[blockIdx.x] = t;
        if (t) {
            const int sI = blockIdx.x % kStripes;
            atomicAdd(&a.cnt->vis[0][sI][0], (unsigned long long)t);
            atomicAdd(&a.cnt->vis[1][sI][0], (unsigned long long)t);
        }
    }
    __syncthreads();
    if (c) {
        int k = s_wave[wave] + incl - c;
        int32_t *seg = a.seg.list + (int64_t)blockIdx.x * kSegEntries;
        const uint32_t w2[2] = {f.x, f.y};
#pragma unroll
        for (int q = 0; q < 8; q++)
            if ((w2[q >> 2] >> (8 * (q & 3))) & 0xffu) {
                const int32_t e = (int32_t)(w8 * 8 + q);
                s_list[k] = e;
                seg[k] = e;
                k++;
            }
    }
    __syncthreads();
    const int n = s_n;
    uint32_t n_upd = 0;
    for (int j = wave; j < n; j += nwaves) {
        unsigned long long key;
        n_upd += integrate_block<FMT>(a, s_list[j], lane, key);
        if (a.rb.cnt && lane == 0) s_key[j] = key;
    }
    if (a.rb.cnt) {
        __syncthreads();
        bin_blocks(a, s_key, n);
    }
    // one counter update per workgroup, on one of kStripes separate lines
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) n_upd += __shfl_xor(n_upd, o, kWave);
    __syncthreads();
    if (lane == 0) s_wave[wave] = (int)n_upd;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < nwaves; w++) t += (unsigned)s_wave[w];
        if (t) {
            const int sI = blockIdx.x % kStripes;
            atomicAdd(&a.cnt->upd[0][sI][0], t);
            atomicAdd(&a.cnt->upd[1][sI][0], t);
        }
    }
}

hipError_t launch_integrate(int fmt, const IntegrateArgs &a, hipStream_t st)
{
    const int grid = (int)((a.n_words8 + kScanThreads - 1) / kScanThreads);
    switch (fmt) {
    case ITM_VOX_F32: k_integrate<ITM_VOX_F32><<<grid, 256, 0, st>>>(a); break;
    case ITM_VOX_F16: k_integrate<ITM_VOX_F16><<<grid, 256, 0, st>>>(a); break;
    default: k_integrate<ITM_VOX_S16U8><<<grid, 256, 0, st>>>(a); break;
    }
    return hipGetLastError();
}

}  // namespace itm
