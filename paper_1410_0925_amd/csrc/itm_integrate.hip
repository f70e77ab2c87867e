// Integration (section "Integration", computeUpdatedVoxelDepthInfo) over the
// voxels of the frame's visible blocks.
//
// One wave per visible block, taken from the visible list the allocation built
// (its counters are read on the device: no count goes to the host).  Lane l
// owns voxels 4l..4l+3 and 256+4l..256+4l+3 of the block, so every voxel load
// or store instruction of a wave covers one contiguous range
// (16 B per lane in the float form).  A lane reads its 8 voxels, decides for
// each whether it is updated -- that needs only the voxel's position and the
// depth image -- and writes back a group of 4 voxels only when one of them is.
//
// Decisions follow a fixed binary32 evaluation order (so that they can be
// reproduced exactly): the block origin's camera coordinates are formed in binary64
// once per block and split into a binary32 pair hi + lo; the in-block offset
// (lx g_x + ly g_y) + lz g_z is added to lo first.  The value eta = d - p_z is
// formed as (d - hi_z) - (lo_z + offset_z), accurate to ~1e-8 m at room scale.
#include <algorithm>

#include "itm_alloc.hpp"

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
// Colour sample of a voxel (section "Framework Flexibility" gives the voxel's
// RGB and colour weight; the update is the library's reading): each channel keeps
// the running average of its samples rounded to the nearest integer, ties to
// even, in exact integer arithmetic; the weight counts samples up to cap.
__device__ __forceinline__ uchar4 colour_step(uchar4 c, uchar4 s, int cap)
{
    const int w = c.w, den = w + 1;
    int ch[3] = {c.x, c.y, c.z};
    const int smp[3] = {s.x, s.y, s.z};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int num = w * ch[k] + smp[k];
        int q = num / den;
        const int r2 = 2 * (num - q * den);
        if (r2 > den || (r2 == den && (q & 1))) q++;
        ch[k] = q;
    }
    return make_uchar4((unsigned char)ch[0], (unsigned char)ch[1], (unsigned char)ch[2],
                       (unsigned char)min(w + 1, cap));
}

template <int FMT, bool CLR>
__device__ uint32_t integrate_block(const FuseArgs &a, unsigned long long key, int32_t e, int lane)
{
    const FrameGeom &g = a.fg;
    const int32_t ptr = block_of(a.h, e);   // the entry's voxel block
    if (ptr < 0) return 0;                  // swapping: no device block this frame
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
    const int ccap = min((int)g.max_w_f, 255);
    uint32_t n_upd = 0;
    // depth-only form: both groups' voxels projected first and their 8 depth
    // reads issued together (one memory round; a read whose value decides a
    // branch is waited for before the next one is issued)
    float dep[2][4];
    uint32_t seen[2] = {0u, 0u};
    if constexpr (!CLR) {
#pragma unroll
        for (int grp = 0; grp < 2; grp++) {
            const int li0 = 4 * lane + 256 * grp;
            const float fy_ = (float)((li0 >> 3) & 7), fz_ = (float)(li0 >> 6);
            // the group's y and z steps, shared by its 4 voxels
            float yz[3];
#pragma unroll
            for (int c = 0; c < 3; c++) yz[c] = fy_ * g.g[1][c] + fz_ * g.g[2][c];
            int pix[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float fx_ = (float)((li0 & 7) + j);
                float p[3];
#pragma unroll
                for (int c = 0; c < 3; c++) p[c] = hi[c] + (lo[c] + (fx_ * g.g[0][c] + yz[c]));
                pix[j] = 0;
                if (p[2] <= 0.0f) continue;
                const float rz = __builtin_amdgcn_rcpf(p[2]);   // 1 ulp; one reciprocal for x and y
                const float x = g.fx * p[0] * rz + g.cx;
                const float y = g.fy * p[1] * rz + g.cy;
                if (x < 1.0f || x > (float)(g.W - 2) || y < 1.0f || y > (float)(g.H - 2)) continue;
                pix[j] = (int)(x + 0.5f) + (int)(y + 0.5f) * g.W;
                seen[grp] |= 1u << j;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) dep[grp][j] = a.depth[pix[j]];   // pixel 0 when unseen: not used
        }
    }
#pragma unroll
    for (int grp = 0; grp < 2; grp++) {
        const int li0 = 4 * lane + 256 * grp;
        // the group's 4 colour voxels (16 bytes), loaded here rather than with the
        // depth voxels: fewer live registers keep 5 waves per SIMD
        uint4 cgg;
        if (CLR) cgg = *reinterpret_cast<const uint4 *>(a.clr + vbase + li0);
        const float fy_ = (float)((li0 >> 3) & 7), fz_ = (float)(li0 >> 6);
        float eta[4];
        int pix[4];
        uchar4 smp[4];
        uint32_t upd = 0, cupd = 0;
        if constexpr (!CLR) {
            const float yz2 = fy_ * g.g[1][2] + fz_ * g.g[2][2];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                eta[j] = 0.0f;
                if (!(seen[grp] & (1u << j))) continue;
                const float d = dep[grp][j];
                if (!(d > 0.0f) || isinf(d)) continue;
                // the voxel's camera-z step, as in its projection (same operations)
                const float dl2 = (float)((li0 & 7) + j) * g.g[0][2] + yz2;
                const float e32 = (d - hi[2]) - (lo[2] + dl2);
                if (e32 < -mu) continue;
                eta[j] = e32;
                upd |= 1u << j;
            }
        } else {
            // the colour form keeps one voxel at a time (its registers are full)
            float yz[3];
#pragma unroll
            for (int c = 0; c < 3; c++) yz[c] = fy_ * g.g[1][c] + fz_ * g.g[2][c];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float fx_ = (float)((li0 & 7) + j);
                float p[3], dl2 = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const float t = fx_ * g.g[0][c] + yz[c];
                    p[c] = hi[c] + (lo[c] + t);
                    if (c == 2) dl2 = t;
                }
                eta[j] = 0.0f;
                if (p[2] <= 0.0f) continue;
                const float rz = __builtin_amdgcn_rcpf(p[2]);
                const float x = g.fx * p[0] * rz + g.cx;
                const float y = g.fy * p[1] * rz + g.cy;
                if (x < 1.0f || x > (float)(g.W - 2) || y < 1.0f || y > (float)(g.H - 2)) continue;
                pix[j] = (int)(x + 0.5f) + (int)(y + 0.5f) * g.W;
                smp[j] = a.rgbx[pix[j]];   // with the depth: no dependent read later
                const float d = a.depth[pix[j]];
                if (!(d > 0.0f) || isinf(d)) continue;
                const float e32 = (d - hi[2]) - (lo[2] + dl2);
                if (e32 < -mu) continue;
                eta[j] = e32;
                upd |= 1u << j;
                if (e32 <= mu) cupd |= 1u << j;   // inside the band: a colour sample
            }
        }
        if (upd) {
            Group4<FMT> &v = vg[grp];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (!(upd & (1u << j))) continue;
                const float f = fminf(1.0f, eta[j] * inv_mu);
                const float F = v.F(j), W = v.Wv(j);
                const float Wn = W + 1.0f;
                // running average F <- (W F + f) / (W + 1), in incremental form (the
                // reciprocal of the integer W + 1 to 1 ulp)
                const float Fn = F + (f - F) * __builtin_amdgcn_rcpf(Wn);
                v.set(j, Fn, fminf(Wn, g.max_w_f));
            }
            v.store(a.sdf, a.w, vbase + li0);
            n_upd += __builtin_popcount(upd);
            if (CLR && cupd) {
                uint32_t c4[4] = {cgg.x, cgg.y, cgg.z, cgg.w};
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if (!(cupd & (1u << j))) continue;
                    const uchar4 c = colour_step(__builtin_bit_cast(uchar4, c4[j]), smp[j], ccap);
                    c4[j] = __builtin_bit_cast(uint32_t, c);
                }
                *reinterpret_cast<uint4 *>(a.clr + vbase + li0) = make_uint4(c4[0], c4[1], c4[2], c4[3]);
            }
        }
    }
    return n_upd;
}

// Allocation and visible list (itm_alloc.hpp), one thread per pixel:
//   1. housekeeping, every workgroup its share: the previous frame's claim slots
//      and, with the search range on, the next frame's bin counts are cleared
//      (the stores go out after step 2, the one count they need is loaded with
//      the depth);
//   2. each thread walks its pixel's band segment and claims the blocks' keys in
//      the workgroup's LDS set; the lane that claims a key first finds or inserts
//      the block and records its entry there;
//   3. every block of the set is stamped with the frame number (by the lane that
//      found it, as soon as it has the entry); the workgroup that stamps a block
//      first lists it (one atomic per workgroup on one of 32 list stripes), so
//      each visible block is listed exactly once;
//   4. with the search range on, the listed blocks' expected-depth rectangles
//      are binned by image tile.
__global__ __launch_bounds__(256) void k_alloc(FuseArgs a)
{
    const FrameGeom &g = a.fg;
    __shared__ int32_t s_e[kSet];
    __shared__ unsigned long long s_k[kSet];
    __shared__ int s_wave[4], s_n, s_base, s_ovf;
    // the previous frame's claim count (for the housekeeping) and the pixel's
    // depth are loaded first, together: one memory round before the allocation
    const int su = *a.set_used_prev;
    int tx, ty;
    if (!xcd_tile((g.W + 15) / 16, (g.H + 15) / 16, tx, ty)) {   // whole workgroup
        frame_housekeeping(a, su);
        return;
    }
    const int u = tx * 16 + (threadIdx.x & 15);
    const int v = ty * 16 + (threadIdx.x >> 4);
    const bool in_image = u < g.W && v < g.H;
    float depth = 0.0f;
    if (in_image) depth = a.depth[(int64_t)v * g.W + u];
#pragma unroll
    for (int j = 0; j < kSet / 256; j++) {
        s_e[threadIdx.x + 256 * j] = -1;
        s_k[threadIdx.x + 256 * j] = 0ull;
    }
    __syncthreads();
    // 2. allocation
    if (in_image && depth > 0.0f && !isinf(depth)) alloc_pixel(a, u, v, depth, s_e, s_k);
    __syncthreads();
    // 1. housekeeping, its stores off the allocation's path
    frame_housekeeping(a, su);
    // 3. the visible list: thread t takes set slots 8t..8t+7 (those its workgroup
    //    stamped first hold their entry)
    uint32_t win = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int32_t e = s_e[8 * threadIdx.x + j];
        if (e >= 0) win |= 1u << j;   // stamped and won in step 2
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int c = __builtin_popcount(win);
    int incl = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    unsigned long long wkey[8];
    int32_t went[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
        wkey[j] = s_k[8 * threadIdx.x + j];
        went[j] = s_e[8 * threadIdx.x + j];
    }
    __syncthreads();
    // thread 0 reserves the workgroup's list records; the reservation is consumed
    // only after the binning's projections, which hide its round trip (barriers
    // wait for LDS traffic, not for this atomic)
    const int stripe = blockIdx.x % 32;
    int base = 0;
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < 4; w++) {
            const int x = s_wave[w];
            s_wave[w] = t;
            t += x;
        }
        s_n = t;
        // mbcnt of an empty mask is 0 on every lane, but not uniform to the
        // compiler: the atomic stays a plain returning one, waited for where
        // base is used, instead of a wave-aggregated one broadcast at once
        if (t) base = atomicAdd(&a.list.cnt[32 * stripe + (int)__builtin_amdgcn_mbcnt_lo(0u, 0u)], t);
    }
    __syncthreads();
    const int n_won = s_n;
    const int k0 = s_wave[wave] + incl - c;   // workgroup index of this thread's first record
    {
        int k = k0;
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (win & (1u << j)) s_k[k++] = wkey[j];   // the won keys, in list order, for the binning
    }
    auto publish = [&]() {
        if (threadIdx.x != 0) return;
        // records past the stripe's capacity go to the overflow segment
        const int spill = min(n_won, max(0, base + n_won - a.list.cap));
        s_ovf = spill ? atomicAdd(&a.list.cnt[32 * 32], spill) : 0;
        s_base = base;
    };
    // 4. expected-depth rectangles
    if (a.rb.cnt && n_won > 0) {   // uniform
        __syncthreads();
        bin_blocks(g, a.rb, s_k, n_won, s_e, publish);   // s_e is free again: its entries are in registers
    } else {
        publish();
    }
    __syncthreads();
    const int lbase = s_base, ovf = s_ovf;
    int k = k0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        if (!(win & (1u << j))) continue;
        VisRec r;
        r.key = s_k[k];   // the binning only read the keys
        r.e = went[j];
        r.pad = 0;
        const int pos = lbase + k;   // stripe position
        const int64_t slot = pos < a.list.cap ? (int64_t)stripe * a.list.cap + pos
                                              : (int64_t)32 * a.list.cap + ovf + (pos - max(lbase, a.list.cap));
        a.list.rec[slot] = r;
        k++;
    }
}

// Integration: one wave per visible block.  Wave gw serves list stripe
// gw % 32, items gw / 32, gw / 32 + nw / 32, ... (the grid is a multiple of 8
// workgroups), then the overflow segment.  The record is loaded together with
// the stripe's counter -- it lies inside the stripe's storage whatever the
// count -- so the two take one memory round instead of two.
// (5 waves per SIMD: the grid's 5 workgroups per CU then run in one round; the
// colour variant is held to 96 registers for it)
template <int FMT, bool CLR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_integrate(FuseArgs a)
{
    __shared__ unsigned long long s_red[2][4];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int gw = blockIdx.x * 4 + wave, nw = gridDim.x * 4;
    const int stripe = gw & 31, step = nw >> 5;
    uint32_t n_upd = 0, n_blk = 0;
    {
        const int n = a.list.cnt[32 * stripe];
        for (int i = gw >> 5; i < a.list.cap; i += step) {   // uniform over the wave
            const VisRec r = a.list.rec[(int64_t)stripe * a.list.cap + i];
            if (i >= n) break;
            n_upd += integrate_block<FMT, CLR>(a, r.key, r.e, lane);
            n_blk++;
        }
    }
    {   // the overflow segment (records of full stripes)
        const int n = a.list.cnt[32 * 32];
        for (int i = gw; i < n; i += nw) {
            const VisRec r = a.list.rec[(int64_t)32 * a.list.cap + i];
            n_upd += integrate_block<FMT, CLR>(a, r.key, r.e, lane);
            n_blk++;
        }
    }
    // one counter update per workgroup, on one of kStripes separate lines
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) n_upd += __shfl_xor(n_upd, o, kWave);
    if (lane == 0) {
        s_red[0][wave] = n_upd;
        s_red[1][wave] = n_blk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long u = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
        const unsigned long long v = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
        const int sI = blockIdx.x % kStripes;
        if (u) {
            atomicAdd(&a.cnt->upd[a.parity][sI][0], u);
            atomicAdd(&a.cnt->upd[2][sI][0], u);
        }
        if (v) {
            atomicAdd(&a.cnt->vis[a.parity][sI][0], v);
            atomicAdd(&a.cnt->vis[2][sI][0], v);
        }
    }
}

// Loading a volume (itm_import_blocks): a frame of its own whose visited blocks
// are the n given keys.  One thread per key: housekeeping as in k_alloc, then
// find or insert the block, stamp it, and list it when this thread stamped it
// first (the key list has no repeats, so that is every key that found an
// entry); entry[i] = the block's entry (= its voxel block), -1 when dropped.
__global__ __launch_bounds__(256) void k_import_keys(FuseArgs a, const int32_t *coords, int32_t n, int32_t *entry)
{
    frame_housekeeping(a, *a.set_used_prev);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int bx = coords[3 * i], by = coords[3 * i + 1], bz = coords[3 * i + 2];
    const int32_t e = find_or_insert(a, bx, by, bz);
    entry[i] = e;
    if (e < 0) return;
    if (atomicExch(&a.stamp[e], a.stamp_now) == a.stamp_now) return;
    const int stripe = i % 32, sI = i % kStripes;
    const int pos = atomicAdd(&a.list.cnt[32 * stripe], 1);
    VisRec r;
    r.key = pack_key(bx, by, bz);
    r.e = e;
    r.pad = 0;
    if (pos < a.list.cap) a.list.rec[(int64_t)stripe * a.list.cap + pos] = r;
    else a.list.rec[(int64_t)32 * a.list.cap + atomicAdd(&a.list.cnt[32 * 32], 1)] = r;
    atomicAdd(&a.cnt->vis[a.parity][sI][0], 1ull);
    atomicAdd(&a.cnt->vis[2][sI][0], 1ull);
}

hipError_t launch_import_keys(const FuseArgs &a, const int32_t *coords, int32_t n, int32_t *entry, hipStream_t st)
{
    k_import_keys<<<std::max(1, (n + 255) / 256), 256, 0, st>>>(a, coords, n, entry);
    return hipGetLastError();
}

hipError_t launch_alloc(const FuseArgs &a, hipStream_t st)
{
    launch_k(k_alloc, xcd_grid(((a.fg.W + 15) / 16) * ((a.fg.H + 15) / 16)), 256, st, a);
    return hipGetLastError();
}

hipError_t launch_integrate(int fmt, const FuseArgs &a, int grid, hipStream_t st)
{
    const bool clr = a.clr && a.rgbx;
    switch (fmt * 2 + (clr ? 1 : 0)) {
    case 2 * ITM_VOX_F32: launch_k(k_integrate<ITM_VOX_F32, false>, grid, 256, st, a); break;
    case 2 * ITM_VOX_F32 + 1: launch_k(k_integrate<ITM_VOX_F32, true>, grid, 256, st, a); break;
    case 2 * ITM_VOX_F16: launch_k(k_integrate<ITM_VOX_F16, false>, grid, 256, st, a); break;
    case 2 * ITM_VOX_F16 + 1: launch_k(k_integrate<ITM_VOX_F16, true>, grid, 256, st, a); break;
    case 2 * ITM_VOX_S16U8 + 1: launch_k(k_integrate<ITM_VOX_S16U8, true>, grid, 256, st, a); break;
    default: launch_k(k_integrate<ITM_VOX_S16U8, false>, grid, 256, st, a); break;
    }
    return hipGetLastError();
}

}  // namespace itm
