// Raycast (section "Raycast"): one ray per pixel through the hashed volume.
//
// Ray set-up (origin, unit direction, search range) is binary64 and rounded once;
// the march is binary32 in voxel units, q(t) = o/s + t d/s with t in metres.
// The search range is [z_near, z_far] along the camera axis or, with expected
// depths on, that range narrowed to the pixel's expected range (section
// "Raycast": visible blocks projected into the image).
// Reads:
//   nearest  n(q) = floor(q + 1/2); found when the block of n is allocated;
//            F_n = F at n
//   F_t(q)   trilinear interpolation over the 8 lattice voxels around q, voxels of
//            unallocated blocks reading F = 1
// State machine (coarse block steps of 8 s with one step back on a hit, fine
// steps of mu, steps of max(F_n mu, s) in front of the surface, steps of
// max(|F_n| mu, s) when a block is entered from behind, and two refinement steps
// t += F_t mu once behind the surface); the normal is the normalised central
// difference of F_t at +-1 voxel along the world axes.
// A one-entry register cache of the last block looked up saves most hash probes:
// consecutive samples of a ray mostly fall in the same block, and a probe is one
// load of the bucket's two keys.  Coarse samples in space with no allocated block
// are skipped a macro cell (4^3 blocks) at a time through a hashed occupancy
// bitmap staged in LDS; the samples taken keep the 8 s spacing.
#include "itm_internal.hpp"

namespace itm {

enum { RC_COARSE = 0, RC_FINE, RC_SURFACE, RC_BEHIND, RC_WRONG_SIDE };

// Where the raycast reads F: the voxel block array, or, with REF, for blocks the
// learned refiner refined in the current frame (stamp == frame), its side buffer
template <int FMT, bool REF>
struct VoxSrc {
    const typename Vox<FMT>::S *sdf;
    const __half *ref;      // [capacity][512] refined F, REF only
    const int32_t *stamp;   // [capacity] frame of the last refinement, REF only
    int32_t frame;

    __device__ bool refined(int32_t ptr) const { return REF && ptr >= 0 && stamp[ptr] == frame; }
    __device__ float read(int32_t ptr, bool r, int32_t li) const
    {
        if (REF && r) return __half2float(ref[(int64_t)ptr * kBlockVox + li]);
        return Vox<FMT>::to_f(sdf[(int64_t)ptr * kBlockVox + li]);
    }
};

template <int FMT, bool REF>
struct BlockReader {
    const HashView &h;
    VoxSrc<FMT, REF> src;
    int cx, cy, cz;
    int32_t cptr;
    bool cref;              // the cached block reads its refined F

    __device__ BlockReader(const HashView &hv, const VoxSrc<FMT, REF> &s)
        : h(hv), src(s), cx(INT_MIN), cy(0), cz(0), cptr(-1), cref(false) {}

    __device__ int32_t block(int bx, int by, int bz)
    {
        if (bx != cx || by != cy || bz != cz) {
            cx = bx; cy = by; cz = bz;
            cptr = block_of(h, find_block_direct(h, bx, by, bz));
            if (REF) cref = src.refined(cptr);
        }
        return cptr;
    }
    // F at the nearest lattice voxel of q; false (F = 1) when its block is absent
    __device__ bool nearest(float qx, float qy, float qz, float &F)
    {
        const int vx = (int)floorf(qx + 0.5f), vy = (int)floorf(qy + 0.5f), vz = (int)floorf(qz + 0.5f);
        const int32_t p = block(vx >> 3, vy >> 3, vz >> 3);
        if (p < 0) { F = 1.0f; return false; }
        F = src.read(p, cref, (int32_t)((vx & 7) | (vy & 7) << 3 | (vz & 7) << 6));
        return true;
    }
};

// The blocks covering a lattice region of at most 9 voxels per axis (so at most
// 2 x 2 x 2 blocks), looked up together so that their hash probes overlap; then
// any voxel of the region is read with one gather.
template <int FMT>
struct Cube {
    int bx0, by0, bz0;   // first block per axis
    int bx1, by1, bz1;   // last block per axis (bx0 or bx0 + 1)
    int32_t p[8];   // block pointer of (dx, dy, dz) = (c & 1, c >> 1 & 1, c >> 2 & 1)
    uint32_t rmask; // bit c: block c reads its refined F

    // whether every voxel of the region [l, h] lies in the blocks fetched
    __device__ bool holds(int lx, int ly, int lz, int hx, int hy, int hz) const
    {
        return (lx >> 3) >= bx0 && (hx >> 3) <= bx1 && (ly >> 3) >= by0 && (hy >> 3) <= by1 &&
               (lz >> 3) >= bz0 && (hz >> 3) <= bz1;
    }

    // Every block is probed (the march's cached block is not reused: keeping it
    // live costs registers).  The 8 buckets are read together -- every block's
    // bucket is a valid address, and the records of blocks the region does not
    // reach are dropped -- then matched; a block whose bucket holds two other
    // keys walks the excess chain.  (Read under a branch each, the buckets were
    // waited for one at a time.)
    template <bool REF>
    __device__ void fetch(const HashView &h, const VoxSrc<FMT, REF> &src, int lx, int ly, int lz, int hx, int hy,
                          int hz)
    {
        bx0 = lx >> 3; by0 = ly >> 3; bz0 = lz >> 3;
        bx1 = hx >> 3; by1 = hy >> 3; bz1 = hz >> 3;
        const bool sx = bx1 != bx0, sy = by1 != by0, sz = bz1 != bz0;
        ulonglong2 k2[8];
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const int kx = (c & 1) ? bx1 : bx0, ky = (c & 2) ? by1 : by0, kz = (c & 4) ? bz1 : bz0;
            k2[c] = *reinterpret_cast<const ulonglong2 *>(h.buckets[hash_index(kx, ky, kz, h.mask)].key);
        }
        // (opaque from here: the compiler would otherwise move the first
        // block's read into the key-range test's branch and split it there)
#pragma unroll
        for (int c = 0; c < 8; c++) asm volatile("" : "+v"(k2[c].x), "+v"(k2[c].y));
        uint32_t slow = 0;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
            const bool need = (!dx || sx) && (!dy || sy) && (!dz || sz);
            const int kx = dx ? bx1 : bx0, ky = dy ? by1 : by0, kz = dz ? bz1 : bz0;
            const unsigned long long key = pack_key(kx, ky, kz);
            const int32_t bi = 2 * (int32_t)hash_index(kx, ky, kz, h.mask);
            int32_t e = -1;
            if (need && in_key_range(kx, ky, kz)) {
                if (k2[c].x == key) e = bi;
                else if (k2[c].y == key) e = bi + 1;
                else if (k2[c].y != 0ull) slow |= 1u << c;   // both slots taken: the chain
            }
            p[c] = e;
        }
        while (slow) {
            const int c = __builtin_ctz(slow);
            slow &= slow - 1;
            int kx = bx0, ky = by0, kz = bz0;
            if (c & 1) kx = bx1;
            if (c & 2) ky = by1;
            if (c & 4) kz = bz1;
            const unsigned long long key = pack_key(kx, ky, kz);
            int32_t e = -1;
            for (int32_t x = h.head[hash_index(kx, ky, kz, h.mask)]; x >= 0;) {
                const Excess E = h.excess[x];
                if (E.key == key) {
                    e = 2 * h.n_buckets + x;
                    break;
                }
                x = E.next;
            }
#pragma unroll
            for (int r = 0; r < 8; r++)   // register selects, no indexed array
                if (r == c) p[r] = e;
        }
        if (h.blk) {   // swapping: the entry's device voxel block, all 8 read together
            int32_t q[8];
#pragma unroll
            for (int c = 0; c < 8; c++) q[c] = h.blk[max(p[c], 0)];
#pragma unroll
            for (int c = 0; c < 8; c++) p[c] = p[c] >= 0 ? q[c] : -1;
        }
        rmask = 0u;
        if (REF) {
            int32_t st[8];
#pragma unroll
            for (int c = 0; c < 8; c++) st[c] = src.stamp[max(p[c], 0)];
#pragma unroll
            for (int c = 0; c < 8; c++) rmask |= (p[c] >= 0 && st[c] == src.frame) ? 1u << c : 0u;
        }
    }
};

// the block of voxel v among a Cube's (-1 when absent)
template <int FMT>
__device__ __forceinline__ int32_t cube_block(const Cube<FMT> &cb, int vx, int vy, int vz)
{
    const bool ex = (vx >> 3) != cb.bx0, ey = (vy >> 3) != cb.by0, ez = (vz >> 3) != cb.bz0;
    const int32_t a0 = ex ? cb.p[1] : cb.p[0], a1 = ex ? cb.p[3] : cb.p[2];
    const int32_t a2 = ex ? cb.p[5] : cb.p[4], a3 = ex ? cb.p[7] : cb.p[6];
    const int32_t b0 = ey ? a1 : a0, b1 = ey ? a3 : a2;
    return ez ? b1 : b0;
}

// Voxel reads of a Cube: a short select of the voxel's block, then one load (an
// absent block reads as F = 1)
template <int FMT, bool REF>
__device__ __forceinline__ float cube_F(const Cube<FMT> &cb, const VoxSrc<FMT, REF> &src, int vx, int vy, int vz)
{
    const int32_t ptr = cube_block(cb, vx, vy, vz);
    if (ptr < 0) return 1.0f;
    bool r = false;
    if (REF) {
        const int c = ((vx >> 3) != cb.bx0 ? 1 : 0) | ((vy >> 3) != cb.by0 ? 2 : 0) | ((vz >> 3) != cb.bz0 ? 4 : 0);
        r = (cb.rmask >> c) & 1u;
    }
    return src.read(ptr, r, (int32_t)((vx & 7) | (vy & 7) << 3 | (vz & 7) << 6));
}

// the 8 lattice voxels of the cell with corner i
template <int FMT, bool REF>
__device__ __forceinline__ void cube_cell(const Cube<FMT> &cb, const VoxSrc<FMT, REF> &sdf, int ix, int iy,
                                          int iz, float Fc[8])
{
#pragma unroll
    for (int c = 0; c < 8; c++) Fc[c] = cube_F(cb, sdf, ix + (c & 1), iy + ((c >> 1) & 1), iz + ((c >> 2) & 1));
}

__device__ __forceinline__ float trilinear8(const float Fc[8], float rx, float ry, float rz)
{
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; c++) {
        const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        const float w = (dx ? rx : 1.0f - rx) * (dy ? ry : 1.0f - ry) * (dz ? rz : 1.0f - rz);
        acc = fmaf(w, Fc[c], acc);
    }
    return acc;
}

// the cell with corner i and the outer layers of its 6 face neighbours: the
// 32 voxels of the central differences of F_t at +- one voxel (the cell's own 8
// already in Fc when have_cell)
template <int FMT, bool REF>
__device__ __forceinline__ void stencil(const Cube<FMT> &cb, const VoxSrc<FMT, REF> &sdf, int ix, int iy,
                                        int iz, bool have_cell, float Fc[8], float Ex[2][4], float Ey[2][4],
                                        float Ez[2][4])
{
    if (!have_cell) cube_cell(cb, sdf, ix, iy, iz, Fc);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int a0 = k & 1, a1 = k >> 1;
        Ex[0][k] = cube_F(cb, sdf, ix - 1, iy + a0, iz + a1);
        Ex[1][k] = cube_F(cb, sdf, ix + 2, iy + a0, iz + a1);
        Ey[0][k] = cube_F(cb, sdf, ix + a0, iy - 1, iz + a1);
        Ey[1][k] = cube_F(cb, sdf, ix + a0, iy + 2, iz + a1);
        Ez[0][k] = cube_F(cb, sdf, ix + a0, iy + a1, iz - 1);
        Ez[1][k] = cube_F(cb, sdf, ix + a0, iy + a1, iz + 2);
    }
}

// gradient of F_t at fractions r of the cell whose 8 voxels are Fc, by central
// differences at +- one voxel per axis (each side one trilinear interpolation,
// sharing Fc), accumulated into g
__device__ __forceinline__ void gradient(const float Fc[8], const float Ex[2][4], const float Ey[2][4],
                                         const float Ez[2][4], float rx, float ry, float rz, float &gx, float &gy,
                                         float &gz)
{
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int a0 = k & 1, a1 = k >> 1;
        // x pair: corners (y, z) = (a0, a1) of the cell; Fc index dx + 2 dy + 4 dz
        const float wyz = (a0 ? ry : 1.0f - ry) * (a1 ? rz : 1.0f - rz);
        const float xp = (1.0f - rx) * Fc[1 + 2 * a0 + 4 * a1] + rx * Ex[1][k];
        const float xm = (1.0f - rx) * Ex[0][k] + rx * Fc[0 + 2 * a0 + 4 * a1];
        gx = fmaf(wyz, xp - xm, gx);
        const float wxz = (a0 ? rx : 1.0f - rx) * (a1 ? rz : 1.0f - rz);
        const float yp = (1.0f - ry) * Fc[a0 + 2 + 4 * a1] + ry * Ey[1][k];
        const float ym = (1.0f - ry) * Ey[0][k] + ry * Fc[a0 + 0 + 4 * a1];
        gy = fmaf(wxz, yp - ym, gy);
        const float wxy = (a0 ? rx : 1.0f - rx) * (a1 ? ry : 1.0f - ry);
        const float zp = (1.0f - rz) * Fc[a0 + 2 * a1 + 4] + rz * Ez[1][k];
        const float zm = (1.0f - rz) * Ez[0][k] + rz * Fc[a0 + 2 * a1 + 0];
        gz = fmaf(wxy, zp - zm, gz);
    }
}

template <int FMT, bool CLR, bool REF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_raycast(RaycastArgs a)
{
    const FrameGeom &g = a.fg;
    int tx, ty;
    if (!xcd_tile((g.W + 15) / 16, (g.H + 15) / 16, tx, ty)) return;  // whole workgroup
    // the tile's expected-depth bin, loaded while the macro filter is staged
    TileBin bin;
    if (a.rb.cnt) bin = tile_bin(a.rb, tx, ty);
    // the macro-cell filter, staged in LDS: empty-space tests cost an LDS read
    __shared__ uint32_t s_filt[kMacroWords];
    {   // all of a thread's reads issued before its LDS writes: one round trip
        constexpr int kPer = kMacroWords / 4 / 256;
        static_assert(kPer * 4 * 256 == kMacroWords, "the filter fills whole 256-thread rounds");
        const uint4 *src = reinterpret_cast<const uint4 *>(a.h.macro);
        uint4 *dst = reinterpret_cast<uint4 *>(s_filt);
        uint4 w[kPer];
#pragma unroll
        for (int k = 0; k < kPer; k++) w[k] = src[threadIdx.x + 256 * k];
#pragma unroll
        for (int k = 0; k < kPer; k++) dst[threadIdx.x + 256 * k] = w[k];
    }
    __syncthreads();
    const uint32_t *s_macro = s_filt;
    // a workgroup covers 16 x 16 pixels, each wave an 8 x 8 quadrant of it
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int u = tx * 16 + (wave & 1) * 8 + (lane & 7);
    const int v = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
    // expected depth range of the pixel (whole workgroup)
    float zlo = 0.0f, zhi = 0.0f;
    if (a.rb.cnt) {
        __shared__ RangeLds s_range;
        tile_range(g, a.list, a.rb, tx, ty, bin, u, v, s_range, zlo, zhi);
    }
    if (u >= g.W || v >= g.H) return;
    const int64_t pix = (int64_t)v * g.W + u;

    // binary64 ray set-up, rounded once (the camera centre in voxel units comes
    // from the host)
    const double cdx = ((double)u - g.cxd) * g.inv_fx, cdy = ((double)v - g.cyd) * g.inv_fy;
    const double len = sqrt(cdx * cdx + cdy * cdy + 1.0);
    const double w = g.inv_s / len;   // unit direction, in voxels per metre of t
    const float ox = g.o_vox[0], oy = g.o_vox[1], oz = g.o_vox[2];
    const float dx = (float)((g.Rwc[0] * cdx + g.Rwc[1] * cdy + g.Rwc[2]) * w);
    const float dy = (float)((g.Rwc[3] * cdx + g.Rwc[4] * cdy + g.Rwc[5]) * w);
    const float dz = (float)((g.Rwc[6] * cdx + g.Rwc[7] * cdy + g.Rwc[8]) * w);
    // search range: [z_near, z_far], narrowed to the expected range when there is one
    double t0 = (double)g.z_near * len, t1 = (double)g.z_far * len;
    if (a.rb.cnt) {
        if (zlo <= zhi) {
            t0 = fmax(t0, (double)zlo * len);
            t1 = fmin(t1, (double)zhi * len);
        } else {
            t1 = t0;   // no visible block projects here: nothing to search
        }
    }
    const float t_near = (float)t0, t_far = (float)t1;
    const float s = g.s_f, mu = g.mu_f, bs = 8.0f * g.s_f;
    const int fine_budget = (int)ceilf(bs / mu) + 1;
    const int cap = (int)((t_far - t_near) / s) * 4 + 1000;
    // Macro-cell exit, per axis: the exit plane's offset from the cell's low
    // corner (the cell shrunk by 1e-3 voxel against rounding) and the reciprocal
    // direction; an axis the ray does not move along never exits.
    const float e_mc = 1e-3f;
    const float ex = dx > 0.0f ? 32.0f - e_mc : e_mc, ey = dy > 0.0f ? 32.0f - e_mc : e_mc;
    const float ez = dz > 0.0f ? 32.0f - e_mc : e_mc;
    const float idx = dx != 0.0f ? 1.0f / dx : 0.0f, idy = dy != 0.0f ? 1.0f / dy : 0.0f;
    const float idz = dz != 0.0f ? 1.0f / dz : 0.0f;
    const float inv_bs = 1.0f / bs;

    VoxSrc<FMT, REF> src;
    src.sdf = (const typename Vox<FMT>::S *)a.sdf;
    src.ref = a.refined;
    src.stamp = a.rstamp;
    src.frame = a.rframe;
    BlockReader<FMT, REF> rd(a.h, src);
    float t = t_near;
    int state = RC_COARSE, fine_miss = 0;
    for (int it = 0; it < cap && t < t_far; it++) {
        const float qx = fmaf(t, dx, ox), qy = fmaf(t, dy, oy), qz = fmaf(t, dz, oz);
        if (state == RC_COARSE) {
            const int vx = (int)floorf(qx + 0.5f), vy = (int)floorf(qy + 0.5f), vz = (int)floorf(qz + 0.5f);
            const int bx = vx >> 3, by = vy >> 3, bz = vz >> 3;
            const uint32_t mi = macro_index(bx, by, bz);
            if (!((s_macro[mi >> 5] >> (mi & 31)) & 1u)) {
                // Every sample whose nearest voxel lies in this empty macro cell is a
                // miss: jump over them, keeping the sample spacing of 8 s.  The cell
                // in sample space is [32 m - 1/2, 32 (m + 1) - 1/2) per axis, shrunk
                // by 1e-3 voxel against rounding.
                const float lx = (float)((bx >> kMacroShift) * 32) - 0.5f;
                const float ly = (float)((by >> kMacroShift) * 32) - 0.5f;
                const float lz = (float)((bz >> kMacroShift) * 32) - 0.5f;
                const float tx = dx != 0.0f ? (lx + ex - ox) * idx : INFINITY;
                const float ty = dy != 0.0f ? (ly + ey - oy) * idy : INFINITY;
                const float tz = dz != 0.0f ? (lz + ez - oz) * idz : INFINITY;
                const float t_exit = fminf(tx, fminf(ty, tz));
                // samples to skip, rounded down by a relative 2^-20 so that the
                // product's rounding never skips past the exit (one sample too
                // few only costs another skip)
                const float m = fmaxf(ceilf((t_exit - t) * inv_bs * (1.0f - 0x1p-20f)), 1.0f);
                t = fmaf(m, bs, t);
                continue;
            }
        }
        // one sample site for every state, so that a wave whose lanes are in
        // different states runs the hash probe once
        float F;
        const bool found = rd.nearest(qx, qy, qz, F);
        if (state == RC_COARSE) {
            if (!found) t += bs;
            else { t = fmaxf(t - bs, t_near); state = RC_FINE; fine_miss = 0; }
        } else if (state == RC_FINE) {
            if (!found) {
                t += mu;
                if (++fine_miss > fine_budget) state = RC_COARSE;
            } else state = F < 0.0f ? RC_WRONG_SIDE : RC_SURFACE;
        } else if (state == RC_SURFACE) {
            if (!found) state = RC_COARSE;
            else if (F < 0.0f) { state = RC_BEHIND; break; }
            else t += fmaxf(F * mu, s);
        } else {  // RC_WRONG_SIDE
            if (!found) state = RC_COARSE;
            else if (F > 0.0f) state = RC_SURFACE;
            else t += fmaxf(-F * mu, s);
        }
    }
    float4 P = make_float4(0.f, 0.f, 0.f, 0.f), N = make_float4(0.f, 0.f, 0.f, 0.f);
    uchar4 C = make_uchar4(0, 0, 0, 0);
    if (state == RC_BEHIND) {
        const VoxSrc<FMT, REF> &sdf = src;
        // One block neighbourhood for the whole final phase: the blocks of voxels
        // [i - 3, i + 4] per axis around the first refinement cell i (at most
        // 2 x 2 x 2 blocks, probed together) hold both refinement cells and the
        // normal's stencil unless the second step moves more than 2 voxels.
        float qx = fmaf(t, dx, ox), qy = fmaf(t, dy, oy), qz = fmaf(t, dz, oz);
        float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
        int ix = (int)fx, iy = (int)fy, iz = (int)fz;
        Cube<FMT> cb;
        cb.fetch(a.h, src, ix - 3, iy - 3, iz - 3, ix + 4, iy + 4, iz + 4);
        float Fc[8];
        cube_cell(cb, sdf, ix, iy, iz, Fc);
        t = fmaf(trilinear8(Fc, qx - fx, qy - fy, qz - fz), mu, t);
        // Second refinement in the cell j of the new point.  The neighbourhood is
        // first widened to voxels [j - 2, j + 3], which holds the normal's stencil
        // of j and of its 26 neighbours; the final point nearly always lies in one
        // of those cells.
        // A lane whose point stays in its cell keeps the cell's voxels (fewer
        // gathers for the wave's memory pipeline, which bounds this kernel).
        qx = fmaf(t, dx, ox); qy = fmaf(t, dy, oy); qz = fmaf(t, dz, oz);
        fx = floorf(qx); fy = floorf(qy); fz = floorf(qz);
        int jx = (int)fx, jy = (int)fy, jz = (int)fz;
        if (!cb.holds(jx - 2, jy - 2, jz - 2, jx + 3, jy + 3, jz + 3))
            cb.fetch(a.h, src, jx - 2, jy - 2, jz - 2, jx + 3, jy + 3, jz + 3);
        if (jx != ix || jy != iy || jz != iz) cube_cell(cb, sdf, jx, jy, jz, Fc);
        t = fmaf(trilinear8(Fc, qx - fx, qy - fy, qz - fz), mu, t);
        // The normal: central differences of F_t over the stencil of the final
        // point's cell (blocks fetched again only if that point moved farther)
        qx = fmaf(t, dx, ox); qy = fmaf(t, dy, oy); qz = fmaf(t, dz, oz);
        fx = floorf(qx); fy = floorf(qy); fz = floorf(qz);
        ix = (int)fx; iy = (int)fy; iz = (int)fz;
        if (!cb.holds(ix - 1, iy - 1, iz - 1, ix + 2, iy + 2, iz + 2))
            cb.fetch(a.h, src, ix - 1, iy - 1, iz - 1, ix + 2, iy + 2, iz + 2);
        float Ex[2][4], Ey[2][4], Ez[2][4];   // [minus/plus][(a, b) of the other two axes]
        stencil(cb, sdf, ix, iy, iz, ix == jx && iy == jy && iz == jz, Fc, Ex, Ey, Ez);
        float gx = 0.0f, gy = 0.0f, gz = 0.0f;
        gradient(Fc, Ex, Ey, Ez, qx - fx, qy - fy, qz - fz, gx, gy, gz);
        if (CLR) {   // colour of the final point's nearest voxel (held by the Cube)
            const int nx = (int)floorf(qx + 0.5f), ny = (int)floorf(qy + 0.5f), nz = (int)floorf(qz + 0.5f);
            const int32_t p = cube_block(cb, nx, ny, nz);
            if (p >= 0) {
                const uchar4 c = a.clr[(int64_t)p * kBlockVox + ((nx & 7) | (ny & 7) << 3 | (nz & 7) << 6)];
                C = make_uchar4(c.x, c.y, c.z, 255);
            }
        }
        // the hit in metres, (o + t d) s in binary64 from the march's binary32 terms
        P = make_float4((float)(g.s * ((double)ox + (double)t * (double)dx)),
                        (float)(g.s * ((double)oy + (double)t * (double)dy)),
                        (float)(g.s * ((double)oz + (double)t * (double)dz)), 1.0f);
        const float n2 = gx * gx + gy * gy + gz * gz;
        if (n2 > 0.0f) {
            const float r = 1.0f / sqrtf(n2);
            N = make_float4(gx * r, gy * r, gz * r, 1.0f);
        }
    }
    a.pts[pix] = P;
    a.nrm[pix] = N;
    if (CLR) a.rgb_out[pix] = C;
}

template <int FMT>
void launch_fmt(const RaycastArgs &a, bool clr, bool ref, int grid, hipStream_t st)
{
    if (ref) {
        if (clr) launch_k(k_raycast<FMT, true, true>, grid, 256, st, a);
        else launch_k(k_raycast<FMT, false, true>, grid, 256, st, a);
    } else {
        if (clr) launch_k(k_raycast<FMT, true, false>, grid, 256, st, a);
        else launch_k(k_raycast<FMT, false, false>, grid, 256, st, a);
    }
}

hipError_t launch_raycast(int fmt, const RaycastArgs &a, hipStream_t st)
{
    const int grid = xcd_grid(((a.fg.W + 15) / 16) * ((a.fg.H + 15) / 16));
    // the colour variant and the one that reads refined blocks are kernels of
    // their own: the plain depth raycast carries neither
    const bool clr = a.clr && a.rgb_out;
    const bool ref = a.refined != nullptr;
    switch (fmt) {
    case ITM_VOX_F32: launch_fmt<ITM_VOX_F32>(a, clr, ref, grid, st); break;
    case ITM_VOX_F16: launch_fmt<ITM_VOX_F16>(a, clr, ref, grid, st); break;
    default: launch_fmt<ITM_VOX_S16U8>(a, clr, ref, grid, st); break;
    }
    return hipGetLastError();
}

}  // namespace itm
