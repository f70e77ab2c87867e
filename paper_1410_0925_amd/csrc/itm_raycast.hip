// Raycast (section "Raycast"): one ray per pixel through the hashed volume.
//
// Ray set-up (origin, unit direction, search range) is binary64 and rounded once;
// the march is binary32 in voxel units, q(t) = o/s + t d/s with t in metres.
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
// consecutive samples of a ray mostly fall in the same block.  Coarse samples in
// space with no allocated block are skipped a macro cell (4^3 blocks) at a time
// through a hashed occupancy bitmap; the samples taken keep the 8 s spacing.
#include "itm_internal.hpp"

namespace itm {

enum { RC_COARSE = 0, RC_FINE, RC_SURFACE, RC_BEHIND, RC_WRONG_SIDE };

template <int FMT>
struct BlockReader {
    const HashView &h;
    const typename Vox<FMT>::S *sdf;
    int cx, cy, cz;
    int32_t cptr;

    __device__ BlockReader(const HashView &hv, const void *s)
        : h(hv), sdf((const typename Vox<FMT>::S *)s), cx(INT_MIN), cy(0), cz(0), cptr(-1) {}

    __device__ int32_t block(int bx, int by, int bz)
    {
        if (bx != cx || by != cy || bz != cz) {
            cx = bx; cy = by; cz = bz;
            cptr = find_block(h, bx, by, bz);
        }
        return cptr;
    }
    // F at the nearest lattice voxel of q; false (F = 1) when its block is absent
    __device__ bool nearest(float qx, float qy, float qz, float &F)
    {
        const int vx = (int)floorf(qx + 0.5f), vy = (int)floorf(qy + 0.5f), vz = (int)floorf(qz + 0.5f);
        const int32_t p = block(vx >> 3, vy >> 3, vz >> 3);
        if (p < 0) { F = 1.0f; return false; }
        F = Vox<FMT>::to_f(sdf[(int64_t)p * kBlockVox + (vx & 7) + 8 * (vy & 7) + 64 * (vz & 7)]);
        return true;
    }
};

// The blocks covering a lattice region of at most 9 voxels per axis (so at most
// 2 x 2 x 2 blocks), looked up together so that their hash probes overlap; then
// any voxel of the region is read with one gather.
template <int FMT>
struct Cube {
    int bx0, by0, bz0;
    int32_t p[8];   // block pointer of (dx, dy, dz) = (c & 1, c >> 1 & 1, c >> 2 & 1)

    // blocks near a surface are almost always allocated, so they are probed
    // directly; the march's cached block is reused without a probe
    __device__ void fetch(const HashView &h, const BlockReader<FMT> &rd, int lx, int ly, int lz, int hx,
                          int hy, int hz)
    {
        bx0 = lx >> 3; by0 = ly >> 3; bz0 = lz >> 3;
        const int bx1 = hx >> 3, by1 = hy >> 3, bz1 = hz >> 3;
        const bool sx = bx1 != bx0, sy = by1 != by0, sz = bz1 != bz0;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
            const bool need = (!dx || sx) && (!dy || sy) && (!dz || sz);
            const int kx = dx ? bx1 : bx0, ky = dy ? by1 : by0, kz = dz ? bz1 : bz0;
            const bool cached = kx == rd.cx && ky == rd.cy && kz == rd.cz;
            p[c] = !need ? -1 : cached ? rd.cptr : find_block_direct(h, kx, ky, kz);
        }
    }
    __device__ float F(const typename Vox<FMT>::S *sdf, int vx, int vy, int vz) const
    {
        const bool ex = (vx >> 3) != bx0, ey = (vy >> 3) != by0, ez = (vz >> 3) != bz0;
        const int32_t a0 = ex ? p[1] : p[0], a1 = ex ? p[3] : p[2];
        const int32_t a2 = ex ? p[5] : p[4], a3 = ex ? p[7] : p[6];
        const int32_t b0 = ey ? a1 : a0, b1 = ey ? a3 : a2;
        const int32_t ptr = ez ? b1 : b0;
        if (ptr < 0) return 1.0f;
        return Vox<FMT>::to_f(sdf[(int64_t)ptr * kBlockVox + (vx & 7) + 8 * (vy & 7) + 64 * (vz & 7)]);
    }
    // trilinear interpolation at q with i = floor(q) inside the region
    __device__ float trilinear(const typename Vox<FMT>::S *sdf, int ix, int iy, int iz, float rx,
                               float ry, float rz) const
    {
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
            const float w = (dx ? rx : 1.0f - rx) * (dy ? ry : 1.0f - ry) * (dz ? rz : 1.0f - rz);
            acc = fmaf(w, F(sdf, ix + dx, iy + dy, iz + dz), acc);
        }
        return acc;
    }
};

template <int FMT>
__device__ float trilinear_at(const HashView &h, const BlockReader<FMT> &rd,
                              const typename Vox<FMT>::S *sdf, float qx, float qy, float qz)
{
    const float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    Cube<FMT> cb;
    cb.fetch(h, rd, ix, iy, iz, ix + 1, iy + 1, iz + 1);
    return cb.trilinear(sdf, ix, iy, iz, qx - fx, qy - fy, qz - fz);
}

template <int FMT>
__global__ __launch_bounds__(256) void k_raycast(RaycastArgs a)
{
    const FrameGeom &g = a.fg;
    int tx, ty;
    if (!xcd_tile((g.W + 15) / 16, (g.H + 15) / 16, tx, ty)) return;  // whole workgroup
    // the macro-cell bitmap, staged in LDS: empty-space tests cost an LDS read
    __shared__ uint32_t s_macro[kMacroWords];
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.h.macro);
        uint4 *dst = reinterpret_cast<uint4 *>(s_macro);
        for (int i = threadIdx.x; i < kMacroWords / 4; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    // a workgroup covers 16 x 16 pixels, each wave an 8 x 8 quadrant of it
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int u = tx * 16 + (wave & 1) * 8 + (lane & 7);
    const int v = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (u >= g.W || v >= g.H) return;
    const int64_t pix = (int64_t)v * g.W + u;

    // binary64 ray set-up, rounded once
    const double cdx = ((double)u - g.cxd) / g.fxd, cdy = ((double)v - g.cyd) / g.fyd;
    const double len = sqrt(cdx * cdx + cdy * cdy + 1.0);
    double dir[3];
#pragma unroll
    for (int c = 0; c < 3; c++) dir[c] = (g.Rwc[3 * c] * cdx + g.Rwc[3 * c + 1] * cdy + g.Rwc[3 * c + 2]) / len;
    const float ox = (float)(g.twc[0] / g.s), oy = (float)(g.twc[1] / g.s), oz = (float)(g.twc[2] / g.s);
    const float dx = (float)(dir[0] / g.s), dy = (float)(dir[1] / g.s), dz = (float)(dir[2] / g.s);
    const float t_near = (float)((double)g.z_near * len), t_far = (float)((double)g.z_far * len);
    const float s = g.s_f, mu = g.mu_f, bs = 8.0f * g.s_f;
    const int fine_budget = (int)ceilf(bs / mu) + 1;
    const int cap = (int)((t_far - t_near) / s) * 4 + 1000;
    // reciprocal direction for the macro-cell exit
    const float idx = 1.0f / dx, idy = 1.0f / dy, idz = 1.0f / dz;

    BlockReader<FMT> rd(a.h, a.sdf);
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
                const float e = 1e-3f;
                const float lx = (float)((bx >> kMacroShift) * 32) - 0.5f;
                const float ly = (float)((by >> kMacroShift) * 32) - 0.5f;
                const float lz = (float)((bz >> kMacroShift) * 32) - 0.5f;
                const float tx = dx > 0.0f ? (lx + 32.0f - e - ox) * idx
                                 : dx < 0.0f ? (lx + e - ox) * idx : INFINITY;
                const float ty = dy > 0.0f ? (ly + 32.0f - e - oy) * idy
                                 : dy < 0.0f ? (ly + e - oy) * idy : INFINITY;
                const float tz = dz > 0.0f ? (lz + 32.0f - e - oz) * idz
                                 : dz < 0.0f ? (lz + e - oz) * idz : INFINITY;
                const float t_exit = fminf(tx, fminf(ty, tz));
                const float m = fmaxf(ceilf((t_exit - t) / bs), 1.0f);
                t = fmaf(m, bs, t);
                continue;
            }
            float F;
            if (!rd.nearest(qx, qy, qz, F)) t += bs;
            else { t = fmaxf(t - bs, t_near); state = RC_FINE; fine_miss = 0; }
            continue;
        }
        float F;
        const bool found = rd.nearest(qx, qy, qz, F);
        if (state == RC_FINE) {
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
    if (state == RC_BEHIND) {
        const auto *sdf = (const typename Vox<FMT>::S *)a.sdf;
#pragma unroll
        for (int k = 0; k < 2; k++)
            t = fmaf(trilinear_at<FMT>(a.h, rd, sdf, fmaf(t, dx, ox), fmaf(t, dy, oy), fmaf(t, dz, oz)), mu, t);
        const float qx = fmaf(t, dx, ox), qy = fmaf(t, dy, oy), qz = fmaf(t, dz, oz);
        P = make_float4((float)(g.twc[0] + (double)t * dir[0]), (float)(g.twc[1] + (double)t * dir[1]),
                        (float)(g.twc[2] + (double)t * dir[2]), 1.0f);
        // the six samples q +- e_a read voxels floor(q) - 1 .. floor(q) + 2
        const float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
        const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
        const float rx = qx - fx, ry = qy - fy, rz = qz - fz;
        Cube<FMT> cb;
        cb.fetch(a.h, rd, ix - 1, iy - 1, iz - 1, ix + 2, iy + 2, iz + 2);
        const float gx = cb.trilinear(sdf, ix + 1, iy, iz, rx, ry, rz) - cb.trilinear(sdf, ix - 1, iy, iz, rx, ry, rz);
        const float gy = cb.trilinear(sdf, ix, iy + 1, iz, rx, ry, rz) - cb.trilinear(sdf, ix, iy - 1, iz, rx, ry, rz);
        const float gz = cb.trilinear(sdf, ix, iy, iz + 1, rx, ry, rz) - cb.trilinear(sdf, ix, iy, iz - 1, rx, ry, rz);
        const float n2 = gx * gx + gy * gy + gz * gz;
        if (n2 > 0.0f) {
            const float r = 1.0f / sqrtf(n2);
            N = make_float4(gx * r, gy * r, gz * r, 1.0f);
        }
    }
    a.pts[pix] = P;
    a.nrm[pix] = N;
}

hipError_t launch_raycast(int fmt, const RaycastArgs &a, hipStream_t st)
{
    const int grid = xcd_grid(((a.fg.W + 15) / 16) * ((a.fg.H + 15) / 16));
    switch (fmt) {
    case ITM_VOX_F32: k_raycast<ITM_VOX_F32><<<grid, 256, 0, st>>>(a); break;
    case ITM_VOX_F16: k_raycast<ITM_VOX_F16><<<grid, 256, 0, st>>>(a); break;
    default: k_raycast<ITM_VOX_S16U8><<<grid, 256, 0, st>>>(a); break;
    }
    return hipGetLastError();
}

}  // namespace itm
