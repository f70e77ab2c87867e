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
// consecutive samples of a ray mostly fall in the same block.
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
    // F at lattice voxel (vx, vy, vz); returns false (F = 1) when unallocated
    __device__ bool voxel(int vx, int vy, int vz, float &F)
    {
        const int32_t p = block(vx >> 3, vy >> 3, vz >> 3);
        if (p < 0) { F = 1.0f; return false; }
        F = Vox<FMT>::to_f(sdf[(int64_t)p * kBlockVox + (vx & 7) + 8 * (vy & 7) + 64 * (vz & 7)]);
        return true;
    }
    __device__ bool nearest(float qx, float qy, float qz, float &F)
    {
        return voxel((int)floorf(qx + 0.5f), (int)floorf(qy + 0.5f), (int)floorf(qz + 0.5f), F);
    }
    __device__ float trilinear(float qx, float qy, float qz)
    {
        const float flx = floorf(qx), fly = floorf(qy), flz = floorf(qz);
        const int ix = (int)flx, iy = (int)fly, iz = (int)flz;
        const float rx = qx - flx, ry = qy - fly, rz = qz - flz;
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
            float F;
            voxel(ix + dx, iy + dy, iz + dz, F);
            const float w = (dx ? rx : 1.0f - rx) * (dy ? ry : 1.0f - ry) * (dz ? rz : 1.0f - rz);
            acc = fmaf(w, F, acc);
        }
        return acc;
    }
};

template <int FMT>
__global__ __launch_bounds__(256) void k_raycast(RaycastArgs a)
{
    const FrameGeom &g = a.fg;
    const int u = blockIdx.x * 16 + (threadIdx.x & 15);
    const int v = blockIdx.y * 16 + (threadIdx.x >> 4);
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

    BlockReader<FMT> rd(a.h, a.sdf);
    float t = t_near;
    int state = RC_COARSE, fine_miss = 0;
    for (int it = 0; it < cap && t < t_far; it++) {
        const float qx = fmaf(t, dx, ox), qy = fmaf(t, dy, oy), qz = fmaf(t, dz, oz);
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
    if (state == RC_BEHIND) {
#pragma unroll
        for (int k = 0; k < 2; k++)
            t = fmaf(rd.trilinear(fmaf(t, dx, ox), fmaf(t, dy, oy), fmaf(t, dz, oz)), mu, t);
        const float qx = fmaf(t, dx, ox), qy = fmaf(t, dy, oy), qz = fmaf(t, dz, oz);
        P = make_float4((float)(g.twc[0] + (double)t * dir[0]), (float)(g.twc[1] + (double)t * dir[1]),
                        (float)(g.twc[2] + (double)t * dir[2]), 1.0f);
        const float gx = rd.trilinear(qx + 1.0f, qy, qz) - rd.trilinear(qx - 1.0f, qy, qz);
        const float gy = rd.trilinear(qx, qy + 1.0f, qz) - rd.trilinear(qx, qy - 1.0f, qz);
        const float gz = rd.trilinear(qx, qy, qz + 1.0f) - rd.trilinear(qx, qy, qz - 1.0f);
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
    dim3 grid((a.fg.W + 15) / 16, (a.fg.H + 15) / 16);
    switch (fmt) {
    case ITM_VOX_F32: k_raycast<ITM_VOX_F32><<<grid, 256, 0, st>>>(a); break;
    case ITM_VOX_F16: k_raycast<ITM_VOX_F16><<<grid, 256, 0, st>>>(a); break;
    default: k_raycast<ITM_VOX_S16U8><<<grid, 256, 0, st>>>(a); break;
    }
    return hipGetLastError();
}

}  // namespace itm
