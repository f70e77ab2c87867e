// Depth tracker (itm_track.hip): arguments of its kernels.
#pragma once

#include "itm_internal.hpp"

namespace itm {

// depth tracker (itm_track.hip)
constexpr int kTrackLevels = 4;
constexpr int kIcpSums = 29;   // upper triangle of A (21), g (6), sum d^2, pairs

struct PoseInit {
    double T[16];        // the pose to start from (row-major camera -> world)
    double *pose;        // device double[16]
    int32_t *stop;       // device int32[kTrackLevels], cleared
    int32_t *steps;      // device int32, cleared
};

struct IcpArgs {
    const float *depth;          // the input depth image, W x H
    int32_t level, wl, hl;       // level l: pixel (u, v) < (wl, hl) is input pixel (2^l u, 2^l v)
    float fxl, fyl, cxl, cyl;    // the level's intrinsics
    float fx, fy, cx, cy;        // the reference view (full resolution W x H)
    int32_t W, H;                // input and reference size
    const float4 *V, *N;         // reference maps, world frame, w > 0 = hit
    float Rr[9], tr[3];          // reference pose (camera -> world)
    float dist;                  // pairing distance
    const double *pose;          // current estimate, device double[16]
    const int32_t *stop;         // the level's stop flag, or nullptr
    float *part;                 // per-workgroup sums [grid][kIcpSums]
};

struct SolveArgs {
    const float *part;
    int32_t n_part;
    double *pose;
    int32_t *stop;               // nullptr with update == 0
    int32_t *steps;
    double *sys;                 // out: device double[kIcpSums]
    int32_t min_inliers;
    int32_t update;              // 0: sums only
};

hipError_t launch_track_init(const PoseInit &a, hipStream_t st);
hipError_t launch_icp_sums(const IcpArgs &a, int grid, hipStream_t st);
hipError_t launch_icp_solve(const SolveArgs &a, hipStream_t st);

}  // namespace itm
