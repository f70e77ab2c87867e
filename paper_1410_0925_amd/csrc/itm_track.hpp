// Depth tracker (itm_track.hip): arguments of its kernels.
#pragma once

#include "itm_internal.hpp"

namespace itm {

// depth tracker (itm_track.hip)
constexpr int kTrackLevels = 4;
constexpr int kIcpSums = 29;      // upper triangle of A (21), g (6), sum d^2, pairs
constexpr int kIcpThreads = 1024; // threads per workgroup of k_icp_step

struct PoseInit {
    double T[16];        // the pose to start from (row-major camera -> world)
    double *pose;        // device double[16]
    int32_t *stop;       // device int32[kTrackLevels], cleared
    int32_t *steps;      // device int32, cleared
    uint32_t *done;      // device uint32, cleared
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
    double *pose;                // current estimate, device double[16]; moved by the step
    int32_t *stop;               // the level's stop flag (read even when update == 0)
    int32_t *steps;              // steps taken, or nullptr (then update == 0)
    float *part;                 // per-workgroup sums, sum k of workgroup j at part[k * part_stride + j]
    int32_t part_stride;         // >= the grid
    uint32_t *done;              // workgroups finished; zero between launches
    double *sys;                 // out: device double[kIcpSums], the summed system
    int32_t min_inliers;         // fewer pairs stop the level
    int32_t update;              // 0: sums only
};

hipError_t launch_track_init(const PoseInit &a, hipStream_t st);
hipError_t launch_icp_step(const IcpArgs &a, int grid, hipStream_t st);

}  // namespace itm
