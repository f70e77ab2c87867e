// Depth tracker (section "Tracking", the depth tracker): point-to-plane alignment
// of a depth image to the surface a raycast rendered from a reference pose, by
// Gauss-Newton steps over a resolution hierarchy.
//
//   k_icp_sums     per pixel of a level (level l reads input pixel (2^l u, 2^l v):
//                  the hierarchy by decimation needs no images of its own):
//                  back-project with the level's intrinsics, move by
//                  the current pose, project into the reference view, pair with
//                  the nearest reference pixel, and accumulate J J^T (21), J d
//                  (6), d^2 and the pair count in float32; one float32 partial
//                  per workgroup
//   k_icp_solve    one workgroup: the partials summed in float64 in a fixed order,
//                  the 6 x 6 system solved by Cholesky, the pose moved by
//                  (exp([w]x), v) -- all on the GPU, so the steps of a level run
//                  back to back without the host
// The current pose lives in device memory (float64, row-major 4 x 4); a level
// that runs out of pairs sets its stop flag, after which the level's remaining
// launches return at once.
#include "itm_track.hpp"

namespace itm {

__global__ void k_track_init(PoseInit a)
{
    if (threadIdx.x < 16) a.pose[threadIdx.x] = a.T[threadIdx.x];
    if (threadIdx.x < kTrackLevels) a.stop[threadIdx.x] = 0;
    if (threadIdx.x == 0) *a.steps = 0;
}

__global__ __launch_bounds__(256) void k_icp_sums(IcpArgs a)
{
    float acc[kIcpSums];
#pragma unroll
    for (int k = 0; k < kIcpSums; k++) acc[k] = 0.0f;
    if (!(a.stop && *a.stop)) {   // uniform
        float R[9], t[3];
#pragma unroll
        for (int i = 0; i < 3; i++) {
#pragma unroll
            for (int j = 0; j < 3; j++) R[3 * i + j] = (float)a.pose[4 * i + j];
            t[i] = (float)a.pose[4 * i + 3];
        }
        const int n_px = a.wl * a.hl;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_px; i += gridDim.x * blockDim.x) {
            const int u = i % a.wl, v = i / a.wl;
            const float d = a.depth[(int64_t)(v << a.level) * a.W + (u << a.level)];
            if (!(d > 0.0f) || isinf(d)) continue;
            const float p0 = d * ((float)u - a.cxl) / a.fxl, p1 = d * ((float)v - a.cyl) / a.fyl, p2 = d;
            float P[3], X[3];
#pragma unroll
            for (int c = 0; c < 3; c++) P[c] = R[3 * c] * p0 + R[3 * c + 1] * p1 + R[3 * c + 2] * p2 + t[c];
            const float q0 = P[0] - a.tr[0], q1 = P[1] - a.tr[1], q2 = P[2] - a.tr[2];
#pragma unroll
            for (int c = 0; c < 3; c++) X[c] = a.Rr[c] * q0 + a.Rr[3 + c] * q1 + a.Rr[6 + c] * q2;
            if (!(X[2] > 0.0f)) continue;
            const float x = a.fx * X[0] / X[2] + a.cx, y = a.fy * X[1] / X[2] + a.cy;
            const float xf = floorf(x + 0.5f), yf = floorf(y + 0.5f);
            if (!(xf >= 0.0f && xf <= (float)(a.W - 1) && yf >= 0.0f && yf <= (float)(a.H - 1))) continue;
            const int64_t q = (int64_t)yf * a.W + (int64_t)xf;
            const float4 V = a.V[q], N = a.N[q];
            if (!(V.w > 0.0f) || !(N.w > 0.0f)) continue;
            const float e0 = P[0] - V.x, e1 = P[1] - V.y, e2 = P[2] - V.z;
            if (sqrtf(e0 * e0 + e1 * e1 + e2 * e2) > a.dist) continue;
            const float r = e0 * N.x + e1 * N.y + e2 * N.z;
            const float J[6] = {P[1] * N.z - P[2] * N.y, P[2] * N.x - P[0] * N.z, P[0] * N.y - P[1] * N.x,
                                N.x, N.y, N.z};
            int k = 0;
#pragma unroll
            for (int m = 0; m < 6; m++)
#pragma unroll
                for (int j = m; j < 6; j++) acc[k++] += J[m] * J[j];
#pragma unroll
            for (int m = 0; m < 6; m++) acc[21 + m] += J[m] * r;
            acc[27] += r * r;
            acc[28] += 1.0f;
        }
    }
    // workgroup sums: within each wave by butterfly, then across the 4 waves
    __shared__ float s_w[4][kIcpSums];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < kIcpSums; k++) {
        float x = acc[k];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
        if (lane == 0) s_w[wave][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < kIcpSums) {
        const int k = threadIdx.x;
        a.part[(int64_t)blockIdx.x * kIcpSums + k] = ((s_w[0][k] + s_w[1][k]) + s_w[2][k]) + s_w[3][k];
    }
}

// Solve the 6 x 6 system (upper triangle packed row by row) by Cholesky; false
// when it is not positive definite.
__device__ bool solve6(const double *Aup, const double *b, double *x)
{
    double A[36], L[36], y[6];
    int k = 0;
    for (int i = 0; i < 6; i++)
        for (int j = i; j < 6; j++) {
            A[6 * i + j] = Aup[k];
            A[6 * j + i] = Aup[k];
            k++;
        }
    for (int i = 0; i < 36; i++) L[i] = 0.0;
    for (int j = 0; j < 6; j++) {
        double s = A[6 * j + j];
        for (int m = 0; m < j; m++) s -= L[6 * j + m] * L[6 * j + m];
        if (!(s > 0.0)) return false;
        L[6 * j + j] = sqrt(s);
        for (int i = j + 1; i < 6; i++) {
            double r = A[6 * i + j];
            for (int m = 0; m < j; m++) r -= L[6 * i + m] * L[6 * j + m];
            L[6 * i + j] = r / L[6 * j + j];
        }
    }
    for (int i = 0; i < 6; i++) {
        double s = b[i];
        for (int m = 0; m < i; m++) s -= L[6 * i + m] * y[m];
        y[i] = s / L[6 * i + i];
    }
    for (int i = 5; i >= 0; i--) {
        double s = y[i];
        for (int m = i + 1; m < 6; m++) s -= L[6 * m + i] * x[m];
        x[i] = s / L[6 * i + i];
    }
    return true;
}

// T <- (exp([w]x), v) T, the rotation by Rodrigues' formula
__device__ void pose_step(const double *xi, double *T)
{
    const double th = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
    double Ri[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (th > 0.0) {
        const double kx = xi[0] / th, ky = xi[1] / th, kz = xi[2] / th;
        const double c = cos(th), s = sin(th), c1 = 1.0 - c;
        // I + s [k]x + (1 - c) [k]x^2, with [k]x^2 = k k^T - I
        const double kk[3] = {kx, ky, kz};
        const double Kx[9] = {0, -kz, ky, kz, 0, -kx, -ky, kx, 0};
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                Ri[3 * i + j] = (i == j ? 1.0 : 0.0) + s * Kx[3 * i + j] + c1 * (kk[i] * kk[j] - (i == j ? 1.0 : 0.0));
    }
    double R[9], t[3];
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) R[3 * i + j] = T[4 * i + j];
        t[i] = T[4 * i + 3];
    }
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++)
            T[4 * i + j] = Ri[3 * i] * R[j] + Ri[3 * i + 1] * R[3 + j] + Ri[3 * i + 2] * R[6 + j];
        T[4 * i + 3] = Ri[3 * i] * t[0] + Ri[3 * i + 1] * t[1] + Ri[3 * i + 2] * t[2] + xi[3 + i];
    }
}

// 32 threads per component: thread (k, l) sums partials l, l + 32, ... of
// component k, then the wave adds its 32 in a fixed butterfly -- the same order
// every call
__global__ __launch_bounds__(1024) void k_icp_solve(SolveArgs a)
{
    if (a.stop && *a.stop) return;   // the level has stopped: its last system stays
    __shared__ double s_sys[kIcpSums];
    const int k = threadIdx.x >> 5, l = threadIdx.x & 31;
    double acc = 0.0;
    if (k < kIcpSums)
        for (int j = l; j < a.n_part; j += 32) acc += (double)a.part[(int64_t)j * kIcpSums + k];
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 32);
    if (k < kIcpSums && l == 0) {
        s_sys[k] = acc;
        a.sys[k] = acc;
    }
    __syncthreads();
    if (threadIdx.x != 0 || !a.update) return;
    double xi[6], b[6];
    for (int i = 0; i < 6; i++) b[i] = -s_sys[21 + i];
    if (s_sys[28] < (double)a.min_inliers || !solve6(s_sys, b, xi)) {
        *a.stop = 1;
        return;
    }
    double T[16];
    for (int i = 0; i < 16; i++) T[i] = a.pose[i];
    pose_step(xi, T);
    for (int i = 0; i < 12; i++) a.pose[i] = T[i];
    *a.steps += 1;
}

hipError_t launch_track_init(const PoseInit &a, hipStream_t st)
{
    k_track_init<<<1, 64, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_icp_sums(const IcpArgs &a, int grid, hipStream_t st)
{
    launch_k(k_icp_sums, grid, 256, st, a);
    return hipGetLastError();
}

hipError_t launch_icp_solve(const SolveArgs &a, hipStream_t st)
{
    launch_k(k_icp_solve, 1, 1024, st, a);
    return hipGetLastError();
}

}  // namespace itm
