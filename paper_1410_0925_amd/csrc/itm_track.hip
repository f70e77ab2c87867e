// Depth tracker (section "Tracking", the depth tracker): point-to-plane alignment
// of a depth image to the surface a raycast rendered from a reference pose, by
// Gauss-Newton steps over a resolution hierarchy.
//
//   k_icp_step     one Gauss-Newton step.  Per pixel of a level (level l reads
//                  input pixel (2^l u, 2^l v): the hierarchy by decimation needs
//                  no images of its own): back-project with the level's
//                  intrinsics, move by the current pose, project into the
//                  reference view, pair with the nearest reference pixel, and
//                  accumulate J J^T (21), J d (6), d^2 and the pair count in
//                  float32; one float32 partial per workgroup.  The workgroup
//                  that finishes last sums the partials in float64 in a fixed
//                  order, solves the 6 x 6 system by Cholesky and moves the pose
//                  by (exp([w]x), v) -- all on the GPU, so the steps of a level
//                  run back to back, one launch each, without the host
// The current pose lives in device memory (float64, row-major 4 x 4); a level
// that runs out of pairs sets its stop flag, after which the level's remaining
// launches return at once.
#include "itm_track.hpp"

namespace itm {

static_assert(kIcpSums <= kWave, "the partials are written by the first wave");
static_assert(kIcpThreads >= 32 * kIcpSums, "the last workgroup gives each sum 32 threads");
constexpr int kIcpWaves = kIcpThreads / kWave;

__global__ void k_track_init(PoseInit a)
{
    if (threadIdx.x < 16) a.pose[threadIdx.x] = a.T[threadIdx.x];
    if (threadIdx.x < kTrackLevels) a.stop[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        *a.steps = 0;
        *a.done = 0;
    }
}

// lane l's value of v from lane l ^ 15 (ctrl 0x140, mirror within 16 lanes),
// l ^ 7 (0x141, mirror within 8 lanes), l ^ 2 (0x4e) or l ^ 1 (0xb1) by DPP
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// One halving exchange over the lane bit that the DPP pattern flips: a lane
// with the bit set keeps the upper half of its H pairs (x[i], x[i + H]), a lane
// without it the lower half, each adding its partner's copy of the half it keeps.
template <int CTRL, int H>
__device__ __forceinline__ void halve_dpp(float *x, bool up)
{
#pragma unroll
    for (int i = 0; i < H; i++) {
        const float lo = x[i] + dpp_f<CTRL>(x[i]), hi = x[i + H] + dpp_f<CTRL>(x[i + H]);
        x[i] = up ? hi : lo;
    }
}

// Sum 32 values over the 64 lanes of a wave by recursive halving: each exchange
// hands the partner the half of the values it keeps, so 31 exchanges leave one
// value per lane and one more finishes the sum.  Lane l returns the sum of value
// l >> 1.  The exchanges over lane bits 5 and 4 are lane swaps (the swapped
// halves land where they are kept), the rest DPP moves.
__device__ __forceinline__ float wave_sum32(float (&x)[32], int lane)
{
#pragma unroll
    for (int i = 0; i < 16; i++) {   // bit 5: lanes 0-31 keep values 0-15
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[i]), __float_as_uint(x[i + 16]), false,
                                                        false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 8; i++) {    // bit 4: even rows of 16 lanes keep the lower half
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[i]), __float_as_uint(x[i + 8]), false,
                                                        false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    halve_dpp<0x140, 4>(x, lane & 8);   // bit 3, partner l ^ 15
    halve_dpp<0x141, 2>(x, lane & 4);   // bit 2, partner l ^ 7
    halve_dpp<0x4e, 1>(x, lane & 2);    // bit 1, partner l ^ 2
    return x[0] + dpp_f<0xb1>(x[0]);   // bit 0, partner l ^ 1
}

// depth of the level's pixel i (row-major over wl x hl)
__device__ __forceinline__ float level_depth(const IcpArgs &a, int i)
{
    const int u = i % a.wl, v = i / a.wl;
    return a.depth[(int64_t)(v << a.level) * a.W + (u << a.level)];
}

// pair the level's pixel i, of depth d, with the nearest reference pixel and add
// its terms to acc (nothing for a pixel without depth or without a pair)
__device__ __forceinline__ void icp_pixel(const IcpArgs &a, const float *R, const float *t, int i, float d,
                                          float *acc)
{
    if (!(d > 0.0f) || isinf(d)) return;
    const int u = i % a.wl, v = i / a.wl;
    const float p0 = d * ((float)u - a.cxl) / a.fxl, p1 = d * ((float)v - a.cyl) / a.fyl, p2 = d;
    float P[3], X[3];
#pragma unroll
    for (int c = 0; c < 3; c++) P[c] = R[3 * c] * p0 + R[3 * c + 1] * p1 + R[3 * c + 2] * p2 + t[c];
    const float q0 = P[0] - a.tr[0], q1 = P[1] - a.tr[1], q2 = P[2] - a.tr[2];
#pragma unroll
    for (int c = 0; c < 3; c++) X[c] = a.Rr[c] * q0 + a.Rr[3 + c] * q1 + a.Rr[6 + c] * q2;
    if (!(X[2] > 0.0f)) return;
    const float x = a.fx * X[0] / X[2] + a.cx, y = a.fy * X[1] / X[2] + a.cy;
    const float xf = floorf(x + 0.5f), yf = floorf(y + 0.5f);
    if (!(xf >= 0.0f && xf <= (float)(a.W - 1) && yf >= 0.0f && yf <= (float)(a.H - 1))) return;
    const int64_t q = (int64_t)yf * a.W + (int64_t)xf;
    const float4 V = a.V[q], N = a.N[q];
    // both maps' texels are waited for together: without the empty statement the
    // tests below split them into three reads, and without the scheduling
    // barrier the first test is moved between the two reads, each waited for in turn
    asm volatile("" ::"v"(V.x), "v"(V.y), "v"(V.z), "v"(V.w), "v"(N.x), "v"(N.y), "v"(N.z), "v"(N.w));
    __builtin_amdgcn_sched_barrier(0);
    if (!(V.w > 0.0f) || !(N.w > 0.0f)) return;
    const float e0 = P[0] - V.x, e1 = P[1] - V.y, e2 = P[2] - V.z;
    if (sqrtf(e0 * e0 + e1 * e1 + e2 * e2) > a.dist) return;
    const float r = e0 * N.x + e1 * N.y + e2 * N.z;
    const float J[6] = {P[1] * N.z - P[2] * N.y, P[2] * N.x - P[0] * N.z, P[0] * N.y - P[1] * N.x, N.x, N.y, N.z};
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

// Solve the 6 x 6 system (upper triangle packed row by row) by Cholesky; false
// when it is not positive definite.  Each pivot is inverted once and multiplied
// by (one serial float64 thread: 6 divisions rather than 33).
__device__ bool solve6(const double *Aup, const double *b, double *x)
{
    double A[36], L[36], y[6], inv[6];
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
        inv[j] = 1.0 / L[6 * j + j];
        for (int i = j + 1; i < 6; i++) {
            double r = A[6 * i + j];
            for (int m = 0; m < j; m++) r -= L[6 * i + m] * L[6 * j + m];
            L[6 * i + j] = r * inv[j];
        }
    }
    for (int i = 0; i < 6; i++) {
        double s = b[i];
        for (int m = 0; m < i; m++) s -= L[6 * i + m] * y[m];
        y[i] = s * inv[i];
    }
    for (int i = 5; i >= 0; i--) {
        double s = y[i];
        for (int m = i + 1; m < 6; m++) s -= L[6 * m + i] * x[m];
        x[i] = s * inv[i];
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

__global__ __launch_bounds__(kIcpThreads) void k_icp_step(IcpArgs a)
{
    const int n_px = a.wl * a.hl, stride = gridDim.x * kIcpThreads;
    int i = blockIdx.x * kIcpThreads + threadIdx.x;
    // The first pixel's depth, the stop flag and the pose are all requested
    // before any of them is waited for.  Every depth read is of a valid address,
    // clamped rather than branched around, so that the compiler issues it early.
    float d = level_depth(a, min(i, n_px - 1));
    double T0[12];
#pragma unroll
    for (int k = 0; k < 12; k++) T0[k] = a.pose[k];
    const int32_t stopped = *a.stop;
    // one wait for the flag and the pose (the depth read stays in flight): the
    // compiler would otherwise read the pose only after the branch below
    asm volatile("" ::"s"(stopped), "s"(T0[0]), "s"(T0[1]), "s"(T0[2]), "s"(T0[3]), "s"(T0[4]), "s"(T0[5]),
                 "s"(T0[6]), "s"(T0[7]), "s"(T0[8]), "s"(T0[9]), "s"(T0[10]), "s"(T0[11]));
    if (stopped) return;   // uniform: the level's pose and last system stay
    float R[9], t[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
#pragma unroll
        for (int c = 0; c < 3; c++) R[3 * r + c] = (float)T0[4 * r + c];
        t[r] = (float)T0[4 * r + 3];
    }
    float acc[32];
#pragma unroll
    for (int k = 0; k < 32; k++) acc[k] = 0.0f;
    for (; i < n_px; i += stride) {
        const float dn = level_depth(a, min(i + stride, n_px - 1));   // the next pixel's, in flight meanwhile
        icp_pixel(a, R, t, i, d, acc);
        d = dn;
    }

    // workgroup sums: within each wave by halving, then across the waves in order
    __shared__ float s_w[kIcpWaves][32];
    __shared__ uint32_t s_ticket;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    {
        const float x = wave_sum32(acc, lane);   // sum lane >> 1
        if (!(lane & 1)) s_w[wave][lane >> 1] = x;
    }
    __syncthreads();
    if (threadIdx.x < kIcpSums) {
        const int k = threadIdx.x;
        float s = s_w[0][k];
#pragma unroll
        for (int w = 1; w < kIcpWaves; w++) s += s_w[w][k];
        // The partials are the only data one workgroup hands another, so they
        // are device-scope stores (written through to where every XCD's L2
        // reads device-scope loads from), and the store is complete before the
        // ticket below is drawn.  A release fence would instead write back the
        // XCD's whole L2, and an acquire fence drop the lines that the
        // workgroups still running read: measured, 5 us more per step.
        __hip_atomic_store(&a.part[(int64_t)k * a.part_stride + blockIdx.x], s, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the store above is complete
    }
    __syncthreads();
    if (threadIdx.x == 0) s_ticket = __hip_atomic_fetch_add(a.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (s_ticket != gridDim.x - 1) return;   // uniform: not the last workgroup

    // The last workgroup: every other partial was complete before its ticket,
    // and it reads them with device-scope loads.
    if (threadIdx.x == 0)   // the count starts from zero at the next launch
        __hip_atomic_store(a.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Thread (k, l) adds partials l, l + 32, ... of sum k in float64, eight loads
    // in flight at a time, and the 32 threads of a sum are added by a fixed
    // butterfly -- the same order at every call.
    __shared__ double s_sys[32];
    {
        const int k = threadIdx.x >> 5, l = threadIdx.x & 31, n = gridDim.x;
        double x = 0.0;
        if (k < kIcpSums) {
            const float *p = a.part + (int64_t)k * a.part_stride;
            for (int j0 = l; j0 < n; j0 += 8 * 32) {
                float v[8];
#pragma unroll
                for (int q = 0; q < 8; q++)
                    v[q] = __hip_atomic_load(&p[min(j0 + 32 * q, n - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int q = 0; q < 8; q++) x += j0 + 32 * q < n ? (double)v[q] : 0.0;
            }
        }
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) x += __shfl_xor(x, o, 32);
        if (k < kIcpSums && l == 0) {
            s_sys[k] = x;
            a.sys[k] = x;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0 || !a.update) return;
    double xi[6], b[6];
    for (int k = 0; k < 6; k++) b[k] = -s_sys[21 + k];
    if (s_sys[28] < (double)a.min_inliers || !solve6(s_sys, b, xi)) {
        *a.stop = 1;
        return;
    }
    double T[16];
    for (int k = 0; k < 16; k++) T[k] = a.pose[k];
    pose_step(xi, T);
    for (int k = 0; k < 12; k++) a.pose[k] = T[k];
    *a.steps += 1;
}

hipError_t launch_track_init(const PoseInit &a, hipStream_t st)
{
    k_track_init<<<1, 64, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_icp_step(const IcpArgs &a, int grid, hipStream_t st)
{
    launch_k(k_icp_step, grid, kIcpThreads, st, a);
    return hipGetLastError();
}

}  // namespace itm
