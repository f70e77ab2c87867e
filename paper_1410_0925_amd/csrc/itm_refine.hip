// Learned block refiner: a 4-layer 3D convolutional network on bf16 MFMA.
//
// Every layer is the same operation: a 3^3 convolution from a 10^3 grid (the
// block with a one-voxel halo, or the 8^3 block zero-padded) to the 8^3 block,
// 16 input and 16 output channels (layer 1 uses 2 real input channels, layer 4
// one real output channel; the others hold zeros).  As an implicit GEMM per
// block: M = 512 voxels, N = 16 output channels, K = 27 taps x 16 channels, two
// taps per K step of gfx950's v_mfma_f32_16x16x32_bf16 (layer 1, with its 2 real
// input channels stored as 4, takes 8 taps per K step).  A workgroup of 16 waves
// takes a block; wave w owns the voxel tiles 2w, 2w + 1 of its 32 (16-voxel
// tiles), so each SIMD has 4 waves to overlap LDS reads and MFMA chains (the
// LDS footprint allows few workgroups per CU).  Activations live in LDS
// as bf16 [voxel][channel], so a lane's 8 K values are one 16-byte LDS read;
// weights are read from global memory (L1-resident) as bf16.
//
// Back-propagation reuses the same operation: the data gradient is the
// convolution of the output gradient with the tap-flipped, channel-transposed
// kernel; the weight gradient is, per tap, a 16 x 16 GEMM over the 512 voxels.
// Each block writes its gradient to its own row of a partial buffer; a second
// kernel sums the rows in a fixed order (deterministic) and, in a training step,
// applies Adam to the float32 master weights and re-rounds the bf16 copies.
#include <algorithm>

#include "itm_internal.hpp"

namespace itm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 16, kTaps = 27, kLayers = 4;
constexpr int kNW = kRefineWeights;
constexpr int kNP = kRefineParams;

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 16 x 16 x 32: a lane holds 8 consecutive K values of its row (A) / column (B)
__device__ __forceinline__ f32x4 mfma32(i32x4 a, i32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// LDS working set of one block (16-byte aligned rows: a lane's 8 channels are one
// read).  Training keeps all three hidden activations for the backward pass
// (92 KB, with the weight gradient's transposed copies 125 KB: one workgroup per
// CU); inference alternates two (42 KB: two 16-wave workgroups per CU).
template <int NACT>
struct alignas(16) RefineAct {
    uint16_t x0[1000 * 4];          // network input, 10^3 grid, channels F, W/max_w, 0, 0
    uint16_t act[NACT][512 * kC];   // layer l's output (8^3 x 16) in act[l % NACT]
    float centre[512];              // F of the block itself (float32), for the residual
};
struct alignas(16) RefineLds : RefineAct<3> {
    uint16_t grad[2][512 * kC];     // back-propagated gradient, ping-pong
};
using RefineLdsInf = RefineAct<2>;

// one wave's TPW tiles of a 3^3 convolution: acc[t] (lane: voxel 4 kq + r of tile
// TPW w + t, channel lane & 15) = sum over taps of A(tap) x W(tap).
// K order of one instruction (lane group kq = lane >> 4 holds K 8 kq .. 8 kq + 7):
//   layer 0 (4 stored input channels): taps 8 g + 2 kq and 8 g + 2 kq + 1, their
//            channels 0..3 each, g = 0..3 (taps past 26 read zeros);
//   layers 1..3 and data gradients (16 channels): tap 2 p + (kq >> 1), channels
//            8 (kq & 1) .. + 7, p = 0..13.
template <int TPW>
__device__ __forceinline__ void conv_tiles(const uint16_t *x0, const uint16_t *in, int layer,
                                           const uint16_t *Wl, bool flip, int wave, int lane,
                                           f32x4 acc[TPW])
{
    const int kq = lane >> 4, n = lane & 15;
    const i32x4 zero = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < TPW; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (layer == 0) {
#pragma unroll 1
        for (int g = 0; g < 4; g++) {
            const int ta = 8 * g + 2 * kq, tb = ta + 1;
            const bool va = ta < kTaps, vb = tb < kTaps;
            const uint2 wa = va ? *reinterpret_cast<const uint2 *>(&Wl[(ta * kC + n) * kC]) : make_uint2(0, 0);
            const uint2 wb = vb ? *reinterpret_cast<const uint2 *>(&Wl[(tb * kC + n) * kC]) : make_uint2(0, 0);
            const i32x4 b = {(int)wa.x, (int)wa.y, (int)wb.x, (int)wb.y};
            const int oa = (ta % 3) + 10 * ((ta / 3) % 3) + 100 * (ta / 9);
            const int ob = (tb % 3) + 10 * ((tb / 3) % 3) + 100 * (tb / 9);
#pragma unroll
            for (int t = 0; t < TPW; t++) {
                const int vox = (wave * TPW + t) * 16 + n;
                const int u = (vox & 7) + 10 * ((vox >> 3) & 7) + 100 * (vox >> 6);
                const uint2 xa = va ? *reinterpret_cast<const uint2 *>(&x0[(u + oa) * 4]) : make_uint2(0, 0);
                const uint2 xb = vb ? *reinterpret_cast<const uint2 *>(&x0[(u + ob) * 4]) : make_uint2(0, 0);
                const i32x4 a = {(int)xa.x, (int)xa.y, (int)xb.x, (int)xb.y};
                acc[t] = mfma32(a, b, acc[t]);
            }
        }
        return;
    }
    const int h = kq & 1;
#pragma unroll 1
    for (int p = 0; p < (kTaps + 1) / 2; p++) {
        const int tap = 2 * p + (kq >> 1);
        const bool valid = tap < kTaps;
        const int wt = flip ? kTaps - 1 - tap : tap;
        // B operand: 8 consecutive reduction channels of output column n
        const i32x4 b = valid ? *reinterpret_cast<const i32x4 *>(&Wl[(wt * kC + n) * kC + 8 * h]) : zero;
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
#pragma unroll
        for (int t = 0; t < TPW; t++) {
            const int vox = (wave * TPW + t) * 16 + n;
            const int ux = (vox & 7) + dx - 1, uy = ((vox >> 3) & 7) + dy - 1, uz = (vox >> 6) + dz - 1;
            const bool inside = valid && (unsigned)ux < 8u && (unsigned)uy < 8u && (unsigned)uz < 8u;
            const i32x4 a = inside ? *reinterpret_cast<const i32x4 *>(&in[(ux + 8 * uy + 64 * uz) * kC + 8 * h])
                                   : zero;
            acc[t] = mfma32(a, b, acc[t]);
        }
    }
}

// forward through the 4 layers; leaves activations in L.act and returns, for the
// lanes with output channel 0, the residual delta of their 4 voxels per tile
template <int NACT, int TPW>
__device__ void refine_forward(RefineAct<NACT> &L, const RefineParams &P, int wave, int lane, f32x4 delta[TPW])
{
    const int kq = lane >> 4, n = lane & 15;
    f32x4 acc[TPW];
    for (int l = 0; l < kLayers; l++) {
        const uint16_t *in = l == 0 ? nullptr : L.act[(l - 1) % NACT];
        conv_tiles<TPW>(L.x0, in, l, P.Wf + (size_t)l * kTaps * kC * kC, false, wave, lane, acc);
        const float b = P.bias[l * kC + n];
        if (l < kLayers - 1) {
#pragma unroll
            for (int t = 0; t < TPW; t++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int vox = (wave * TPW + t) * 16 + 4 * kq + r;
                    L.act[l % NACT][vox * kC + n] = to_bf16(fmaxf(acc[t][r] + b, 0.0f));
                }
        } else {
#pragma unroll
            for (int t = 0; t < TPW; t++)
#pragma unroll
                for (int r = 0; r < 4; r++) delta[t][r] = acc[t][r] + b;
        }
        __syncthreads();
    }
}

// fill L.x0 / L.centre from a float32 input block [2][10^3] in global memory
template <int NACT>
__device__ void load_input(RefineAct<NACT> &L, const float *in)
{
    for (int u = threadIdx.x; u < 1000; u += blockDim.x) {
        const float F = in[u], W = in[1000 + u];
        uint16_t *d = &L.x0[u * 4];
        d[0] = to_bf16(F);
        d[1] = to_bf16(W);
        d[2] = 0;
        d[3] = 0;
        const int x = u % 10, y = (u / 10) % 10, z = u / 100;
        if (x >= 1 && x <= 8 && y >= 1 && y <= 8 && z >= 1 && z <= 8)
            L.centre[(x - 1) + 8 * (y - 1) + 64 * (z - 1)] = F;
    }
}

// The inference kernels' workgroups: kInferWaves waves, kInferTPW voxel tiles each
constexpr int kInferWaves = 16;
constexpr int kInferTPW = 32 / kInferWaves;

// inference only: the refined F of each block
__global__ __launch_bounds__(kInferWaves * 64) void k_refine_infer(RefineArgs a)
{
    constexpr int TPW = kInferTPW;
    __shared__ RefineLdsInf L;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, n = lane & 15;
    for (int64_t blk = blockIdx.x; blk < a.n; blk += gridDim.x) {
        load_input(L, a.in + blk * 2000);
        __syncthreads();
        f32x4 delta[TPW];
        refine_forward<2, TPW>(L, a.P, wave, lane, delta);
        if (n == 0) {
#pragma unroll
            for (int t = 0; t < TPW; t++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int vox = (wave * TPW + t) * 16 + 4 * kq + r;
                    a.out[blk * 512 + vox] = fminf(fmaxf(L.centre[vox] + delta[t][r], -1.0f), 1.0f);
                }
        }
        __syncthreads();
    }
}

// The training kernel's LDS (all activations and the gradients) allows one
// workgroup per CU, so a block is split over 16 waves (4 per SIMD, 2 voxel tiles
// and about 2 weight-gradient taps each) to hide its LDS and MFMA latencies.
constexpr int kTrainWaves = 16;
constexpr int kTrainTPW = 32 / kTrainWaves;

// [channel][voxel] copies of a layer's output gradient and input for its weight
// gradient (rows padded by 8 elements, so the 16-byte reads of lanes with
// consecutive channels fall in different LDS banks)
constexpr int kRowT = 512 + 8;

// 8 bf16 of an x-row (x = 0..7) moved by s = -1, 0, +1 elements: element j of the
// result is element j + s of the row, zero outside it
__device__ __forceinline__ i32x4 shift_row(i32x4 r, int s)
{
    if (s == 0) return r;
    i32x4 o;
    if (s > 0) {
        o[0] = (int)__builtin_amdgcn_alignbit((uint32_t)r[1], (uint32_t)r[0], 16);
        o[1] = (int)__builtin_amdgcn_alignbit((uint32_t)r[2], (uint32_t)r[1], 16);
        o[2] = (int)__builtin_amdgcn_alignbit((uint32_t)r[3], (uint32_t)r[2], 16);
        o[3] = (int)__builtin_amdgcn_alignbit(0u, (uint32_t)r[3], 16);
    } else {
        o[0] = (int)__builtin_amdgcn_alignbit((uint32_t)r[0], 0u, 16);
        o[1] = (int)__builtin_amdgcn_alignbit((uint32_t)r[1], (uint32_t)r[0], 16);
        o[2] = (int)__builtin_amdgcn_alignbit((uint32_t)r[2], (uint32_t)r[1], 16);
        o[3] = (int)__builtin_amdgcn_alignbit((uint32_t)r[3], (uint32_t)r[2], 16);
    }
    return o;
}

// elements d .. d + 7 (d = 0, 1, 2) of the 16 bf16 in (r0, r1)
__device__ __forceinline__ i32x4 window8(i32x4 r0, i32x4 r1, int d)
{
    if (d == 0) return r0;
    if (d == 2) return i32x4{r0[1], r0[2], r0[3], r1[0]};
    i32x4 o;
    o[0] = (int)__builtin_amdgcn_alignbit((uint32_t)r0[1], (uint32_t)r0[0], 16);
    o[1] = (int)__builtin_amdgcn_alignbit((uint32_t)r0[2], (uint32_t)r0[1], 16);
    o[2] = (int)__builtin_amdgcn_alignbit((uint32_t)r0[3], (uint32_t)r0[2], 16);
    o[3] = (int)__builtin_amdgcn_alignbit((uint32_t)r1[0], (uint32_t)r0[3], 16);
    return o;
}

template <bool TRAIN>
__global__ __launch_bounds__(kTrainWaves * 64) void k_refine(RefineArgs a)
{
    constexpr int TPW = kTrainTPW;
    __shared__ RefineLds L;
    __shared__ __attribute__((aligned(16))) uint16_t s_gT[kC * kRowT];   // output gradient, [channel][voxel]
    __shared__ __attribute__((aligned(16))) uint16_t s_xT[kC * kRowT];   // layer input, [channel][voxel]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, n = lane & 15;
    for (int64_t blk = blockIdx.x; blk < a.n; blk += gridDim.x) {
        load_input(L, a.in + blk * 2000);
        __syncthreads();
        f32x4 delta[TPW];
        refine_forward<3, TPW>(L, a.P, wave, lane, delta);
        // residual, clamp, loss gradient (lanes with output channel 0)
        float sq = 0.0f, cnt = 0.0f;
        if (TRAIN) {
            for (int i = threadIdx.x; i < 512 * kC; i += blockDim.x) {
                L.grad[0][i] = 0;
                L.grad[1][i] = 0;
            }
            __syncthreads();
        }
        if (n == 0) {
#pragma unroll
            for (int t = 0; t < TPW; t++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int vox = (wave * TPW + t) * 16 + 4 * kq + r;
                    const float z = L.centre[vox] + delta[t][r];
                    const float Fo = fminf(fmaxf(z, -1.0f), 1.0f);
                    if (!TRAIN) {
                        a.out[blk * 512 + vox] = Fo;
                    } else {
                        const bool m = a.mask[blk * 512 + vox] != 0;
                        const float e = Fo - a.target[blk * 512 + vox];
                        if (m) { sq += e * e; cnt += 1.0f; }
                        const float g = (m && z > -1.0f && z < 1.0f) ? 2.0f * e : 0.0f;
                        L.grad[0][vox * kC] = to_bf16(g);
                        if (a.out) a.out[blk * 512 + vox] = Fo;
                    }
                }
        }
        if (!TRAIN) {
            __syncthreads();
            continue;
        }
        // loss partial: reduce over the wave, then over the waves in wave order
        __shared__ float red[2][kTrainWaves];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            sq += __shfl_xor(sq, o, 64);
            cnt += __shfl_xor(cnt, o, 64);
        }
        if (lane == 0) { red[0][wave] = sq; red[1][wave] = cnt; }
        __syncthreads();
        if (threadIdx.x == 0) {
            float s0 = 0.0f, s1 = 0.0f;
            for (int w = 0; w < kTrainWaves; w++) {
                s0 += red[0][w];
                s1 += red[1][w];
            }
            a.loss_part[blk * 2] = s0;
            a.loss_part[blk * 2 + 1] = s1;
        }
        float *gp = a.grad_part + blk * kNP;
        int cur = 0;
        for (int l = kLayers - 1; l >= 0; l--) {
            const uint16_t *G = L.grad[cur];
            // bias gradient: sum of the (bf16) output gradient over the voxels, by
            // the last wave (it has the fewest weight-gradient taps): lane = channel
            // + 16 quarter, each quarter's 128 voxels in order, the quarters
            // combined by a fixed butterfly
            if (wave == kTrainWaves - 1) {
                float s = 0.0f;
                for (int v = 128 * kq; v < 128 * (kq + 1); v++) s += from_bf16(G[v * kC + n]);
                s += __shfl_xor(s, 16, 64);
                s += __shfl_xor(s, 32, 64);
                if (kq == 0) gp[kNW + l * kC + n] = s;
            }
            // weight gradient, taps split over the waves: per tap a 16 x 16 GEMM
            // over the 512 voxels (M = output channel, N = input channel)
            const uint16_t *X = l == 0 ? nullptr : L.act[l - 1];
            if (l > 0) {
                // K = 32 voxels per step (4 x-rows); lane group kq takes row 4 ks + kq:
                // A = 8 voxels of the gradient's channel row, B = the input row at the
                // tap's (y, z) offset, moved by its x offset
                for (int i = threadIdx.x; i < 512 * kC; i += blockDim.x) {
                    s_gT[(i & 15) * kRowT + (i >> 4)] = G[i];
                    s_xT[(i & 15) * kRowT + (i >> 4)] = X[i];
                }
                __syncthreads();
                for (int tap = wave; tap < kTaps; tap += kTrainWaves) {
                    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
                    for (int ks = 0; ks < 16; ks++) {
                        const int row = 4 * ks + kq;   // y = row & 7, z = row >> 3
                        const i32x4 av = *reinterpret_cast<const i32x4 *>(&s_gT[n * kRowT + 8 * row]);
                        const int uy = (row & 7) + dy - 1, uz = (row >> 3) + dz - 1;
                        i32x4 bv = {0, 0, 0, 0};
                        if ((unsigned)uy < 8u && (unsigned)uz < 8u)
                            bv = shift_row(*reinterpret_cast<const i32x4 *>(&s_xT[n * kRowT + 8 * (uy + 8 * uz)]),
                                           dx - 1);
                        acc = mfma32(av, bv, acc);
                    }
#pragma unroll
                    for (int r = 0; r < 4; r++) gp[((l * kTaps + tap) * kC + 4 * kq + r) * kC + n] = acc[r];
                }
            } else {
                // layer 0's input is the 10^3 grid (4 stored channels): its copy is
                // [channel][z][y][x, padded to 16], and a tap's 8 inputs of a row are
                // elements dx .. dx + 7 of it (two 16-byte reads); channels past the
                // 4 stored read zeros
                for (int i = threadIdx.x; i < 512 * kC; i += blockDim.x) s_gT[(i & 15) * kRowT + (i >> 4)] = G[i];
                for (int i = threadIdx.x; i < 4 * 1000; i += blockDim.x) {
                    const int u = i >> 2, c = i & 3;
                    s_xT[((c * 10 + u / 100) * 10 + (u / 10) % 10) * 16 + u % 10] = L.x0[i];
                }
                __syncthreads();
                for (int tap = wave; tap < kTaps; tap += kTrainWaves) {
                    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
                    for (int ks = 0; ks < 16; ks++) {
                        const int row = 4 * ks + kq;
                        const i32x4 av = *reinterpret_cast<const i32x4 *>(&s_gT[n * kRowT + 8 * row]);
                        i32x4 bv = {0, 0, 0, 0};
                        if (n < 4) {
                            const uint16_t *r = &s_xT[((n * 10 + (row >> 3) + dz) * 10 + (row & 7) + dy) * 16];
                            bv = window8(*reinterpret_cast<const i32x4 *>(r), *reinterpret_cast<const i32x4 *>(r + 8), dx);
                        }
                        acc = mfma32(av, bv, acc);
                    }
#pragma unroll
                    for (int r = 0; r < 4; r++) gp[((l * kTaps + tap) * kC + 4 * kq + r) * kC + n] = acc[r];
                }
            }
            if (l == 0) break;
            // data gradient into the previous layer's output, masked by its ReLU
            f32x4 acc[TPW];
            conv_tiles<TPW>(L.x0, G, 1, a.P.Wt + (size_t)l * kTaps * kC * kC, true, wave, lane, acc);
            uint16_t *Gn = L.grad[cur ^ 1];
            const uint16_t *A = L.act[l - 1];
#pragma unroll
            for (int t = 0; t < TPW; t++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int vox = (wave * TPW + t) * 16 + 4 * kq + r;
                    const bool on = from_bf16(A[vox * kC + n]) > 0.0f;
                    Gn[vox * kC + n] = on ? to_bf16(acc[t][r]) : (uint16_t)0;
                }
            __syncthreads();
            cur ^= 1;
        }
        __syncthreads();
    }
}

// Sum the per-block partial gradients, divide by the batch's count of supervised
// voxels.  A workgroup takes 64 parameters; its 4 waves each add a contiguous
// quarter of the block rows (in row order), and the quarters are added in a fixed
// order, so the result does not depend on scheduling.
// Adam's constants for one step (bias corrections from the step count)
struct AdamConst {
    float lr, b1, b2, eps, c1, c2;
};

// Adam on float32 master weight p (value w0, moments m0 and v0) with gradient
// g, then its bf16 copies
__device__ __forceinline__ void adam_update(const AdamStep &ad, const AdamConst &k, int p, float g, float w0,
                                            float m0, float v0)
{
    const float mm = k.b1 * m0 + (1.0f - k.b1) * g;
    const float vv = k.b2 * v0 + (1.0f - k.b2) * g * g;
    ad.m[p] = mm;
    ad.v[p] = vv;
    const float w = w0 - k.lr * (mm / k.c1) / (sqrtf(vv / k.c2) + k.eps);
    ad.master[p] = w;
    if (p < kNW) {
        ad.Wf[p] = to_bf16(w);
        const int ci = p % kC, co = (p / kC) % kC, lt = p / (kC * kC);
        ad.Wt[(lt * kC + ci) * kC + co] = to_bf16(w);
    } else {
        ad.bias[p - kNW] = w;
    }
}

// The mean gradient (and with ADAM the step it drives): per parameter, the
// partial rows added in a fixed order, divided by the count of masked voxels
template <bool ADAM>
__global__ __launch_bounds__(256) void k_refine_reduce(const float *grad_part, const float *loss_part, int64_t n,
                                                       float *grad, float *loss, AdamStep ad, AdamConst k)
{
    __shared__ float part[4][64];
    __shared__ float s_inv;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    const int64_t r0 = n * q / 4, r1 = n * (q + 1) / 4;
    // the weight and its moments are read first, so that their round trip
    // overlaps the partial rows'
    float w0 = 0.0f, m0 = 0.0f, v0 = 0.0f;
    if (ADAM && q == 0 && p < kNP) {
        w0 = ad.master[p];
        m0 = ad.m[p];
        v0 = ad.v[p];
    }
    // the quarter's rows added in row order, sixteen loads in flight ahead of
    // the additions (the scheduling barrier keeps the compiler from moving the
    // first additions, and so their waits, between the loads)
    float acc = 0.0f;
    if (p < kNP) {
        int64_t b = r0;
        for (; b + 16 <= r1; b += 16) {
            float v[16];
#pragma unroll
            for (int j = 0; j < 16; j++) v[j] = grad_part[(b + j) * kNP + p];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < 16; j++) acc += v[j];
        }
        for (; b < r1; b++) acc += grad_part[b * kNP + p];
    }
    part[q][lane] = acc;
    if (q == 0) {
        // the counted voxels (integers, exact in any order) and, for the loss,
        // the squared errors: the first wave, a fixed butterfly, lane 0's sums
        float cnt = 0.0f, sq = 0.0f;
        for (int64_t b = lane; b < n; b += 64) {
            cnt += loss_part[2 * b + 1];
            if (blockIdx.x == 0) sq += loss_part[2 * b];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            cnt += __shfl_xor(cnt, o, 64);
            sq += __shfl_xor(sq, o, 64);
        }
        if (lane == 0) {
            s_inv = 1.0f / fmaxf(cnt, 1.0f);
            if (blockIdx.x == 0) loss[0] = sq * s_inv;
        }
    }
    __syncthreads();
    if (q == 0 && p < kNP) {
        const float g = ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane])) * s_inv;
        grad[p] = g;
        if (ADAM) adam_update(ad, k, p, g, w0, m0, v0);
    }
}

// bf16 copies of a master vector (after a parameter upload)
__global__ void k_refine_cast(const float *master, uint16_t *Wf, uint16_t *Wt, float *bias)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNP) return;
    const float w = master[p];
    if (p < kNW) {
        Wf[p] = to_bf16(w);
        const int ci = p % kC, co = (p / kC) % kC, lt = p / (kC * kC);
        Wt[(lt * kC + ci) * kC + co] = to_bf16(w);
    } else {
        bias[p - kNW] = w;
    }
}

// network input of a block from the volume: F and W / max_w on the 10^3 grid
// around it; voxels of absent neighbour blocks read F = 1, W = 0
template <int FMT>
__global__ void k_refine_gather(HashView h, const void *sdf, const void *w, const int32_t *coords, int64_t n,
                                float inv_max_w, float *out)
{
    using V = Vox<FMT>;
    const auto *S = (const typename V::S *)sdf;
    const auto *Wv = (const typename V::Wt *)w;
    for (int64_t b = blockIdx.x; b < n; b += gridDim.x) {
        const int kx = coords[3 * b], ky = coords[3 * b + 1], kz = coords[3 * b + 2];
        for (int u = threadIdx.x; u < 1000; u += blockDim.x) {
            const int vx = 8 * kx - 1 + u % 10, vy = 8 * ky - 1 + (u / 10) % 10, vz = 8 * kz - 1 + u / 100;
            const int32_t p = block_of(h, find_block_direct(h, vx >> 3, vy >> 3, vz >> 3));
            float F = 1.0f, Wf = 0.0f;
            if (p >= 0) {
                const int64_t i = (int64_t)p * kBlockVox + (vx & 7) + 8 * (vy & 7) + 64 * (vz & 7);
                F = V::to_f(S[i]);
                Wf = V::w_to_f(Wv[i]) * inv_max_w;
            }
            out[b * 2000 + u] = F;
            out[b * 2000 + 1000 + u] = Wf;
        }
    }
}

// Per-frame inference gate: every visible block whose largest weight is below
// the threshold is refined; its network input is gathered straight from the
// volume into LDS and the refined F goes to a side buffer (half precision,
// indexed like the voxel block array) stamped with the frame number.
template <int FMT>
__global__ __launch_bounds__(kInferWaves * 64) void k_refine_gated(RefineGateArgs a)
{
    constexpr int TPW = kInferTPW;
    using V = Vox<FMT>;
    __shared__ RefineLdsInf L;
    __shared__ int s_go;
    const auto *S = (const typename V::S *)a.sdf;
    const auto *Wv = (const typename V::Wt *)a.w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, n = lane & 15;
    // the visible list (workgroup-uniform loop)
    const VisPrefix vp = vis_prefix(a.list, lane);
    for (int bi = blockIdx.x; bi < vp.total; bi += gridDim.x) {
        const VisRec rec = vis_item(a.list, vp, bi);
        const unsigned long long key = rec.key;
        const int32_t ptr = block_of(a.h, rec.e);
        int kx, ky, kz;
        unpack_key(key, kx, ky, kz);
        // gate on the block's largest weight
        if (threadIdx.x == 0) s_go = 0;
        __syncthreads();
        if (ptr >= 0)
            for (int i = threadIdx.x; i < kBlockVox; i += blockDim.x)
                if (V::w_to_f(Wv[(int64_t)ptr * kBlockVox + i]) >= a.w_threshold) s_go = 1;  // benign race
        __syncthreads();
        const bool skip = ptr < 0 || s_go != 0;
        __syncthreads();                 // every thread has read s_go before it is reset
        if (skip) continue;              // uniform over the workgroup
        for (int u = threadIdx.x; u < 1000; u += blockDim.x) {
            const int vx = 8 * kx - 1 + u % 10, vy = 8 * ky - 1 + (u / 10) % 10, vz = 8 * kz - 1 + u / 100;
            const int32_t p = block_of(a.h, find_block_direct(a.h, vx >> 3, vy >> 3, vz >> 3));
            float F = 1.0f, Wf = 0.0f;
            if (p >= 0) {
                const int64_t i = (int64_t)p * kBlockVox + (vx & 7) + 8 * (vy & 7) + 64 * (vz & 7);
                F = V::to_f(S[i]);
                Wf = V::w_to_f(Wv[i]) * a.inv_max_w;
            }
            uint16_t *d = &L.x0[u * 4];
            d[0] = to_bf16(F);
            d[1] = to_bf16(Wf);
            d[2] = 0;
            d[3] = 0;
            const int x = u % 10, y = (u / 10) % 10, z = u / 100;
            if (x >= 1 && x <= 8 && y >= 1 && y <= 8 && z >= 1 && z <= 8)
                L.centre[(x - 1) + 8 * (y - 1) + 64 * (z - 1)] = F;
        }
        __syncthreads();
        f32x4 delta[TPW];
        refine_forward<2, TPW>(L, a.P, wave, lane, delta);
        if (n == 0) {
#pragma unroll
            for (int t = 0; t < TPW; t++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int vox = (wave * TPW + t) * 16 + 4 * kq + r;
                    const float Fo = fminf(fmaxf(L.centre[vox] + delta[t][r], -1.0f), 1.0f);
                    a.refined[(int64_t)ptr * kBlockVox + vox] = __float2half_rn(Fo);
                }
        }
        if (threadIdx.x == 0) a.stamp[ptr] = a.frame;
        __syncthreads();
    }
}

hipError_t launch_refine_gated(int fmt, const RefineGateArgs &a, int grid, hipStream_t st)
{
    switch (fmt) {
    case ITM_VOX_F32: launch_k(k_refine_gated<ITM_VOX_F32>, grid, kInferWaves * 64, st, a); break;
    case ITM_VOX_F16: launch_k(k_refine_gated<ITM_VOX_F16>, grid, kInferWaves * 64, st, a); break;
    default: launch_k(k_refine_gated<ITM_VOX_S16U8>, grid, kInferWaves * 64, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_refine(const RefineArgs &a, bool train, int grid, hipStream_t st)
{
    if (train) k_refine<true><<<grid, kTrainWaves * 64, 0, st>>>(a);
    else k_refine_infer<<<grid, kInferWaves * 64, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_refine_reduce(const float *grad_part, const float *loss_part, int64_t n, float *grad,
                                float *loss, const AdamStep *adam, hipStream_t st)
{
    const int grid = (kNP + 63) / 64;
    if (adam) {
        AdamConst k;
        k.lr = adam->lr;
        k.b1 = 0.9f;
        k.b2 = 0.999f;
        k.eps = 1e-8f;
        k.c1 = 1.0f - powf(k.b1, (float)adam->step);
        k.c2 = 1.0f - powf(k.b2, (float)adam->step);
        k_refine_reduce<true><<<grid, 256, 0, st>>>(grad_part, loss_part, n, grad, loss, *adam, k);
    } else {
        k_refine_reduce<false><<<grid, 256, 0, st>>>(grad_part, loss_part, n, grad, loss, AdamStep{}, AdamConst{});
    }
    return hipGetLastError();
}

hipError_t launch_refine_cast(const float *master, uint16_t *Wf, uint16_t *Wt, float *bias, hipStream_t st)
{
    k_refine_cast<<<(kNP + 255) / 256, 256, 0, st>>>(master, Wf, Wt, bias);
    return hipGetLastError();
}

hipError_t launch_refine_gather(int fmt, const HashView &h, const void *sdf, const void *w, const int32_t *coords,
                                int64_t n, float inv_max_w, float *out, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>(n, 4096);
    if (grid <= 0) return hipSuccess;
    switch (fmt) {
    case ITM_VOX_F32: k_refine_gather<ITM_VOX_F32><<<grid, 256, 0, st>>>(h, sdf, w, coords, n, inv_max_w, out); break;
    case ITM_VOX_F16: k_refine_gather<ITM_VOX_F16><<<grid, 256, 0, st>>>(h, sdf, w, coords, n, inv_max_w, out); break;
    default: k_refine_gather<ITM_VOX_S16U8><<<grid, 256, 0, st>>>(h, sdf, w, coords, n, inv_max_w, out); break;
    }
    return hipGetLastError();
}

}  // namespace itm
