// Internal device-side definitions shared by the library's kernels.
//
// HBM layout of a scene (one allocation each):
//   buckets  n_buckets x 16 B   {key[2] (u64)} the ordered part of the hash table,
//                               2 entries per bucket: one 16-byte load probes both
//   head     n_buckets x i32    first excess entry of the bucket's chain (-1 =
//                               none), i.e. the offset the paper keeps in the
//                               bucket's last entry
//   excess   n_excess x 16 B    {key (u64), next (i32), pad}  unordered part
//   stamp    n_entries x u32    frame (+1) in which the entry was last listed visible
//   vis_list (32 cap + n_entries) x 16 B   the frame's visible blocks {key, entry}:
//                               32 stripes of `cap` records, appended to by the
//                               allocation's workgroups (stripe = workgroup % 32),
//                               and an overflow segment for full stripes
//   bins     3 x n_tiles x (4 B + cap x 16 B)   expected-depth rectangles binned
//                               by 16 x 16 pixel tile (two frame parities + one
//                               for raycasts at another pose)
//   sdf, w   n_entries x 512    voxel block array, structure of arrays, one
//                               element type per storage form.  The array has a
//                               block for every hash entry, so the paper's
//                               pointer into it is the entry id itself: a probe
//                               that finds the key has the block, with no second
//                               load and no free-list pop on insertion
//   set      2 x R x u64        per-frame sets of blocks claimed for the excess list
//                               (alternating by frame)
//   cnt      Counters           device counters
// Entry ids follow the paper's layout: 2 b + i for slot i of bucket b, then
// 2 n_buckets + x for excess entry x.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <climits>
#include <stdint.h>

#include "itm.h"

namespace itm {

// Events a profiled launch attaches to its dispatch (hipExtLaunchKernelGGL: they
// take the kernel's own start and end times, not those of markers queued around
// it).  The host sets them for the next launch on its thread; launch_k consumes
// them, and a plain launch is made when none are set.
struct DispatchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
DispatchEvents &dispatch_events();

template <typename... KArgs, typename... Args>
inline void launch_k(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t st, Args... args)
{
    DispatchEvents &ev = dispatch_events();
    if (ev.start) {
        const DispatchEvents e = ev;
        ev = DispatchEvents{};
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e.start, e.stop, 0, args...);
    } else {
        kernel<<<grid, block, 0, st>>>(args...);
    }
}

constexpr int kBlockVox = 512;
constexpr unsigned long long kKeyValid = 1ull << 63;
constexpr int kWave = 64;
constexpr int kStripes = 32;

struct alignas(16) Bucket {
    unsigned long long key[2];   // 0 = empty slot
};
static_assert(sizeof(Bucket) == 16, "bucket record is 16 bytes");

struct alignas(16) Excess {
    unsigned long long key;
    int32_t next;
    int32_t pad;
};
static_assert(sizeof(Excess) == 16, "excess record is 16 bytes");

struct Counters {
    int32_t vba_next;       // voxel blocks allocated (a count: block = entry id)
    int32_t excess_next;    // excess entries handed out (may run past n_excess)
    int32_t pad0;
    int32_t set_used[3];    // claim-set slots used, by frame % 3
    unsigned long long dropped_total;
    unsigned long long pad2[5];
    // counts striped over separate 128-byte lines so that the per-workgroup
    // additions do not all hit one address: [frame parity][stripe] for a frame,
    // [2][stripe] since creation.  A frame's kernel adds to its parity's counters
    // and clears the other parity's: a counter is never both stored to and added
    // to in one kernel (a plain store, written back from one XCD's L2 at the
    // kernel's end, is not ordered with other XCDs' device-scope atomics)
    unsigned long long upd[3][kStripes][16];   // updated voxels
    unsigned long long vis[3][kStripes][16];   // visible blocks
    // records appended to the visible list, [frame parity][segment], one line each
    int32_t lst[2][33][32];
    // [frame parity][0]: the frame listed a block outside its workgroup's set and
    // did not bin that block's rectangle (its bins then give no tile's range)
    int32_t unbinned[2][32];
};

struct HashView {
    Bucket *buckets;
    int32_t *head;
    Excess *excess;
    uint32_t *occ;      // one bit per bucket: set once the bucket holds a block
    uint32_t *macro;    // kMacroBits bits, one per hashed macro cell (4^3 blocks): set
                        // once any block of a cell hashing there is allocated
    uint32_t mask;
    int32_t n_buckets;
    int32_t n_excess;
    int32_t *blk;       // with swapping: per entry, the device voxel block it holds
                        // (-1: none); nullptr: the entry is its own block
};

// the voxel block of entry e (-1 when e is -1 or, with swapping, holds none)
__device__ __forceinline__ int32_t block_of(const HashView &h, int32_t e)
{
    return (h.blk && e >= 0) ? h.blk[e] : e;
}

// Swapping: the device pool of free voxel blocks, a stack popped by the
// allocation (top may run below zero when the pool is empty; the next swap
// kernel clears that) and pushed by the swap-out
struct PoolView {
    int32_t *stack;               // nullptr: no swapping
    int32_t *top;
    unsigned long long *no_block; // visible blocks left without a device block (total)
};

// block key: valid bit | x | y << 16 | z << 32 (16-bit two's complement each)
__device__ __forceinline__ unsigned long long pack_key(int x, int y, int z)
{
    return kKeyValid | (unsigned long long)(uint16_t)x | ((unsigned long long)(uint16_t)y << 16) |
           ((unsigned long long)(uint16_t)z << 32);
}

__device__ __forceinline__ void unpack_key(unsigned long long k, int &x, int &y, int &z)
{
    x = (int16_t)(k & 0xffffu);
    y = (int16_t)((k >> 16) & 0xffffu);
    z = (int16_t)((k >> 32) & 0xffffu);
}

__device__ __forceinline__ bool in_key_range(int x, int y, int z)
{
    return x >= -32768 && x <= 32767 && y >= -32768 && y <= 32767 && z >= -32768 && z <= 32767;
}

// hashIndex of section "Hash Table and Hashing Function": unsigned 32-bit products
// of the coordinates with three primes, xor-ed, masked to the bucket count
__device__ __forceinline__ uint32_t hash_raw(int x, int y, int z)
{
    return ((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349669u) ^ ((uint32_t)z * 83492791u);
}
__device__ __forceinline__ uint32_t hash_index(int x, int y, int z, uint32_t mask)
{
    return hash_raw(x, y, z) & mask;
}

// the bucket's two entries, then (both taken) the excess chain; returns the
// entry id, which is also the block's place in the voxel block array, or -1
__device__ __forceinline__ int32_t probe_bucket(const HashView &h, uint32_t b, unsigned long long key)
{
    const ulonglong2 keys = *reinterpret_cast<const ulonglong2 *>(h.buckets[b].key);
    if (keys.x == key) return 2 * (int32_t)b;
    if (keys.y == key) return 2 * (int32_t)b + 1;
    if (keys.y == 0ull) return -1;   // a free slot: the bucket has no chain
    int32_t x_i = h.head[b];
    while (x_i >= 0) {
        const Excess E = h.excess[x_i];
        if (E.key == key) return 2 * h.n_buckets + x_i;
        x_i = E.next;
    }
    return -1;
}

// Read-only retrieval (section "Hash Table Operations"): the bucket's two
// entries, then the excess chain.  Returns the block (entry id) or -1.
__device__ __forceinline__ int32_t find_block(const HashView &h, int x, int y, int z)
{
    if (!in_key_range(x, y, z)) return -1;
    const uint32_t b = hash_index(x, y, z, h.mask);
    // an empty bucket holds no block (the bitmap is small enough to stay in L2)
    if (!((h.occ[b >> 5] >> (b & 31)) & 1u)) return -1;
    return probe_bucket(h, b, pack_key(x, y, z));
}

// ---------------------------------------------------------------------------
// voxel storage forms
// ---------------------------------------------------------------------------
template <int FMT>
struct Vox;

template <>
struct Vox<ITM_VOX_F32> {
    using S = float;
    using Wt = float;
    static constexpr int bytes = 8;
    __device__ static float to_f(float s) { return s; }
    __device__ static float from_f(float f) { return f; }
    __device__ static float w_to_f(float w) { return w; }
    __device__ static float w_from_f(float w) { return w; }
};

template <>
struct Vox<ITM_VOX_F16> {
    using S = __half;
    using Wt = __half;
    static constexpr int bytes = 4;
    __device__ static float to_f(__half s) { return __half2float(s); }
    __device__ static __half from_f(float f) { return __float2half_rn(f); }
    __device__ static float w_to_f(__half w) { return __half2float(w); }
    __device__ static __half w_from_f(float w) { return __float2half_rn(w); }
};

template <>
struct Vox<ITM_VOX_S16U8> {
    using S = int16_t;
    using Wt = uint8_t;
    static constexpr int bytes = 3;
    __device__ static float to_f(int16_t s) { return (float)s * (1.0f / 32767.0f); }
    __device__ static int16_t from_f(float f)
    {
        float q = rintf(f * 32767.0f);
        q = fminf(fmaxf(q, -32767.0f), 32767.0f);
        return (int16_t)q;
    }
    __device__ static float w_to_f(uint8_t w) { return (float)w; }
    __device__ static uint8_t w_from_f(float w) { return (uint8_t)w; }
};

// ---------------------------------------------------------------------------
// kernel argument blocks
// ---------------------------------------------------------------------------
struct FrameGeom {
    // camera
    int32_t W, H;
    float fx, fy, cx, cy;               // binary32 copies for the projection decision
    double fxd, fyd, cxd, cyd, inv_fx, inv_fy;
    double Rwc[9], twc[3];
    double Rcw[9], tcw[3];
    float g[3][3];                      // g[j][a]: camera-frame step of one voxel along world axis j
    float o_vox[3];                     // camera centre in voxel units, (float)(t_wc / s)
    // scene
    double s, inv_s, inv_bs;            // voxel size, 1 / s, 1 / (8 s)
    float s_f, mu_f, max_w_f;
    double mu;
    float z_near, z_far;
};


// The frame's visible list (section "Allocation", stage three): built by the
// allocation kernel, read by the integration, the refiner gate and the
// expected-depth binning.  Segment s < 32 is stripe s (capacity cap), segment 32
// the overflow (capacity n_entries); a stripe's counter may run past cap, the
// records beyond it having gone to the overflow.
constexpr int kListSegs = 33;
struct alignas(16) VisRec {
    unsigned long long key;
    int32_t e;            // entry id = voxel block
    int32_t pad;
};
struct VisList {
    VisRec *rec;          // segment s at rec + s * cap
    int32_t *cnt;         // segment s's counter at cnt[32 * s]
    int32_t cap;
};

// Expected depth ranges (section "Raycast", search range).  Each visible block's
// box -- the region [8k - 1/2, 8k + 7 1/2] s whose samples read the block -- is
// projected; its 2D bounding box gets the box's camera depth range.  The
// rectangles are binned by 16 x 16 pixel tile; a tile's pixels take the min and
// max over the rectangles covering them.
struct alignas(16) RangeRect {
    int16_t u0, u1, v0, v1;   // inclusive pixel rectangle, clipped to the image
    float z0, z1;             // camera depth range, rounded outwards to binary32
};
static_assert(sizeof(RangeRect) == 16, "range rectangle is 16 bytes");
constexpr int kTile = 16;

struct RangeBins {
    int32_t *cnt;         // [n_tiles] rectangles appended (may exceed cap)
    RangeRect *rect;      // [n_tiles][cap]
    int32_t cap;
    int32_t tw, th;       // tiles per row, per column
    int32_t *unbinned;    // non-null for bins the allocation fills: set when a block went
                          // unbinned, and every tile then takes the exact path
};

// the per-frame kernels: allocation and visible list (and the expected-depth
// binning at the frame's pose), then integration of the listed blocks
struct FuseArgs {
    FrameGeom fg;
    const float *depth;
    HashView h;
    int32_t parity;               // frame parity: per-frame counters and list counters
    uint32_t *stamp;              // per entry: frame (+1) in which it was last listed
    uint32_t stamp_now;           // this frame's value
    // claim set of the excess insertions: this frame's table, slot list and count;
    // the previous frame's table is cleared here (slots listed in its list), and
    // the next frame's count zeroed (tables alternate by frame, lists by frame % 3)
    unsigned long long *set;
    int32_t *set_list;
    int32_t *set_used;
    uint32_t set_mask;
    unsigned long long *set_prev;
    const int32_t *set_list_prev;
    const int32_t *set_used_prev;
    int32_t *set_used_next;
    VisList list;                 // this frame's visible list (appended here)
    int32_t *list_clear;          // the other parity's list counters, cleared here
    RangeBins rb;                 // rb.cnt non-null: bin the visible blocks' rectangles at this pose
    int32_t *rb_clear;            // bin counts of the other parity, cleared here (with rb)
    int32_t n_clear;
    void *sdf;
    void *w;
    uchar4 *clr;                  // colour voxels (r, g, b, colour weight), or nullptr
    const uchar4 *rgbx;           // this frame's registered colour image, or nullptr
    Counters *cnt;
    PoolView pool;                // swapping's device pool (pool.stack nullptr: off)
};

struct RaycastArgs {
    FrameGeom fg;
    HashView h;
    const uchar4 *clr;            // colour voxels, or nullptr
    uchar4 *rgb_out;              // per pixel: colour of the hit's nearest voxel, or nullptr
    const void *sdf;
    float4 *pts;
    float4 *nrm;
    RangeBins rb;             // rb.cnt non-null: search each ray inside its expected range
    VisList list;             // for tiles whose bin overflowed
    const __half *refined;    // non-null: blocks refined in frame rframe read F from here
    const int32_t *rstamp;    // per voxel block: frame of its last refinement
    int32_t rframe;
};

// learned refiner (itm_refine.hip)
constexpr int kRefineWeights = 4 * 27 * 16 * 16;       // [layer][tap][co][ci]
constexpr int kRefineParams = kRefineWeights + 4 * 16;  // + biases [layer][co]

struct RefineParams {
    const uint16_t *Wf;   // bf16 [l][tap][co][ci]   (forward operand)
    const uint16_t *Wt;   // bf16 [l][tap][ci][co]   (data-gradient operand)
    const float *bias;    // float32 [l][co]
};

struct RefineArgs {
    RefineParams P;
    const float *in;        // [n][2][1000]
    int64_t n;
    float *out;             // [n][512] refined F, or null
    const float *target;    // [n][512]  (training)
    const uint8_t *mask;    // [n][512]  (training)
    float *grad_part;       // [n][kRefineParams]  (training)
    float *loss_part;       // [n][2]: sum of squared errors, count (training)
};

struct RefineGateArgs {
    RefineParams P;
    HashView h;
    VisList list;
    const void *sdf;
    const void *w;
    float inv_max_w;
    float w_threshold;
    __half *refined;      // [capacity][512]
    int32_t *stamp;       // [capacity]: frame of the last refinement
    int32_t frame;
};

hipError_t launch_refine(const RefineArgs &a, bool train, int grid, hipStream_t st);
hipError_t launch_refine_gated(int fmt, const RefineGateArgs &a, int grid, hipStream_t st);
// one Adam step (beta 0.9, 0.999, eps 1e-8) on the float32 master weights,
// applied by the gradient reduction where it is given
struct AdamStep {
    float *master, *m, *v;   // [kRefineParams] each
    uint16_t *Wf, *Wt;       // bf16 copies of the weights, forward and transposed
    float *bias;             // float32 copy of the biases
    float lr;
    int step;                // 1 at the first step
};

// grad, loss: where the mean gradient and the loss go; adam: nullptr for the
// gradient alone
hipError_t launch_refine_reduce(const float *grad_part, const float *loss_part, int64_t n, float *grad,
                                float *loss, const AdamStep *adam, hipStream_t st);
hipError_t launch_refine_cast(const float *master, uint16_t *Wf, uint16_t *Wt, float *bias, hipStream_t st);
hipError_t launch_refine_gather(int fmt, const HashView &h, const void *sdf, const void *w, const int32_t *coords,
                                int64_t n, float inv_max_w, float *out, hipStream_t st);

hipError_t launch_range_clear(int32_t *cnt, int n, hipStream_t st);
hipError_t launch_range_bin(const FrameGeom &g, const VisList &list, const RangeBins &rb, hipStream_t st);
hipError_t launch_range_image(const FrameGeom &g, const VisList &list, const RangeBins &rb, float2 *zr,
                              hipStream_t st);

// launchers (one translation unit each)
// swapping (itm_swap.hip)
struct alignas(16) SwapRec {
    unsigned long long key;
    int32_t e;
    int32_t pad;
};
struct SwapScanArgs {
    HashView h;
    const uint32_t *stamp;
    uint32_t stamp_now;       // the last frame's stamp: listed in that frame
    const uint8_t *onhost;
    int64_t n_entries;
    SwapRec *in_list, *out_list;
    int32_t *cnt;             // [2]: in, out (cleared by the host)
    PoolView pool;
};
struct SwapMoveArgs {
    HashView h;
    void *sdf, *w;            // the device voxel blocks
    void *xfer_sdf, *xfer_w;  // device transfer buffer, block i at i * 512 voxels
    const int32_t *entries;   // [n]
    int32_t n;
    uint8_t *onhost;
    float max_w;
    PoolView pool;
};
hipError_t launch_swap_scan(const SwapScanArgs &a, hipStream_t st);
hipError_t launch_swap_move(int fmt, bool out, const SwapMoveArgs &a, hipStream_t st);
hipError_t launch_swap_init(int32_t *stack, int32_t n_blocks, int32_t *top, int32_t *blk, uint8_t *onhost,
                            int64_t n_entries, hipStream_t st);
hipError_t launch_alloc(const FuseArgs &a, hipStream_t st);
hipError_t launch_import_keys(const FuseArgs &a, const int32_t *coords, int32_t n, int32_t *entry, hipStream_t st);
hipError_t launch_import_voxels(int fmt, const int32_t *entry, const float *in_sdf, const float *in_w, int64_t n,
                                void *sdf, void *w, uchar4 *clr, hipStream_t st);
hipError_t launch_integrate(int fmt, const FuseArgs &a, int grid, hipStream_t st);
hipError_t launch_raycast(int fmt, const RaycastArgs &a, hipStream_t st);
hipError_t launch_export_gather(int fmt, const void *sdf, const void *w, const int32_t *blocks, int64_t n,
                                void *out_sdf, void *out_w, hipStream_t st);
hipError_t launch_export_colour(const uchar4 *clr, const int32_t *blocks, int64_t n, uchar4 *out, hipStream_t st);
hipError_t launch_init(Bucket *b, int32_t *head, int64_t nb, Excess *x, int64_t nx, uint32_t *stamp, int64_t nstamp,
                       unsigned long long *set, int64_t nset, uint32_t *occ, int64_t nocc,
                       Counters *cnt, int fmt, void *sdf, void *w, int64_t n_vox, hipStream_t st);

// Workgroups are handed to the 8 XCDs round-robin by id.  Image tiles are
// renumbered so that XCD k gets a contiguous band of tiles: rays and pixels of a
// band touch the same hash buckets and voxel blocks, which then stay in that XCD's
// L2.  Returns false for the padding ids past the last tile.
constexpr int kXcds = 8;
__device__ __forceinline__ bool xcd_tile(int n_tx, int n_ty, int &tx, int &ty)
{
    const int n = n_tx * n_ty;
    const int per = (n + kXcds - 1) / kXcds;
    const int b = blockIdx.x;
    const int tile = (b % kXcds) * per + b / kXcds;
    if (tile >= n) return false;
    tx = tile % n_tx;
    ty = tile / n_tx;
    return true;
}
__host__ __forceinline__ int xcd_grid(int n_tiles) { return (n_tiles + kXcds - 1) / kXcds * kXcds; }

// A small hashed occupancy filter of macro cells, staged in LDS by the raycast:
// no false negatives, so a clear bit proves a whole macro cell absent.
constexpr int kMacroShift = 2;              // macro cell = 4 x 4 x 4 blocks
constexpr int kMacroBits = 1 << 16;         // 8 KiB
constexpr int kMacroWords = kMacroBits / 32;

__device__ __forceinline__ uint32_t macro_index(int bx, int by, int bz)
{
    return hash_index(bx >> kMacroShift, by >> kMacroShift, bz >> kMacroShift, kMacroBits - 1);
}

// retrieval without the bucket bitmap, for blocks that are probably allocated
__device__ __forceinline__ int32_t find_block_direct(const HashView &h, int x, int y, int z)
{
    if (!in_key_range(x, y, z)) return -1;
    return probe_bucket(h, hash_index(x, y, z, h.mask), pack_key(x, y, z));
}

// key of hash entry e (entry ids as in the layout above); the block is e itself
__device__ __forceinline__ unsigned long long entry_key(const HashView &h, int32_t e)
{
    return e < 2 * h.n_buckets ? h.buckets[e >> 1].key[e & 1] : h.excess[e - 2 * h.n_buckets].key;
}

// ---------------------------------------------------------------------------
// expected depth ranges: per-block rectangle (binary64, fixed order: corner
// ((8 k - 1/2) + 8 c) s, camera ((R0 X0 + R1 X1) + R2 X2) + t, pixel
// fx X / Z + cx) and per-pixel min / max over a tile's rectangles
// ---------------------------------------------------------------------------
struct BoxAcc {
    double zlo, zhi, xlo, xhi, ylo, yhi;
    bool behind;
};

__device__ __forceinline__ void box_corner(const FrameGeom &g, int kx, int ky, int kz, int c, BoxAcc &b)
{
    const double X0 = ((double)(8 * kx) - 0.5 + ((c & 1) ? 8.0 : 0.0)) * g.s;
    const double X1 = ((double)(8 * ky) - 0.5 + ((c & 2) ? 8.0 : 0.0)) * g.s;
    const double X2 = ((double)(8 * kz) - 0.5 + ((c & 4) ? 8.0 : 0.0)) * g.s;
    double P[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double w = g.Rcw[3 * a + 0] * X0;
        w = w + g.Rcw[3 * a + 1] * X1;
        w = w + g.Rcw[3 * a + 2] * X2;
        P[a] = w + g.tcw[a];
    }
    b.zlo = P[2];
    b.zhi = P[2];
    b.behind = !(P[2] > 0.0);
    if (b.behind) {
        b.xlo = b.ylo = INFINITY;
        b.xhi = b.yhi = -INFINITY;
    } else {
        b.xlo = b.xhi = g.fxd * P[0] / P[2] + g.cxd;
        b.ylo = b.yhi = g.fyd * P[1] / P[2] + g.cyd;
    }
}

__device__ __forceinline__ void box_merge(BoxAcc &a, const BoxAcc &b)
{
    a.zlo = fmin(a.zlo, b.zlo); a.zhi = fmax(a.zhi, b.zhi);
    a.xlo = fmin(a.xlo, b.xlo); a.xhi = fmax(a.xhi, b.xhi);
    a.ylo = fmin(a.ylo, b.ylo); a.yhi = fmax(a.yhi, b.yhi);
    a.behind = a.behind || b.behind;
}

// false when the rectangle misses the image
__device__ __forceinline__ bool box_rect(const FrameGeom &g, const BoxAcc &b, RangeRect &r)
{
    double zlo = b.zlo;
    if (b.behind) {
        // a corner at or behind the camera plane: the whole image, from depth 0
        r.u0 = 0; r.u1 = (int16_t)(g.W - 1); r.v0 = 0; r.v1 = (int16_t)(g.H - 1);
        zlo = 0.0;
    } else {
        const double a0 = ceil(b.xlo), a1 = floor(b.xhi), b0 = ceil(b.ylo), b1 = floor(b.yhi);
        if (a1 < 0.0 || b1 < 0.0 || a0 > (double)(g.W - 1) || b0 > (double)(g.H - 1) || a0 > a1 || b0 > b1)
            return false;
        r.u0 = (int16_t)(a0 < 0.0 ? 0 : (int)a0);
        r.v0 = (int16_t)(b0 < 0.0 ? 0 : (int)b0);
        r.u1 = (int16_t)(a1 > (double)(g.W - 1) ? g.W - 1 : (int)a1);
        r.v1 = (int16_t)(b1 > (double)(g.H - 1) ? g.H - 1 : (int)b1);
    }
    r.z0 = __double2float_rd(zlo);
    r.z1 = __double2float_ru(b.zhi);
    return true;
}

// one thread, all 8 corners
__device__ __forceinline__ bool block_rect(const FrameGeom &g, int kx, int ky, int kz, RangeRect &r)
{
    BoxAcc acc;
    box_corner(g, kx, ky, kz, 0, acc);
#pragma unroll 1
    for (int c = 1; c < 8; c++) {
        BoxAcc b;
        box_corner(g, kx, ky, kz, c, b);
        box_merge(acc, b);
    }
    return box_rect(g, acc, r);
}

__device__ __forceinline__ void rect_tiles(const RangeRect &r, int &tx0, int &ty0, int &ntx, int &n)
{
    tx0 = r.u0 / kTile;
    ty0 = r.v0 / kTile;
    ntx = r.u1 / kTile - tx0 + 1;
    n = ntx * (r.v1 / kTile - ty0 + 1);
}

// One block's rectangle by a group of 8 consecutive lanes: lane c = lane & 7
// projects box corner c and a butterfly merges the 8 (every lane of the group
// ends with the rectangle).  valid is uniform over the group; false when the
// block is invalid or covers no pixel.
__device__ __forceinline__ bool block_rect8(const FrameGeom &g, bool valid, unsigned long long key, RangeRect &r)
{
    const int corner = threadIdx.x & 7;
    BoxAcc b;
    if (valid) {
        int kx, ky, kz;
        unpack_key(key, kx, ky, kz);
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
    return valid && box_rect(g, b, r);
}

// One block's rectangle appended to the bins of the tiles it overlaps by a group
// of 8 consecutive lanes (block_rect8), then lane c takes every 8th tile, so the
// reservations go out together.
__device__ __forceinline__ void bin_block8(const FrameGeom &g, const RangeBins &rb, bool valid,
                                           unsigned long long key)
{
    const int corner = threadIdx.x & 7;
    RangeRect r;
    if (block_rect8(g, valid, key, r)) {
        int tx0, ty0, ntx, n_tiles;
        rect_tiles(r, tx0, ty0, ntx, n_tiles);
        for (int t = corner; t < n_tiles; t += 8) {
            const int tile = (ty0 + t / ntx) * rb.tw + tx0 + t % ntx;
            const int slot = atomicAdd(&rb.cnt[tile], 1);
            if (slot < rb.cap) rb.rect[(int64_t)tile * rb.cap + slot] = r;
        }
    }
}

// ---------------------------------------------------------------------------
// visible-list access
// ---------------------------------------------------------------------------
__device__ __forceinline__ int vis_count(const VisList &v, int s)
{
    const int c = v.cnt[32 * s];
    return s < 32 ? min(c, v.cap) : c;
}

// Per-wave view of the list: lane s < 33 holds the inclusive prefix of the
// segment counts, every lane the total.
struct VisPrefix {
    int incl, total;
};
__device__ __forceinline__ VisPrefix vis_prefix(const VisList &v, int lane)
{
    int incl = lane < kListSegs ? vis_count(v, lane) : 0;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    return VisPrefix{incl, __shfl(incl, kWave - 1, kWave)};
}

// record of item g < total, g the same on every lane of the wave
__device__ __forceinline__ const VisRec &vis_item(const VisList &v, const VisPrefix &p, int g)
{
    const int s = __popcll(__ballot(p.incl <= g));   // segments wholly before g
    const int excl = s ? __shfl(p.incl, s - 1, kWave) : 0;
    return v.rec[(int64_t)s * v.cap + (g - excl)];
}

// record of item g < total, any g per thread: pre[s] = exclusive prefix of
// segment s (pre[33] = total), e.g. staged in LDS
__device__ __forceinline__ const VisRec &vis_item_at(const VisList &v, const int *pre, int g)
{
    int s = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (s + step < kListSegs && pre[s + step] <= g) s += step;
    return v.rec[(int64_t)s * v.cap + (g - pre[s])];
}

// LDS of the per-tile range computation
struct RangeLds {
    union {
        RangeRect rect[256];
        struct {
            uint32_t zlo[256], zhi[256];   // binary32 bits (all values >= 0: integer order = float order)
        } px;
    };
    int pre[kListSegs + 1];
};

// A tile's bin count and, speculatively, its first 256 rectangles (those lie
// inside the tile's storage whatever the count): issued together, one memory
// round; a caller can issue them before other work it has to wait for.
struct TileBin {
    int n;
    RangeRect first;
};
__device__ __forceinline__ TileBin tile_bin(const RangeBins &rb, int tx, int ty)
{
    const int tile = ty * rb.tw + tx;
    TileBin b;
    if ((int)threadIdx.x < rb.cap) b.first = rb.rect[(int64_t)tile * rb.cap + threadIdx.x];
    b.n = rb.cnt[tile];
    if (rb.unbinned && *rb.unbinned) b.n = rb.cap + 1;   // incomplete bins: the exact path
    return b;
}

// Range of pixel (u, v) of tile (tx, ty) -- whole workgroup of 256 threads, one
// pixel each (any mapping; (u, v) may lie outside the image), bin as loaded by
// tile_bin.  Returns the empty range (+inf, 0) where no rectangle covers the
// pixel.  A tile whose bin overflowed recomputes every visible block's
// rectangle from the visible list.
__device__ __forceinline__ void tile_range(const FrameGeom &g, const VisList &list, const RangeBins &rb, int tx, int ty,
                                  const TileBin &bin, int u, int v, RangeLds &L, float &zlo, float &zhi)
{
    const int tile = ty * rb.tw + tx;
    const int n = __builtin_amdgcn_readfirstlane(bin.n);   // the same for every thread
    zlo = INFINITY;
    zhi = 0.0f;
    if (n <= rb.cap) {
        for (int base = 0; base < n; base += 256) {
            __syncthreads();
            if (base + (int)threadIdx.x < n) {
                // by value (a select between the two places would put bin in
                // scratch memory)
                RangeRect r = bin.first;
                if (base != 0) r = rb.rect[(int64_t)tile * rb.cap + base + threadIdx.x];
                L.rect[threadIdx.x] = r;
            }
            __syncthreads();
            const int m = min(256, n - base);
            // broadcast LDS reads of whole rectangles, four in flight at a time,
            // tested without branches (depths are never NaN)
            const uint4 *R = reinterpret_cast<const uint4 *>(L.rect);
            int j = 0;
            for (; j < m; j += 4) {
                uint4 q[4];
#pragma unroll
                for (int k = 0; k < 4; k++) q[k] = R[min(j + k, m - 1)];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const bool in = (u >= (int)(int16_t)q[k].x) & (u <= ((int)q[k].x >> 16)) &
                                    (v >= (int)(int16_t)q[k].y) & (v <= ((int)q[k].y >> 16));
                    const float z0 = __uint_as_float(q[k].z), z1 = __uint_as_float(q[k].w);
                    zlo = (in & (z0 < zlo)) ? z0 : zlo;
                    zhi = (in & (z1 > zhi)) ? z1 : zhi;
                }
            }
        }
        return;
    }
    // overflow: every visible block, rectangles clipped to the tile, min / max
    // by LDS atomics (threads stride over the list)
    __syncthreads();
    L.px.zlo[threadIdx.x] = __float_as_uint(INFINITY);
    L.px.zhi[threadIdx.x] = 0u;
    if (threadIdx.x < kWave) {
        const VisPrefix p = vis_prefix(list, threadIdx.x);
        if (threadIdx.x < kListSegs) L.pre[threadIdx.x + 1] = p.incl;
        if (threadIdx.x == 0) L.pre[0] = 0;
    }
    __syncthreads();
    const int ux0 = tx * kTile, vy0 = ty * kTile;
    const int total = L.pre[kListSegs];
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        {
            int kx, ky, kz;
            unpack_key(vis_item_at(list, L.pre, i).key, kx, ky, kz);
            RangeRect r;
            if (!block_rect(g, kx, ky, kz, r)) continue;
            const int a0 = max((int)r.u0, ux0), a1 = min((int)r.u1, ux0 + kTile - 1);
            const int b0 = max((int)r.v0, vy0), b1 = min((int)r.v1, vy0 + kTile - 1);
            for (int y = b0; y <= b1; y++)
                for (int x = a0; x <= a1; x++) {
                    const int p = (y - vy0) * kTile + (x - ux0);
                    atomicMin(&L.px.zlo[p], __float_as_uint(r.z0));
                    atomicMax(&L.px.zhi[p], __float_as_uint(r.z1));
                }
        }
    }
    __syncthreads();
    if (u >= ux0 && u < ux0 + kTile && v >= vy0 && v < vy0 + kTile) {
        zlo = __uint_as_float(L.px.zlo[(v - vy0) * kTile + (u - ux0)]);
        zhi = __uint_as_float(L.px.zhi[(v - vy0) * kTile + (u - ux0)]);
    }
    __syncthreads();
}

}  // namespace itm
