// Host side of the C ABI declared in include/itm.h: scene lifetime, per-frame
// launch sequence, export, statistics and per-kernel event timing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <mutex>
#include <new>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "itm_track.hpp"

using namespace itm;

namespace {

thread_local std::string g_err;
thread_local itm_status g_status = ITM_OK;

itm_status fail(itm_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
itm_status fail(itm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    g_status = s;
    return s;
}

#define HIP_TRY(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ITM_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
    } while (0)

int64_t next_pow2(int64_t x)
{
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

constexpr int kProfSlots = 4096;

}  // namespace

struct itm_refiner {
    hipStream_t stream = nullptr;
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr, *bias = nullptr;
    uint16_t *Wf = nullptr, *Wt = nullptr;
    float *grad_part = nullptr, *loss_part = nullptr;
    int64_t part_cap = 0;
    int step = 0;
    int num_cu = 0;
};

struct itm_scene {
    float s, mu;
    int32_t max_w;
    int64_t n_buckets, n_excess, n_entries, vba_cap, set_size;
    uint32_t mask;
    int fmt;
    float z_near, z_far;
    hipStream_t stream;
    int device, num_cu;

    Bucket *buckets = nullptr;
    int32_t *head = nullptr;
    Excess *excess = nullptr;
    uint32_t *vis_stamp = nullptr;    // [n_entries] frame (+1) of the last listing
    VisRec *vis_rec = nullptr;        // [32 list_cap + n_entries] visible list records
    int32_t list_cap = 0;             // records per list stripe
    void *sdf = nullptr;
    void *w = nullptr;
    unsigned long long *set = nullptr;
    int32_t *set_list = nullptr;
    Counters *cnt = nullptr;
    uint32_t *occ = nullptr;
    int64_t occ_words = 0;

    itm_refiner *refiner = nullptr;   // not owned
    float refine_w_threshold = 0.0f;
    __half *refined = nullptr;        // [vba_cap][512], allocated on attach
    int32_t *stamp = nullptr;         // [vba_cap]
    int32_t frame = 0;

    // expected depth ranges: bins for parity 0, parity 1 (filled by the
    // integration at its pose) and 2 (filled for a raycast at another pose)
    bool range_on = false;
    int32_t range_cap = 512;
    int32_t *bin_cnt = nullptr;       // [3][bin_tiles]
    RangeRect *bin_rect = nullptr;    // [3][bin_tiles][range_cap]
    int64_t bin_tiles = 0;
    int32_t fused_frame = -1;         // frame whose own-pose bins are valid, -1 none
    itm_intrinsics fused_K = {};
    double fused_T[16] = {};

    // depth tracker scratch, allocated on first use
    float *trk_part = nullptr;        // [trk_part_cap][kIcpSums] per-workgroup sums
    int32_t trk_part_cap = 0;
    double *trk_pose = nullptr;       // [16] current estimate, [32] the last system, then the flags
                                      // (TrackBufs::flags), read back by one copy

    uchar4 *clr = nullptr;            // [vba_cap][512] colour voxels, allocated on enable

    // swapping (section "Swapping"), set up by itm_scene_enable_swapping: the
    // device pool is the voxel block array (vba_cap blocks), entries hold blocks
    bool swap = false;
    int32_t *blk = nullptr;           // [n_entries] device block held, -1 none
    uint8_t *onhost = nullptr;        // [n_entries] a host copy exists (not merged yet when blk >= 0)
    int32_t *pool_stack = nullptr;    // [vba_cap] free device blocks
    int32_t *pool_top = nullptr;      // [2]: stack top, then the scan counts' home (unused)
    unsigned long long *pool_noblock = nullptr;
    SwapRec *swap_in_list = nullptr, *swap_out_list = nullptr;   // [n_entries] each
    int32_t *swap_cnt = nullptr;      // [2]
    int32_t swap_in_cap = 0, swap_out_cap = 0;
    void *xfer_sdf = nullptr, *xfer_w = nullptr;   // device transfer buffer, max(in, out) blocks
    int32_t *xfer_entries = nullptr;
    uint8_t *xfer_host = nullptr;     // pinned host transfer buffer: in blocks, then out blocks
    std::vector<int32_t> host_slot;   // [n_entries] slot of the entry's host copy, -1 none
    std::vector<uint8_t> host_data;   // host voxel blocks (storage form), one slot each
    std::vector<int32_t> host_free;   // free slots
    int64_t swapped_in_last = 0, swapped_out_last = 0, swapped_in_total = 0, swapped_out_total = 0;

    bool prof = false;
    std::vector<hipEvent_t> ev;     // 2 per slot
    std::vector<int> ev_kernel;
    int ev_used = 0;
    double prof_ms[ITM_KERNEL_COUNT] = {};
    int64_t prof_n[ITM_KERNEL_COUNT] = {};
};

namespace {

size_t sdf_elem(int fmt) { return fmt == ITM_VOX_F32 ? 4 : 2; }
size_t w_elem(int fmt) { return fmt == ITM_VOX_F32 ? 4 : fmt == ITM_VOX_F16 ? 2 : 1; }

// one stored voxel value as a float (F, then W)
float decode_sdf(int fmt, const uint8_t *p)
{
    if (fmt == ITM_VOX_F32) {
        float f;
        std::memcpy(&f, p, 4);
        return f;
    }
    if (fmt == ITM_VOX_F16) {
        __half hv;
        std::memcpy(&hv, p, 2);
        return __half2float(hv);
    }
    int16_t q;
    std::memcpy(&q, p, 2);
    return (float)q / 32767.0f;
}

float decode_w(int fmt, const uint8_t *p)
{
    if (fmt == ITM_VOX_F32) {
        float f;
        std::memcpy(&f, p, 4);
        return f;
    }
    if (fmt == ITM_VOX_F16) {
        __half hv;
        std::memcpy(&hv, p, 2);
        return __half2float(hv);
    }
    return (float)*p;
}

void release(itm_scene *sc)
{
    if (!sc) return;
    (void)hipStreamSynchronize(sc->stream);
    for (hipEvent_t e : sc->ev) (void)hipEventDestroy(e);
    (void)hipFree(sc->buckets);
    (void)hipFree(sc->head);
    (void)hipFree(sc->excess);
    (void)hipFree(sc->vis_stamp);
    (void)hipFree(sc->vis_rec);
    (void)hipFree(sc->bin_cnt);
    (void)hipFree(sc->bin_rect);
    (void)hipFree(sc->sdf);
    (void)hipFree(sc->w);
    (void)hipFree(sc->set);
    (void)hipFree(sc->set_list);
    (void)hipFree(sc->cnt);
    (void)hipFree(sc->occ);
    (void)hipFree(sc->refined);
    (void)hipFree(sc->stamp);
    (void)hipFree(sc->trk_part);
    (void)hipFree(sc->trk_pose);
    (void)hipFree(sc->clr);
    for (void *p : {(void *)sc->blk, (void *)sc->onhost, (void *)sc->pool_stack, (void *)sc->pool_top,
                    (void *)sc->pool_noblock, (void *)sc->swap_in_list, (void *)sc->swap_out_list,
                    (void *)sc->swap_cnt, sc->xfer_sdf, sc->xfer_w, (void *)sc->xfer_entries})
        (void)hipFree(p);
    if (sc->xfer_host) (void)hipHostFree(sc->xfer_host);
    delete sc;
}

itm_status dev_alloc(void **p, size_t bytes, const char *what)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? ITM_ERR_OOM : ITM_ERR_HIP, "hipMalloc(%s, %zu bytes): %s",
                    what, bytes, hipGetErrorString(e));
    }
    return ITM_OK;
}

// camera + scene geometry for one call; binary64 values formed on the host in the
// same fixed order the decisions are specified in
itm_status make_geom(const itm_scene *sc, const itm_intrinsics *K, const double *T, FrameGeom *g)
{
    if (!K || !T) return fail(ITM_ERR_ARG, "NULL intrinsics or pose");
    if (K->width < 3 || K->height < 3 || K->width > 32768 || K->height > 32768)
        return fail(ITM_ERR_ARG, "image size %dx%d out of range", K->width, K->height);
    if (!(K->fx > 0) || !(K->fy > 0) || !std::isfinite(K->cx) || !std::isfinite(K->cy))
        return fail(ITM_ERR_ARG, "invalid intrinsics");
    for (int i = 0; i < 16; i++)
        if (!std::isfinite(T[i])) return fail(ITM_ERR_ARG, "non-finite pose");
    std::memset(g, 0, sizeof *g);
    g->W = K->width;
    g->H = K->height;
    g->fxd = K->fx; g->fyd = K->fy; g->cxd = K->cx; g->cyd = K->cy;
    g->fx = (float)K->fx; g->fy = (float)K->fy; g->cx = (float)K->cx; g->cy = (float)K->cy;
    g->inv_fx = 1.0 / K->fx;
    g->inv_fy = 1.0 / K->fy;
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) g->Rwc[3 * i + j] = T[4 * i + j];
        g->twc[i] = T[4 * i + 3];
    }
    // rigid inverse: R_cw = R_wc^T, t_cw = -R_wc^T t_wc
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) g->Rcw[3 * i + j] = g->Rwc[3 * j + i];
        double acc = g->Rwc[0 * 3 + i] * g->twc[0];
        acc = acc + g->Rwc[1 * 3 + i] * g->twc[1];
        acc = acc + g->Rwc[2 * 3 + i] * g->twc[2];
        g->tcw[i] = -acc;
    }
    g->s = (double)sc->s;
    g->inv_s = 1.0 / g->s;
    g->inv_bs = 1.0 / (8.0 * g->s);
    for (int c = 0; c < 3; c++) g->o_vox[c] = (float)(g->twc[c] / g->s);
    for (int j = 0; j < 3; j++)
        for (int a = 0; a < 3; a++) g->g[j][a] = (float)(g->Rcw[3 * a + j] * g->s);
    g->s_f = sc->s;
    g->mu_f = sc->mu;
    g->mu = (double)sc->mu;
    g->max_w_f = (float)sc->max_w;
    g->z_near = sc->z_near;
    g->z_far = sc->z_far;
    return ITM_OK;
}

// the visible list of the frame with this parity (its counters live on the device)
VisList vis_list(const itm_scene *sc, int parity)
{
    VisList v;
    v.rec = sc->vis_rec;
    v.cnt = &sc->cnt->lst[parity][0][0];
    v.cap = sc->list_cap;
    return v;
}

// parity of the last integrated frame (1 before any: its counters are zero)
int last_parity(const itm_scene *sc) { return (sc->frame - 1) & 1; }

// bins for images of W x H pixels (grown on demand; growing clears them)
itm_status ensure_bins(itm_scene *sc, int W, int H)
{
    const int64_t tiles = (int64_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    if (sc->bin_cnt && tiles <= sc->bin_tiles) return ITM_OK;
    HIP_TRY(hipStreamSynchronize(sc->stream));
    (void)hipFree(sc->bin_cnt);
    (void)hipFree(sc->bin_rect);
    sc->bin_cnt = nullptr;
    sc->bin_rect = nullptr;
    sc->bin_tiles = 0;
    sc->fused_frame = -1;
    if (itm_status st = dev_alloc((void **)&sc->bin_cnt, sizeof(int32_t) * 3 * tiles, "range bin counts")) return st;
    if (itm_status st = dev_alloc((void **)&sc->bin_rect, sizeof(RangeRect) * 3 * tiles * sc->range_cap,
                                  "range bins"))
        return st;
    sc->bin_tiles = tiles;
    HIP_TRY(launch_range_clear(sc->bin_cnt, (int)(3 * tiles), sc->stream));
    return ITM_OK;
}

RangeBins bin_set(const itm_scene *sc, int set, int W, int H)
{
    RangeBins rb;
    rb.cnt = sc->bin_cnt + (int64_t)set * sc->bin_tiles;
    rb.rect = sc->bin_rect + (int64_t)set * sc->bin_tiles * sc->range_cap;
    rb.cap = sc->range_cap;
    rb.tw = (W + kTile - 1) / kTile;
    rb.th = (H + kTile - 1) / kTile;
    rb.unbinned = set < 2 ? &sc->cnt->unbinned[set][0] : nullptr;   // set 2 is re-binned whole
    return rb;
}

HashView hash_view(const itm_scene *sc);

HashView hash_view(const itm_scene *sc)
{
    HashView h;
    h.buckets = sc->buckets;
    h.head = sc->head;
    h.excess = sc->excess;
    h.occ = sc->occ;
    h.macro = sc->occ + sc->occ_words;
    h.mask = sc->mask;
    h.n_buckets = (int32_t)sc->n_buckets;
    h.n_excess = (int32_t)sc->n_excess;
    h.blk = sc->swap ? sc->blk : nullptr;
    return h;
}

itm_status prof_flush(itm_scene *sc)
{
    if (sc->ev_used == 0) return ITM_OK;
    HIP_TRY(hipStreamSynchronize(sc->stream));
    for (int i = 0; i < sc->ev_used; i++) {
        if (sc->ev_kernel[i] < 0) continue;   // its launch never took the events
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, sc->ev[2 * i], sc->ev[2 * i + 1]));
        sc->prof_ms[sc->ev_kernel[i]] += ms;
        sc->prof_n[sc->ev_kernel[i]] += 1;
    }
    sc->ev_used = 0;
    return ITM_OK;
}

}  // namespace

itm::DispatchEvents &itm::dispatch_events()
{
    static thread_local DispatchEvents ev;
    return ev;
}

namespace {

// when profiling is on, the next launch (the one this scope wraps) carries a pair
// of events on its dispatch; a scope whose launch did not take them (an error
// before it) leaves its slot out
struct ProfScope {
    itm_scene *sc;
    int slot = -1;
    ProfScope(itm_scene *s, int kernel) : sc(s)
    {
        if (!sc->prof) return;
        if (sc->ev_used == kProfSlots && prof_flush(sc) != ITM_OK) return;
        slot = sc->ev_used++;
        sc->ev_kernel[slot] = kernel;
        dispatch_events() = DispatchEvents{sc->ev[2 * slot], sc->ev[2 * slot + 1]};
    }
    ~ProfScope()
    {
        if (slot >= 0 && dispatch_events().start) {
            dispatch_events() = DispatchEvents{};
            sc->ev_kernel[slot] = -1;
        }
    }
};

// the bins holding the last frame's visible blocks at pose (K, T): the frame's
// own bins when it was integrated at exactly this pose and image size, else
// set 2, filled now
itm_status bins_for_pose(itm_scene *sc, const itm_intrinsics *K, const double *T, const FrameGeom &g,
                         RangeBins *rb)
{
    if (itm_status st = ensure_bins(sc, g.W, g.H)) return st;
    const bool same = sc->fused_frame >= 0 && sc->fused_frame == sc->frame - 1 &&
                      std::memcmp(&sc->fused_K, K, sizeof *K) == 0 &&
                      std::memcmp(sc->fused_T, T, sizeof sc->fused_T) == 0;
    if (same) {
        *rb = bin_set(sc, sc->fused_frame & 1, g.W, g.H);
        return ITM_OK;
    }
    *rb = bin_set(sc, 2, g.W, g.H);
    HIP_TRY(launch_range_clear(rb->cnt, rb->tw * rb->th, sc->stream));
    HIP_TRY(launch_range_bin(g, vis_list(sc, last_parity(sc)), *rb, sc->stream));
    return ITM_OK;
}


}  // namespace

extern "C" {

const char *itm_last_error(void) { return g_err.c_str(); }

itm_status itm_last_status(void) { return g_status; }

itm_scene *itm_scene_create_ex(float voxel_size, float mu, int32_t max_w, int64_t n_buckets,
                               int64_t n_excess, int32_t fmt, void *hip_stream, float z_near,
                               float z_far)
{
    if (!(voxel_size > 0) || !std::isfinite(voxel_size) || !(mu > 0) || !std::isfinite(mu)) {
        fail(ITM_ERR_ARG, "voxel_size and mu must be finite and > 0");
        return nullptr;
    }
    if (fmt != ITM_VOX_F32 && fmt != ITM_VOX_F16 && fmt != ITM_VOX_S16U8) {
        fail(ITM_ERR_ARG, "unknown voxel format %d", fmt);
        return nullptr;
    }
    const int32_t wmax = fmt == ITM_VOX_S16U8 ? 255 : fmt == ITM_VOX_F16 ? 2048 : (1 << 24);
    if (max_w < 1 || max_w > wmax) {
        fail(ITM_ERR_ARG, "max_w %d out of range [1, %d] for this voxel format", max_w, wmax);
        return nullptr;
    }
    if (n_buckets < 1 || (n_buckets & (n_buckets - 1)) != 0 || n_buckets > (int64_t(1) << 28)) {
        fail(ITM_ERR_ARG, "n_buckets must be a power of two in [1, 2^28]");
        return nullptr;
    }
    if (n_excess < 0 || n_excess > (int64_t(1) << 28)) {
        fail(ITM_ERR_ARG, "n_excess must be in [0, 2^28]");
        return nullptr;
    }
    if (!(z_near > 0) || !(z_far > z_near) || !std::isfinite(z_far)) {
        fail(ITM_ERR_ARG, "raycast range must satisfy 0 < z_near < z_far < inf");
        return nullptr;
    }
    itm_scene *sc = new (std::nothrow) itm_scene();
    if (!sc) {
        fail(ITM_ERR_OOM, "host allocation failed");
        return nullptr;
    }
    sc->s = voxel_size;
    sc->mu = mu;
    sc->max_w = max_w;
    sc->n_buckets = n_buckets;
    sc->n_excess = n_excess;
    sc->n_entries = 2 * n_buckets + n_excess;
    sc->vba_cap = sc->n_entries;
    sc->mask = (uint32_t)(n_buckets - 1);
    sc->fmt = fmt;
    sc->z_near = z_near;
    sc->z_far = z_far;
    sc->stream = (hipStream_t)hip_stream;
    // claim set: holds every distinct block claimed for the excess list in one
    // frame at load <= 1/2 (a VGA frame crosses ~1e4 distinct blocks)
    sc->set_size = std::min<int64_t>(next_pow2(std::max<int64_t>(2 * n_excess, 1 << 16)), 1 << 24);
    if (hipGetDevice(&sc->device) != hipSuccess) {
        fail(ITM_ERR_HIP, "no HIP device");
        release(sc);
        return nullptr;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, sc->device) != hipSuccess) {
        fail(ITM_ERR_HIP, "hipGetDeviceProperties failed");
        release(sc);
        return nullptr;
    }
    sc->num_cu = prop.multiProcessorCount;
    const int64_t n_vox = sc->vba_cap * kBlockVox;
    // visible list: 32 stripes sized for an even share plus slack, and an
    // overflow segment that can hold every entry
    sc->list_cap = (int32_t)((sc->n_entries + 31) / 32 + 4096);
    if (dev_alloc((void **)&sc->buckets, sizeof(Bucket) * n_buckets, "buckets") ||
        dev_alloc((void **)&sc->head, sizeof(int32_t) * n_buckets, "bucket chain heads") ||
        dev_alloc((void **)&sc->excess, sizeof(Excess) * std::max<int64_t>(n_excess, 1), "excess") ||
        dev_alloc((void **)&sc->vis_stamp, sizeof(uint32_t) * sc->n_entries, "visibility stamps") ||
        dev_alloc((void **)&sc->vis_rec, sizeof(VisRec) * (32 * (size_t)sc->list_cap + sc->n_entries),
                  "visible list") ||
        dev_alloc(&sc->sdf, sdf_elem(fmt) * n_vox, "sdf") ||
        dev_alloc(&sc->w, w_elem(fmt) * n_vox, "weights") ||
        dev_alloc((void **)&sc->set, sizeof(unsigned long long) * 2 * sc->set_size, "claim sets") ||
        dev_alloc((void **)&sc->set_list, sizeof(int32_t) * 3 * sc->set_size, "claim lists") ||
        dev_alloc((void **)&sc->cnt, sizeof(Counters), "counters") ||
        dev_alloc((void **)&sc->occ,
                  sizeof(uint32_t) * ((n_buckets + 31) / 32 + kMacroWords),
                  "occupancy bitmaps")) {
        release(sc);
        return nullptr;
    }
    sc->occ_words = (n_buckets + 31) / 32;
    hipError_t e = launch_init(sc->buckets, sc->head, n_buckets, sc->excess, n_excess, sc->vis_stamp, sc->n_entries,
                               sc->set, 2 * sc->set_size, sc->occ, sc->occ_words + kMacroWords,
                               sc->cnt, fmt, sc->sdf, sc->w, n_vox, sc->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
    if (e != hipSuccess) {
        fail(ITM_ERR_HIP, "scene initialisation failed: %s", hipGetErrorString(e));
        release(sc);
        return nullptr;
    }
    return sc;
}

itm_scene *itm_scene_create(float voxel_size, float mu, int32_t max_w, int64_t n_buckets,
                            int64_t n_excess)
{
    return itm_scene_create_ex(voxel_size, mu, max_w, n_buckets, n_excess, ITM_VOX_F32, nullptr, 0.2f,
                               5.0f);
}

void itm_scene_destroy(itm_scene *sc) { release(sc); }

itm_status itm_set_stream(itm_scene *sc, void *hip_stream)
{
    if (!sc) return fail(ITM_ERR_ARG, "NULL scene");
    sc->stream = (hipStream_t)hip_stream;
    return ITM_OK;
}

}  // extern "C"

namespace {

PoolView pool_view(const itm_scene *sc)
{
    PoolView p;
    p.stack = sc->swap ? sc->pool_stack : nullptr;
    p.top = sc->pool_top;
    p.no_block = sc->pool_noblock;
    return p;
}

// the arguments of the kernels of the next frame (claim sets, visible list,
// counters by frame parity); with bin, its expected-depth rectangles are binned
// at the frame's pose (g)
FuseArgs frame_args(itm_scene *sc, const FrameGeom &g, bool bin)
{
    const HashView h = hash_view(sc);
    const int32_t parity = sc->frame & 1;
    FuseArgs a;
    a.fg = g;
    a.depth = nullptr;
    a.h = h;
    a.parity = parity;
    a.stamp = sc->vis_stamp;
    a.stamp_now = (uint32_t)sc->frame + 1u;
    // claim sets: tables alternate by frame, slot lists and counts by frame % 3
    const int f3 = sc->frame % 3, p3 = (sc->frame + 2) % 3, n3 = (sc->frame + 1) % 3;
    a.set = sc->set + (size_t)parity * sc->set_size;
    a.set_list = sc->set_list + (size_t)f3 * sc->set_size;
    a.set_used = &sc->cnt->set_used[f3];
    a.set_mask = (uint32_t)(sc->set_size - 1);
    a.set_prev = sc->set + (size_t)(parity ^ 1) * sc->set_size;
    a.set_list_prev = sc->set_list + (size_t)p3 * sc->set_size;
    a.set_used_prev = &sc->cnt->set_used[p3];
    a.set_used_next = &sc->cnt->set_used[n3];
    a.list = vis_list(sc, parity);
    a.list_clear = vis_list(sc, parity ^ 1).cnt;
    a.rb = RangeBins{};
    a.rb_clear = nullptr;
    a.n_clear = 0;
    if (bin) a.rb = bin_set(sc, parity, g.W, g.H);
    if (sc->bin_cnt) {   // the other parity's bins, for the next frame
        a.rb_clear = bin_set(sc, parity ^ 1, g.W, g.H).cnt;
        a.n_clear = (int32_t)sc->bin_tiles;
    }
    a.sdf = sc->sdf;
    a.w = sc->w;
    a.clr = nullptr;
    a.rgbx = nullptr;
    a.cnt = sc->cnt;
    a.pool = pool_view(sc);
    return a;
}

// the learned refiner over the last frame's visible blocks whose largest weight
// is below the threshold; the refined F goes to the side buffer, stamped with
// the current frame number (which the raycast compares against)
itm_status refine_visible(itm_scene *sc)
{
    RefineGateArgs ra;
    ra.P.Wf = sc->refiner->Wf;
    ra.P.Wt = sc->refiner->Wt;
    ra.P.bias = sc->refiner->bias;
    ra.h = hash_view(sc);
    ra.list = vis_list(sc, last_parity(sc));
    ra.sdf = sc->sdf;
    ra.w = sc->w;
    ra.inv_max_w = 1.0f / (float)sc->max_w;
    ra.w_threshold = sc->refine_w_threshold;
    ra.refined = sc->refined;
    ra.stamp = sc->stamp;
    ra.frame = sc->frame;
    ProfScope ps(sc, 3);
    HIP_TRY(launch_refine_gated(sc->fmt, ra, sc->num_cu * 3, sc->stream));
    return ITM_OK;
}

// the key of a swap record as (x, y, z), for the host's key order
void swap_key(const SwapRec &r, int &x, int &y, int &z)
{
    x = (int16_t)(r.key & 0xffffu);
    y = (int16_t)((r.key >> 16) & 0xffffu);
    z = (int16_t)((r.key >> 32) & 0xffffu);
}

bool swap_key_less(const SwapRec &a, const SwapRec &b)
{
    int ax, ay, az, bx, by, bz;
    swap_key(a, ax, ay, az);
    swap_key(b, bx, by, bz);
    if (ax != bx) return ax < bx;
    if (ay != by) return ay < by;
    return az < bz;
}

// After a frame's integration (section "Swapping"): the candidates are found
// on the device; the host takes, in key order, up to swap_in_cap host copies to
// merge into their device blocks and up to swap_out_cap device blocks that were
// not visible in the frame (and have nothing to merge) to move to the host.
// Two host synchronisations per frame.
itm_status swap_frame(itm_scene *sc)
{
    const size_t es = sdf_elem(sc->fmt), ew = w_elem(sc->fmt);
    const size_t blk_bytes = (es + ew) * kBlockVox;
    HIP_TRY(hipMemsetAsync(sc->swap_cnt, 0, sizeof(int32_t) * 2, sc->stream));
    SwapScanArgs sa;
    sa.h = hash_view(sc);
    sa.stamp = sc->vis_stamp;
    sa.stamp_now = (uint32_t)sc->frame;   // the stamp of the frame just integrated
    sa.onhost = sc->onhost;
    sa.n_entries = sc->n_entries;
    sa.in_list = sc->swap_in_list;
    sa.out_list = sc->swap_out_list;
    sa.cnt = sc->swap_cnt;
    sa.pool = pool_view(sc);
    HIP_TRY(launch_swap_scan(sa, sc->stream));
    int32_t cnt[2];
    HIP_TRY(hipMemcpyAsync(cnt, sc->swap_cnt, sizeof cnt, hipMemcpyDeviceToHost, sc->stream));
    HIP_TRY(hipStreamSynchronize(sc->stream));
    std::vector<SwapRec> in(cnt[0]), out(cnt[1]);
    if (cnt[0]) HIP_TRY(hipMemcpyAsync(in.data(), sc->swap_in_list, sizeof(SwapRec) * cnt[0], hipMemcpyDeviceToHost, sc->stream));
    if (cnt[1]) HIP_TRY(hipMemcpyAsync(out.data(), sc->swap_out_list, sizeof(SwapRec) * cnt[1], hipMemcpyDeviceToHost, sc->stream));
    HIP_TRY(hipStreamSynchronize(sc->stream));
    std::sort(in.begin(), in.end(), swap_key_less);
    std::sort(out.begin(), out.end(), swap_key_less);
    const int32_t n_in = std::min<int32_t>(cnt[0], sc->swap_in_cap);
    const int32_t n_out = std::min<int32_t>(cnt[1], sc->swap_out_cap);
    const int32_t xcap = std::max(sc->swap_in_cap, sc->swap_out_cap);
    SwapMoveArgs ma;
    ma.h = sa.h;
    ma.sdf = sc->sdf;
    ma.w = sc->w;
    ma.xfer_sdf = sc->xfer_sdf;
    ma.xfer_w = sc->xfer_w;
    ma.entries = sc->xfer_entries;
    ma.onhost = sc->onhost;
    ma.max_w = (float)sc->max_w;
    ma.pool = sa.pool;
    std::vector<int32_t> ents;
    // swap in: host copies into the transfer buffer (F then W parts, as on the
    // device), then merged into the device blocks
    if (n_in) {
        uint8_t *hs = sc->xfer_host, *hw = sc->xfer_host + es * kBlockVox * (size_t)xcap;
        ents.resize(n_in);
        for (int32_t i = 0; i < n_in; i++) {
            const int32_t e = in[i].e;
            const int32_t slot = sc->host_slot[e];
            const uint8_t *src = sc->host_data.data() + (size_t)slot * blk_bytes;
            std::memcpy(hs + es * kBlockVox * (size_t)i, src, es * kBlockVox);
            std::memcpy(hw + ew * kBlockVox * (size_t)i, src + es * kBlockVox, ew * kBlockVox);
            ents[i] = e;
        }
        HIP_TRY(hipMemcpyAsync(sc->xfer_sdf, hs, es * kBlockVox * (size_t)n_in, hipMemcpyHostToDevice, sc->stream));
        HIP_TRY(hipMemcpyAsync(sc->xfer_w, hw, ew * kBlockVox * (size_t)n_in, hipMemcpyHostToDevice, sc->stream));
        HIP_TRY(hipMemcpyAsync(sc->xfer_entries, ents.data(), sizeof(int32_t) * n_in, hipMemcpyHostToDevice,
                               sc->stream));
        ma.n = n_in;
        HIP_TRY(launch_swap_move(sc->fmt, false, ma, sc->stream));
        HIP_TRY(hipStreamSynchronize(sc->stream));   // the buffers are reused below
        for (int32_t i = 0; i < n_in; i++) {
            sc->host_free.push_back(sc->host_slot[in[i].e]);
            sc->host_slot[in[i].e] = -1;
        }
    }
    // swap out: device blocks through the transfer buffer to host slots
    if (n_out) {
        ents.resize(n_out);
        for (int32_t i = 0; i < n_out; i++) ents[i] = out[i].e;
        HIP_TRY(hipMemcpyAsync(sc->xfer_entries, ents.data(), sizeof(int32_t) * n_out, hipMemcpyHostToDevice,
                               sc->stream));
        ma.n = n_out;
        HIP_TRY(launch_swap_move(sc->fmt, true, ma, sc->stream));
        uint8_t *hs = sc->xfer_host, *hw = sc->xfer_host + es * kBlockVox * (size_t)xcap;
        HIP_TRY(hipMemcpyAsync(hs, sc->xfer_sdf, es * kBlockVox * (size_t)n_out, hipMemcpyDeviceToHost, sc->stream));
        HIP_TRY(hipMemcpyAsync(hw, sc->xfer_w, ew * kBlockVox * (size_t)n_out, hipMemcpyDeviceToHost, sc->stream));
        HIP_TRY(hipStreamSynchronize(sc->stream));
        for (int32_t i = 0; i < n_out; i++) {
            int32_t slot;
            if (!sc->host_free.empty()) {
                slot = sc->host_free.back();
                sc->host_free.pop_back();
            } else {
                slot = (int32_t)(sc->host_data.size() / blk_bytes);
                sc->host_data.resize(sc->host_data.size() + blk_bytes);
            }
            uint8_t *dst = sc->host_data.data() + (size_t)slot * blk_bytes;
            std::memcpy(dst, hs + es * kBlockVox * (size_t)i, es * kBlockVox);
            std::memcpy(dst + es * kBlockVox, hw + ew * kBlockVox * (size_t)i, ew * kBlockVox);
            sc->host_slot[out[i].e] = slot;
        }
    }
    sc->swapped_in_last = n_in;
    sc->swapped_out_last = n_out;
    sc->swapped_in_total += n_in;
    sc->swapped_out_total += n_out;
    return ITM_OK;
}

// one frame: allocation, visible list and integration; with rgbx set, the
// colour voxels too
itm_status integrate_frame(itm_scene *sc, const float *depth, const uchar4 *rgbx, const itm_intrinsics *K,
                           const double *T_wc)
{
    FrameGeom g;
    if (itm_status st = make_geom(sc, K, T_wc, &g)) return st;
    if (sc->range_on)
        if (itm_status st = ensure_bins(sc, g.W, g.H)) return st;
    FuseArgs a = frame_args(sc, g, sc->range_on);
    a.depth = depth;
    a.clr = rgbx ? sc->clr : nullptr;
    a.rgbx = rgbx;
    {
        ProfScope ps(sc, 0);
        HIP_TRY(launch_alloc(a, sc->stream));
    }
    {
        ProfScope ps(sc, 1);
        // 5 workgroups per CU: every wave resident at once (about one block each at
        // VGA), looping over its share of the list when more are listed; a
        // multiple of 8 workgroups
        const int grid = (int)std::min<int64_t>((int64_t)sc->num_cu * 5, 16384) / 8 * 8;
        HIP_TRY(launch_integrate(sc->fmt, a, grid, sc->stream));
    }
    sc->fused_frame = sc->range_on ? sc->frame : -1;
    if (sc->range_on) {
        sc->fused_K = *K;
        std::memcpy(sc->fused_T, T_wc, sizeof sc->fused_T);
    }
    sc->frame++;
    if (sc->swap && (sc->swap_in_cap > 0 || sc->swap_out_cap > 0)) return swap_frame(sc);
    if (sc->refiner) return refine_visible(sc);
    return ITM_OK;
}

itm_status raycast_frame(itm_scene *sc, const itm_intrinsics *K, const double *T_wc, float *out_pts,
                         float *out_normals, uchar4 *out_rgbx)
{
    if (((uintptr_t)out_pts | (uintptr_t)out_normals) & 15u)
        return fail(ITM_ERR_ARG, "outputs must be 16-byte aligned");
    FrameGeom g;
    if (itm_status st = make_geom(sc, K, T_wc, &g)) return st;
    ProfScope ps(sc, 2);
    RaycastArgs a;
    a.fg = g;
    a.h = hash_view(sc);
    a.sdf = sc->sdf;
    a.pts = reinterpret_cast<float4 *>(out_pts);
    a.nrm = reinterpret_cast<float4 *>(out_normals);
    a.clr = out_rgbx ? sc->clr : nullptr;
    a.rgb_out = out_rgbx;
    a.rb = RangeBins{};
    a.list = vis_list(sc, last_parity(sc));
    // with a refiner, the blocks it refined after the last frame are read from
    // its output (the plain F stays the fallback for every other block)
    const bool ref = sc->refiner && sc->refined && sc->frame > 0;
    a.refined = ref ? sc->refined : nullptr;
    a.rstamp = ref ? sc->stamp : nullptr;
    a.rframe = sc->frame;
    if (sc->range_on)
        if (itm_status st = bins_for_pose(sc, K, T_wc, g, &a.rb)) return st;
    HIP_TRY(launch_raycast(sc->fmt, a, sc->stream));
    return ITM_OK;
}

}  // namespace

extern "C" {

itm_status itm_integrate(itm_scene *sc, const float *depth, const itm_intrinsics *K, const double *T_wc)
{
    if (!sc || !depth) return fail(ITM_ERR_ARG, "NULL scene or depth");
    return integrate_frame(sc, depth, nullptr, K, T_wc);
}

itm_status itm_raycast(itm_scene *sc, const itm_intrinsics *K, const double *T_wc, float *out_pts,
                       float *out_normals)
{
    if (!sc || !out_pts || !out_normals) return fail(ITM_ERR_ARG, "NULL scene or output");
    return raycast_frame(sc, K, T_wc, out_pts, out_normals, nullptr);
}

itm_status itm_scene_enable_colour(itm_scene *sc)
{
    if (!sc) return fail(ITM_ERR_ARG, "NULL scene");
    if (sc->clr) return ITM_OK;
    if (sc->swap) return fail(ITM_ERR_STATE, "colour does not combine with swapping");
    const size_t bytes = sizeof(uchar4) * kBlockVox * (size_t)sc->vba_cap;
    if (itm_status st = dev_alloc((void **)&sc->clr, bytes, "colour voxels")) return st;
    hipError_t e = hipMemsetAsync(sc->clr, 0, bytes, sc->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
    if (e != hipSuccess) {
        (void)hipFree(sc->clr);
        sc->clr = nullptr;
        return fail(ITM_ERR_HIP, "colour voxel initialisation failed: %s", hipGetErrorString(e));
    }
    return ITM_OK;
}

itm_status itm_integrate_colour(itm_scene *sc, const float *depth, const uint8_t *rgbx, const itm_intrinsics *K,
                                const double *T_wc)
{
    if (!sc || !depth || !rgbx) return fail(ITM_ERR_ARG, "NULL scene, depth or colour image");
    if (!sc->clr) return fail(ITM_ERR_ARG, "colour is not enabled on this scene");
    if ((uintptr_t)rgbx & 3u) return fail(ITM_ERR_ARG, "colour image must be 4-byte aligned");
    return integrate_frame(sc, depth, reinterpret_cast<const uchar4 *>(rgbx), K, T_wc);
}

itm_status itm_raycast_colour(itm_scene *sc, const itm_intrinsics *K, const double *T_wc, float *out_pts,
                              float *out_normals, uint8_t *out_rgbx)
{
    if (!sc || !out_pts || !out_normals || !out_rgbx) return fail(ITM_ERR_ARG, "NULL scene or output");
    if (!sc->clr) return fail(ITM_ERR_ARG, "colour is not enabled on this scene");
    if ((uintptr_t)out_rgbx & 3u) return fail(ITM_ERR_ARG, "colour output must be 4-byte aligned");
    return raycast_frame(sc, K, T_wc, out_pts, out_normals, reinterpret_cast<uchar4 *>(out_rgbx));
}

itm_status itm_scene_set_search_range(itm_scene *sc, int32_t enable, int32_t tile_capacity)
{
    if (!sc) return fail(ITM_ERR_ARG, "NULL scene");
    const int32_t cap = tile_capacity <= 0 ? 512 : tile_capacity;
    if (cap > (1 << 16)) return fail(ITM_ERR_ARG, "tile capacity %d > 65536", tile_capacity);
    if (cap != sc->range_cap && sc->bin_cnt) {   // reallocated at the next use
        HIP_TRY(hipStreamSynchronize(sc->stream));
        (void)hipFree(sc->bin_cnt);
        (void)hipFree(sc->bin_rect);
        sc->bin_cnt = nullptr;
        sc->bin_rect = nullptr;
        sc->bin_tiles = 0;
    }
    sc->range_cap = cap;
    if (enable && !sc->range_on && sc->bin_cnt)   // counts left from an earlier period
        HIP_TRY(launch_range_clear(sc->bin_cnt, (int)(3 * sc->bin_tiles), sc->stream));
    sc->range_on = enable != 0;
    sc->fused_frame = -1;
    return ITM_OK;
}

itm_status itm_expected_depths(itm_scene *sc, const itm_intrinsics *K, const double *T_wc, float *zrange)
{
    if (!sc || !zrange) return fail(ITM_ERR_ARG, "NULL scene or output");
    if ((uintptr_t)zrange & 7u) return fail(ITM_ERR_ARG, "output must be 8-byte aligned");
    FrameGeom g;
    if (itm_status st = make_geom(sc, K, T_wc, &g)) return st;
    RangeBins rb;
    if (itm_status st = bins_for_pose(sc, K, T_wc, g, &rb)) return st;
    HIP_TRY(launch_range_image(g, vis_list(sc, last_parity(sc)), rb, reinterpret_cast<float2 *>(zrange),
                               sc->stream));
    return ITM_OK;
}

itm_status itm_get_stats(itm_scene *sc, itm_stats *out)
{
    if (!sc || !out) return fail(ITM_ERR_ARG, "NULL argument");
    Counters c;
    HIP_TRY(hipMemcpyAsync(&c, sc->cnt, sizeof c, hipMemcpyDeviceToHost, sc->stream));
    HIP_TRY(hipStreamSynchronize(sc->stream));
    // entries holding a key (each a block: on the device, or with swapping
    // possibly on the host)
    out->n_allocated = std::min<int64_t>(c.vba_next, sc->swap ? sc->n_entries : sc->vba_cap);
    unsigned long long v_last = 0, v_tot = 0;
    for (int i = 0; i < kStripes; i++) {
        v_last += c.vis[last_parity(sc)][i][0];
        v_tot += c.vis[2][i][0];
    }
    out->n_visible_last = (int64_t)v_last;
    out->n_excess_used = std::min<int64_t>(c.excess_next, sc->n_excess);
    out->n_dropped_total = (int64_t)c.dropped_total;
    out->vba_capacity = sc->vba_cap;
    unsigned long long u_last = 0, u_tot = 0;
    for (int i = 0; i < kStripes; i++) {
        u_last += c.upd[last_parity(sc)][i][0];
        u_tot += c.upd[2][i][0];
    }
    out->n_updated_last = (int64_t)u_last;
    out->n_entries = sc->n_entries;
    out->bytes_per_voxel = (int64_t)(sdf_elem(sc->fmt) + w_elem(sc->fmt));
    out->n_visible_total = (int64_t)v_tot;
    out->n_updated_total = (int64_t)u_tot;
    return ITM_OK;
}

}  // extern "C"

namespace {

struct BlockRec { int32_t x, y, z, blk; };

// every allocated block (key and voxel block = entry id), sorted by (x, y, z)
itm_status collect_blocks(itm_scene *sc, std::vector<BlockRec> &recs)
{
    std::vector<Bucket> hb(sc->n_buckets);
    std::vector<Excess> hx(std::max<int64_t>(sc->n_excess, 1));
    HIP_TRY(hipMemcpyAsync(hb.data(), sc->buckets, sizeof(Bucket) * sc->n_buckets, hipMemcpyDeviceToHost,
                           sc->stream));
    if (sc->n_excess)
        HIP_TRY(hipMemcpyAsync(hx.data(), sc->excess, sizeof(Excess) * sc->n_excess, hipMemcpyDeviceToHost,
                               sc->stream));
    HIP_TRY(hipStreamSynchronize(sc->stream));
    recs.clear();
    auto add = [&](unsigned long long k, int64_t e) {
        if (!(k & kKeyValid)) return;
        BlockRec r;
        r.x = (int16_t)(k & 0xffff);
        r.y = (int16_t)((k >> 16) & 0xffff);
        r.z = (int16_t)((k >> 32) & 0xffff);
        r.blk = (int32_t)e;
        recs.push_back(r);
    };
    for (int64_t b = 0; b < sc->n_buckets; b++) {
        add(hb[b].key[0], 2 * b);
        add(hb[b].key[1], 2 * b + 1);
    }
    for (int64_t i = 0; i < sc->n_excess; i++) add(hx[i].key, 2 * sc->n_buckets + i);
    std::sort(recs.begin(), recs.end(), [](const BlockRec &a, const BlockRec &b) {
        if (a.x != b.x) return a.x < b.x;
        if (a.y != b.y) return a.y < b.y;
        return a.z < b.z;
    });
    return ITM_OK;
}

}  // namespace

extern "C" {

itm_status itm_export_blocks(itm_scene *sc, int32_t *coords, float *sdf, float *w, int64_t capacity,
                             int64_t *n_blocks)
{
    if (!sc || !n_blocks) return fail(ITM_ERR_ARG, "NULL scene or n_blocks");
    std::vector<BlockRec> recs;
    if (itm_status st = collect_blocks(sc, recs)) return st;
    const int64_t n = (int64_t)recs.size();
    *n_blocks = n;
    if (!coords && !sdf && !w) return ITM_OK;
    if (capacity < n) return fail(ITM_ERR_ARG, "capacity %lld < %lld blocks", (long long)capacity, (long long)n);
    for (int64_t i = 0; i < n && coords; i++) {
        coords[3 * i] = recs[i].x;
        coords[3 * i + 1] = recs[i].y;
        coords[3 * i + 2] = recs[i].z;
    }
    if ((!sdf && !w) || n == 0) return ITM_OK;
    // with swapping a block's data may sit on the device, on the host, or both
    // (a host copy not merged yet: exported merged, as the swap-in would merge it)
    const bool swp = sc->swap;
    std::vector<int32_t> dblk;
    std::vector<uint8_t> onh;
    if (swp) {
        dblk.resize(sc->n_entries);
        onh.resize(sc->n_entries);
        HIP_TRY(hipMemcpyAsync(dblk.data(), sc->blk, sizeof(int32_t) * sc->n_entries, hipMemcpyDeviceToHost,
                               sc->stream));
        HIP_TRY(hipMemcpyAsync(onh.data(), sc->onhost, sc->n_entries, hipMemcpyDeviceToHost, sc->stream));
        HIP_TRY(hipStreamSynchronize(sc->stream));
    }
    const bool want_s = sdf || swp, want_w = w || swp;
    // the blocks' voxels, packed on the device in export order, then one copy
    const size_t es = sdf_elem(sc->fmt), ew = w_elem(sc->fmt);
    std::vector<int32_t> blk(n);
    for (int64_t i = 0; i < n; i++) blk[i] = swp ? std::max(dblk[recs[i].blk], 0) : recs[i].blk;
    int32_t *d_blk = nullptr;
    void *d_s = nullptr, *d_w = nullptr;
    itm_status st = dev_alloc((void **)&d_blk, sizeof(int32_t) * n, "export list");
    if (!st && want_s) st = dev_alloc(&d_s, es * kBlockVox * n, "export sdf");
    if (!st && want_w) st = dev_alloc(&d_w, ew * kBlockVox * n, "export weights");
    std::vector<uint8_t> hs(want_s ? es * kBlockVox * n : 0), hw(want_w ? ew * kBlockVox * n : 0);
    hipError_t e = hipSuccess;
    if (!st) {
        e = hipMemcpyAsync(d_blk, blk.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, sc->stream);
        if (e == hipSuccess) e = launch_export_gather(sc->fmt, sc->sdf, sc->w, d_blk, n, d_s, d_w, sc->stream);
        if (e == hipSuccess && want_s) e = hipMemcpyAsync(hs.data(), d_s, hs.size(), hipMemcpyDeviceToHost, sc->stream);
        if (e == hipSuccess && want_w) e = hipMemcpyAsync(hw.data(), d_w, hw.size(), hipMemcpyDeviceToHost, sc->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
    }
    (void)hipFree(d_blk);
    (void)hipFree(d_s);
    (void)hipFree(d_w);
    if (st) return st;
    if (e != hipSuccess) return fail(ITM_ERR_HIP, "export failed: %s", hipGetErrorString(e));
    const size_t blk_bytes = (es + ew) * kBlockVox;
    for (int64_t i = 0; i < n; i++) {
        const size_t src = (size_t)i * kBlockVox;
        int32_t db = 0, slot = -1;
        if (swp) {
            const int32_t ent = recs[i].blk;
            db = dblk[ent];
            slot = onh[ent] ? sc->host_slot[ent] : -1;
        }
        const uint8_t *host = slot >= 0 ? sc->host_data.data() + (size_t)slot * blk_bytes : nullptr;
        for (int l = 0; l < kBlockVox; l++) {
            float f = 1.0f, wf = 0.0f;
            if (db >= 0) {   // the device copy
                if (want_s) f = decode_sdf(sc->fmt, &hs[es * (src + l)]);
                if (want_w) wf = decode_w(sc->fmt, &hw[ew * (src + l)]);
            }
            if (host) {      // the host copy, merged into the device copy when there is one
                const float fh = decode_sdf(sc->fmt, host + es * l);
                const float whv = decode_w(sc->fmt, host + es * kBlockVox + ew * l);
                if (db < 0) {
                    f = fh;
                    wf = whv;
                } else {
                    const float wn = wf + whv;
                    if (wn > 0.0f) {
                        f = (wf * f + whv * fh) / wn;
                        wf = std::min(wn, (float)sc->max_w);
                    }
                }
            }
            if (sdf) sdf[src + l] = f;
            if (w) w[src + l] = wf;
        }
    }
    return ITM_OK;
}

itm_status itm_scene_enable_swapping(itm_scene *sc, int64_t device_blocks, int32_t swap_in, int32_t swap_out)
{
    if (!sc) return fail(ITM_ERR_ARG, "NULL scene");
    if (sc->swap) return fail(ITM_ERR_STATE, "swapping is already on");
    if (sc->frame != 0) return fail(ITM_ERR_STATE, "swapping must be enabled before the first frame");
    if (sc->clr || sc->refiner) return fail(ITM_ERR_STATE, "swapping does not combine with colour or a refiner");
    if (device_blocks < 1 || device_blocks > sc->n_entries || device_blocks > INT32_MAX)
        return fail(ITM_ERR_ARG, "device_blocks %lld not in [1, %lld]", (long long)device_blocks,
                    (long long)sc->n_entries);
    const bool pool_only = swap_in == 0 && swap_out == 0;   // a device pool without transfers
    if (!pool_only && (swap_in < 1 || swap_out < 1 || swap_in > (1 << 20) || swap_out > (1 << 20)))
        return fail(ITM_ERR_ARG, "transfer sizes must be in [1, 2^20] blocks (or both 0)");
    HIP_TRY(hipStreamSynchronize(sc->stream));
    // the voxel block array becomes the device pool
    (void)hipFree(sc->sdf);
    (void)hipFree(sc->w);
    sc->sdf = sc->w = nullptr;
    sc->vba_cap = device_blocks;
    const int64_t n_vox = device_blocks * kBlockVox;
    const size_t es = sdf_elem(sc->fmt), ew = w_elem(sc->fmt);
    const int32_t xcap = std::max(1, std::max(swap_in, swap_out));
    if (itm_status st = dev_alloc(&sc->sdf, es * n_vox, "sdf")) return st;
    if (itm_status st = dev_alloc(&sc->w, ew * n_vox, "weights")) return st;
    if (dev_alloc((void **)&sc->blk, sizeof(int32_t) * sc->n_entries, "entry blocks") ||
        dev_alloc((void **)&sc->onhost, sc->n_entries, "host flags") ||
        dev_alloc((void **)&sc->pool_stack, sizeof(int32_t) * device_blocks, "block pool") ||
        dev_alloc((void **)&sc->pool_top, sizeof(int32_t) * 2, "pool top") ||
        dev_alloc((void **)&sc->pool_noblock, sizeof(unsigned long long), "pool misses") ||
        dev_alloc((void **)&sc->swap_in_list, sizeof(SwapRec) * sc->n_entries, "swap-in candidates") ||
        dev_alloc((void **)&sc->swap_out_list, sizeof(SwapRec) * sc->n_entries, "swap-out candidates") ||
        dev_alloc((void **)&sc->swap_cnt, sizeof(int32_t) * 2, "swap counts") ||
        dev_alloc(&sc->xfer_sdf, es * kBlockVox * (size_t)xcap, "transfer sdf") ||
        dev_alloc(&sc->xfer_w, ew * kBlockVox * (size_t)xcap, "transfer weights") ||
        dev_alloc((void **)&sc->xfer_entries, sizeof(int32_t) * xcap, "transfer entries"))
        return ITM_ERR_OOM;
    if (hipHostMalloc((void **)&sc->xfer_host, (es + ew) * kBlockVox * (size_t)xcap) != hipSuccess)
        return fail(ITM_ERR_OOM, "pinned transfer buffer of %d blocks", xcap);
    hipError_t e = launch_init(sc->buckets, sc->head, sc->n_buckets, sc->excess, sc->n_excess, sc->vis_stamp,
                               sc->n_entries, sc->set, 2 * sc->set_size, sc->occ,
                               sc->occ_words + kMacroWords, sc->cnt, sc->fmt, sc->sdf, sc->w,
                               n_vox, sc->stream);
    if (e == hipSuccess)
        e = launch_swap_init(sc->pool_stack, (int32_t)device_blocks, sc->pool_top, sc->blk, sc->onhost,
                             sc->n_entries, sc->stream);
    if (e == hipSuccess) e = hipMemsetAsync(sc->pool_noblock, 0, sizeof(unsigned long long), sc->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
    if (e != hipSuccess) return fail(ITM_ERR_HIP, "swapping set-up failed: %s", hipGetErrorString(e));
    sc->host_slot.assign(sc->n_entries, -1);
    sc->host_data.clear();
    sc->host_free.clear();
    sc->swap_in_cap = swap_in;
    sc->swap_out_cap = swap_out;
    sc->swap = true;
    return ITM_OK;
}

itm_status itm_swap_stats(itm_scene *sc, int64_t *out)
{
    if (!sc || !out) return fail(ITM_ERR_ARG, "NULL argument");
    if (!sc->swap) return fail(ITM_ERR_STATE, "swapping is off");
    std::vector<int32_t> dblk(sc->n_entries);
    std::vector<uint8_t> onh(sc->n_entries);
    int32_t top = 0;
    unsigned long long nob = 0;
    HIP_TRY(hipMemcpyAsync(dblk.data(), sc->blk, sizeof(int32_t) * sc->n_entries, hipMemcpyDeviceToHost, sc->stream));
    HIP_TRY(hipMemcpyAsync(onh.data(), sc->onhost, sc->n_entries, hipMemcpyDeviceToHost, sc->stream));
    HIP_TRY(hipMemcpyAsync(&top, sc->pool_top, sizeof top, hipMemcpyDeviceToHost, sc->stream));
    HIP_TRY(hipMemcpyAsync(&nob, sc->pool_noblock, sizeof nob, hipMemcpyDeviceToHost, sc->stream));
    HIP_TRY(hipStreamSynchronize(sc->stream));
    int64_t n_dev = 0, host_only = 0, pending = 0;
    for (int64_t e = 0; e < sc->n_entries; e++) {
        n_dev += dblk[e] >= 0;
        host_only += onh[e] && dblk[e] < 0;
        pending += onh[e] && dblk[e] >= 0;
    }
    out[0] = n_dev;
    out[1] = host_only;
    out[2] = pending;
    out[3] = sc->swapped_in_last;
    out[4] = sc->swapped_out_last;
    out[5] = sc->swapped_in_total;
    out[6] = sc->swapped_out_total;
    out[7] = (int64_t)nob;
    (void)top;
    return ITM_OK;
}

itm_status itm_import_blocks(itm_scene *sc, const int32_t *coords, const float *sdf, const float *w, int64_t n)
{
    if (!sc) return fail(ITM_ERR_ARG, "NULL scene");
    if (sc->swap) return fail(ITM_ERR_STATE, "loading blocks does not combine with swapping");
    if (n < 0 || n > (int64_t)INT32_MAX / 4) return fail(ITM_ERR_ARG, "n = %lld out of range", (long long)n);
    if (n > 0 && (!coords || !sdf || !w)) return fail(ITM_ERR_ARG, "NULL coords, sdf or w");
    // host checks: keys in range and distinct, values a valid voxel state
    std::vector<int64_t> keys((size_t)n);
    for (int64_t i = 0; i < n; i++) {
        for (int c = 0; c < 3; c++)
            if (coords[3 * i + c] < -32767 || coords[3 * i + c] > 32767)
                return fail(ITM_ERR_ARG, "block %lld: coordinate %d out of the 16-bit range", (long long)i,
                            coords[3 * i + c]);
        keys[i] = ((int64_t)(coords[3 * i] + 32768) << 32) | ((int64_t)(coords[3 * i + 1] + 32768) << 16) |
                  (int64_t)(coords[3 * i + 2] + 32768);
    }
    std::sort(keys.begin(), keys.end());
    if (std::adjacent_find(keys.begin(), keys.end()) != keys.end())
        return fail(ITM_ERR_ARG, "a block appears twice in the list");
    for (int64_t i = 0; i < n * kBlockVox; i++) {
        const float f = sdf[i], wv = w[i];
        if (!(f >= -1.0f && f <= 1.0f)) return fail(ITM_ERR_ARG, "voxel %lld: F = %g not in [-1, 1]", (long long)i, f);
        if (!(wv >= 0.0f && wv <= (float)sc->max_w) || wv != std::floor(wv))
            return fail(ITM_ERR_ARG, "voxel %lld: W = %g is not an integer in [0, %d]", (long long)i, wv, sc->max_w);
    }
    // a frame of its own: find or insert every key, list it
    FrameGeom g = {};
    FuseArgs a = frame_args(sc, g, false);
    int32_t *d_coords = nullptr, *d_entry = nullptr;
    float *d_s = nullptr, *d_w = nullptr;
    constexpr int64_t kChunk = 16384;   // blocks of voxels per copy (32 MiB per array)
    const int64_t chunk = std::min<int64_t>(std::max<int64_t>(n, 1), kChunk);
    itm_status st = dev_alloc((void **)&d_coords, sizeof(int32_t) * 3 * std::max<int64_t>(n, 1), "import keys");
    if (!st) st = dev_alloc((void **)&d_entry, sizeof(int32_t) * std::max<int64_t>(n, 1), "import entries");
    if (!st) st = dev_alloc((void **)&d_s, sizeof(float) * kBlockVox * chunk, "import sdf");
    if (!st) st = dev_alloc((void **)&d_w, sizeof(float) * kBlockVox * chunk, "import weights");
    hipError_t e = hipSuccess;
    if (!st) {
        if (n > 0) e = hipMemcpyAsync(d_coords, coords, sizeof(int32_t) * 3 * n, hipMemcpyHostToDevice, sc->stream);
        if (e == hipSuccess) e = launch_import_keys(a, d_coords, (int32_t)n, d_entry, sc->stream);
        for (int64_t off = 0; off < n && e == hipSuccess; off += chunk) {
            const int64_t m = std::min(chunk, n - off);
            e = hipMemcpyAsync(d_s, sdf + off * kBlockVox, sizeof(float) * kBlockVox * m, hipMemcpyHostToDevice,
                               sc->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_w, w + off * kBlockVox, sizeof(float) * kBlockVox * m, hipMemcpyHostToDevice,
                                   sc->stream);
            if (e == hipSuccess)
                e = launch_import_voxels(sc->fmt, d_entry + off, d_s, d_w, m, sc->sdf, sc->w, sc->clr, sc->stream);
            // the staging buffers are reused by the next chunk
            if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
    }
    (void)hipFree(d_coords);
    (void)hipFree(d_entry);
    (void)hipFree(d_s);
    (void)hipFree(d_w);
    if (st) return st;
    if (e != hipSuccess) return fail(ITM_ERR_HIP, "import failed: %s", hipGetErrorString(e));
    sc->fused_frame = -1;   // no bins at any pose: a search range re-bins the imported set
    sc->frame++;
    return ITM_OK;
}

itm_status itm_export_colour(itm_scene *sc, uint8_t *rgbw, int64_t capacity, int64_t *n_blocks)
{
    if (!sc || !n_blocks) return fail(ITM_ERR_ARG, "NULL scene or n_blocks");
    if (!sc->clr) return fail(ITM_ERR_ARG, "colour is not enabled on this scene");
    std::vector<BlockRec> recs;
    if (itm_status st = collect_blocks(sc, recs)) return st;
    const int64_t n = (int64_t)recs.size();
    *n_blocks = n;
    if (!rgbw || n == 0) return ITM_OK;
    if (capacity < n) return fail(ITM_ERR_ARG, "capacity %lld < %lld blocks", (long long)capacity, (long long)n);
    std::vector<int32_t> blk(n);
    for (int64_t i = 0; i < n; i++) blk[i] = recs[i].blk;
    int32_t *d_blk = nullptr;
    uchar4 *d_c = nullptr;
    itm_status st = dev_alloc((void **)&d_blk, sizeof(int32_t) * n, "export list");
    if (!st) st = dev_alloc((void **)&d_c, sizeof(uchar4) * kBlockVox * n, "export colour");
    hipError_t e = hipSuccess;
    if (!st) {
        e = hipMemcpyAsync(d_blk, blk.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, sc->stream);
        if (e == hipSuccess) e = launch_export_colour(sc->clr, d_blk, n, d_c, sc->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rgbw, d_c, sizeof(uchar4) * kBlockVox * n, hipMemcpyDeviceToHost, sc->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
    }
    (void)hipFree(d_blk);
    (void)hipFree(d_c);
    if (st) return st;
    if (e != hipSuccess) return fail(ITM_ERR_HIP, "colour export failed: %s", hipGetErrorString(e));
    return ITM_OK;
}

itm_status itm_profile_enable(itm_scene *sc, int enable)
{
    if (!sc) return fail(ITM_ERR_ARG, "NULL scene");
    if (enable && sc->ev.empty()) {
        sc->ev.resize(2 * kProfSlots);
        sc->ev_kernel.resize(kProfSlots);
        for (auto &e : sc->ev) HIP_TRY(hipEventCreate(&e));
    }
    sc->prof = enable != 0;   // recorded events are collected by itm_profile_read
    return ITM_OK;
}

itm_status itm_profile_read(itm_scene *sc, double *ms, int64_t *launches)
{
    if (!sc || !ms || !launches) return fail(ITM_ERR_ARG, "NULL argument");
    if (itm_status st = prof_flush(sc)) return st;
    for (int k = 0; k < ITM_KERNEL_COUNT; k++) {
        ms[k] = sc->prof_ms[k];
        launches[k] = sc->prof_n[k];
        sc->prof_ms[k] = 0;
        sc->prof_n[k] = 0;
    }
    return ITM_OK;
}

// ---------------------------------------------------------------------------
// depth tracker
// ---------------------------------------------------------------------------
namespace {

// where a tracker call keeps its per-workgroup sums, pose and flags
struct TrackBufs {
    float *part;       // [kIcpSums][cap]
    int32_t cap;       // most workgroups whose sums fit
    double *pose;      // [16] current estimate, then [32] the last system
    int32_t *flags;    // [kTrackLevels] stop flags, the step count, the finished-workgroup count;
                       // right after the pose's 48 doubles, so that one copy reads both back
};

constexpr size_t kTrackStateBytes = sizeof(double) * 48 + sizeof(int32_t) * (kTrackLevels + 2);

// the scene's tracker scratch, allocated on first use
itm_status track_scratch(itm_scene *sc, TrackBufs &b)
{
    if (!sc->trk_part) {
        // one workgroup of 1024 threads per CU: a thread takes one or two pixels
        // of the finest level, and the last workgroup has few partials to add
        sc->trk_part_cap = sc->num_cu;
        if (itm_status st = dev_alloc((void **)&sc->trk_part, sizeof(float) * kIcpSums * (size_t)sc->trk_part_cap,
                                      "tracker sums"))
            return st;
        if (itm_status st = dev_alloc((void **)&sc->trk_pose, kTrackStateBytes, "tracker pose and flags")) return st;
    }
    b.part = sc->trk_part;
    b.cap = sc->trk_part_cap;
    b.pose = sc->trk_pose;
    b.flags = reinterpret_cast<int32_t *>(sc->trk_pose + 48);
    return ITM_OK;
}

itm_status track_check(const itm_scene *sc, const float *depth, const itm_intrinsics *K, const float *pts,
                       const float *nrm, const double *T_ref, const double *T)
{
    if (!sc || !depth || !K || !pts || !nrm || !T_ref || !T) return fail(ITM_ERR_ARG, "NULL argument");
    if (K->width < 1 || K->height < 1 || (int64_t)K->width * K->height > (int64_t)1 << 28)
        return fail(ITM_ERR_ARG, "image size %d x %d out of range", K->width, K->height);
    if (!(K->fx > 0) || !(K->fy > 0) || !std::isfinite(K->fx) || !std::isfinite(K->fy) || !std::isfinite(K->cx) ||
        !std::isfinite(K->cy))
        return fail(ITM_ERR_ARG, "intrinsics must have finite fx, fy > 0 and finite cx, cy");
    if (((uintptr_t)pts | (uintptr_t)nrm) & 15u) return fail(ITM_ERR_ARG, "reference maps must be 16-byte aligned");
    for (int i = 0; i < 16; i++)
        if (!std::isfinite(T_ref[i]) || !std::isfinite(T[i])) return fail(ITM_ERR_ARG, "pose not finite");
    return ITM_OK;
}

// level l of the hierarchy: input pixel (2^l u, 2^l v) as pixel (u, v), with
// intrinsics fx / 2^l, fy / 2^l, cx / 2^l, cy / 2^l
IcpArgs icp_args(const TrackBufs &b, const float *depth, const itm_intrinsics *K, int level, const float *pts,
                 const float *nrm, const double *T_ref, float dist)
{
    IcpArgs a;
    a.depth = depth;
    a.level = level;
    a.wl = (K->width + (1 << level) - 1) >> level;
    a.hl = (K->height + (1 << level) - 1) >> level;
    const double f = std::ldexp(1.0, -level);
    a.fxl = (float)(K->fx * f);
    a.fyl = (float)(K->fy * f);
    a.cxl = (float)(K->cx * f);
    a.cyl = (float)(K->cy * f);
    a.fx = (float)K->fx;
    a.fy = (float)K->fy;
    a.cx = (float)K->cx;
    a.cy = (float)K->cy;
    a.W = K->width;
    a.H = K->height;
    a.V = reinterpret_cast<const float4 *>(pts);
    a.N = reinterpret_cast<const float4 *>(nrm);
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) a.Rr[3 * i + j] = (float)T_ref[4 * i + j];
        a.tr[i] = (float)T_ref[4 * i + 3];
    }
    a.dist = dist;
    a.pose = b.pose;
    a.stop = b.flags + level;   // cleared by k_track_init; set only by steps that update
    a.steps = nullptr;
    a.part = b.part;
    a.part_stride = b.cap;
    a.done = reinterpret_cast<uint32_t *>(b.flags + kTrackLevels + 1);
    a.sys = b.pose + 16;
    a.min_inliers = 0;
    a.update = 0;
    return a;
}

int icp_grid(const TrackBufs &b, const IcpArgs &a)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)a.wl * a.hl + kIcpThreads - 1) / kIcpThreads, b.cap));
}

PoseInit pose_init(const TrackBufs &b, const double *T)
{
    PoseInit p;
    std::memcpy(p.T, T, sizeof p.T);
    p.pose = b.pose;
    p.stop = b.flags;
    p.steps = b.flags + kTrackLevels;
    p.done = reinterpret_cast<uint32_t *>(b.flags + kTrackLevels + 1);
    return p;
}

// the Gauss-Newton loop of itm_track over the levels, with its sums, pose and
// flags in b (arguments already checked)
itm_status track_run(itm_scene *sc, const TrackBufs &b, const float *depth, const itm_intrinsics *K,
                     const float *ref_pts, const float *ref_normals, const double *T_ref, const double *T_init,
                     const itm_track_params *params, double *T_out, itm_track_info *info)
{
    if (!T_out) return fail(ITM_ERR_ARG, "NULL T_out");
    itm_track_params p;
    if (params) p = *params;
    else itm_track_default_params(&p);
    if (p.n_levels < 1 || p.n_levels > kTrackLevels)
        return fail(ITM_ERR_ARG, "n_levels %d not in [1, %d]", p.n_levels, kTrackLevels);
    for (int l = 0; l < p.n_levels; l++) {
        if (p.iters[l] < 0 || p.iters[l] > 1000) return fail(ITM_ERR_ARG, "iters[%d] = %d not in [0, 1000]", l, p.iters[l]);
        if (!(p.dist_thresh[l] > 0) || !std::isfinite(p.dist_thresh[l]))
            return fail(ITM_ERR_ARG, "dist_thresh[%d] must be finite and > 0", l);
    }
    for (int l = 1; l < p.n_levels; l++)
        if ((K->width >> l) < 1 || (K->height >> l) < 1)
            return fail(ITM_ERR_ARG, "a %d x %d image has no level %d", K->width, K->height, l);
    HIP_TRY(launch_track_init(pose_init(b, T_init), sc->stream));
    for (int l = p.n_levels - 1; l >= 0; l--) {
        IcpArgs a = icp_args(b, depth, K, l, ref_pts, ref_normals, T_ref, p.dist_thresh[l]);
        a.steps = b.flags + kTrackLevels;
        a.min_inliers = p.min_inliers;
        a.update = 1;
        const int grid = icp_grid(b, a);
        for (int it = 0; it < p.iters[l]; it++) {
            ProfScope ps(sc, l == 0 ? 4 : 5);
            HIP_TRY(launch_icp_step(a, grid, sc->stream));
        }
    }
    alignas(8) unsigned char state[kTrackStateBytes];   // the pose, the last system and the flags
    HIP_TRY(hipMemcpyAsync(state, b.pose, sizeof state, hipMemcpyDeviceToHost, sc->stream));
    HIP_TRY(hipStreamSynchronize(sc->stream));
    double host[48];
    int32_t flags[kTrackLevels + 2];
    std::memcpy(host, state, sizeof host);
    std::memcpy(flags, state + sizeof host, sizeof flags);
    std::memcpy(T_out, host, sizeof(double) * 16);
    if (info) {
        // the last system evaluated (zeros when no step ran)
        bool any = false;
        for (int l = 0; l < p.n_levels; l++) any = any || p.iters[l] > 0;
        const double *sys = host + 16;
        info->n_pairs = any ? (int64_t)sys[28] : 0;
        info->rms = any && sys[28] > 0 ? std::sqrt(sys[27] / sys[28]) : 0.0;
        info->steps = flags[kTrackLevels];
    }
    return ITM_OK;
}

}  // namespace

extern "C" {

void itm_track_default_params(itm_track_params *p)
{
    if (!p) return;
    p->n_levels = 3;
    p->iters[0] = 4; p->iters[1] = 6; p->iters[2] = 10; p->iters[3] = 10;
    p->dist_thresh[0] = 0.02f; p->dist_thresh[1] = 0.05f; p->dist_thresh[2] = 0.1f; p->dist_thresh[3] = 0.2f;
    p->min_inliers = 100;
}

itm_status itm_track(itm_scene *sc, const float *depth, const itm_intrinsics *K, const float *ref_pts,
                     const float *ref_normals, const double *T_ref, const double *T_init,
                     const itm_track_params *params, double *T_out, itm_track_info *info)
{
    if (itm_status st = track_check(sc, depth, K, ref_pts, ref_normals, T_ref, T_init)) return st;
    TrackBufs b;
    if (itm_status st = track_scratch(sc, b)) return st;
    return track_run(sc, b, depth, K, ref_pts, ref_normals, T_ref, T_init, params, T_out, info);
}

itm_status itm_icp_system(itm_scene *sc, const float *depth, const itm_intrinsics *K, int32_t level,
                          const float *ref_pts, const float *ref_normals, const double *T_ref, const double *T,
                          float dist_thresh, double *sys)
{
    if (itm_status st = track_check(sc, depth, K, ref_pts, ref_normals, T_ref, T)) return st;
    if (!sys) return fail(ITM_ERR_ARG, "NULL sys");
    if (level < 0 || level >= kTrackLevels) return fail(ITM_ERR_ARG, "level %d not in [0, %d)", level, kTrackLevels);
    if (!(dist_thresh > 0) || !std::isfinite(dist_thresh)) return fail(ITM_ERR_ARG, "dist_thresh must be finite and > 0");
    if ((K->width >> level) < 1 || (K->height >> level) < 1)
        return fail(ITM_ERR_ARG, "a %d x %d image has no level %d", K->width, K->height, level);
    TrackBufs b;
    if (itm_status st = track_scratch(sc, b)) return st;
    HIP_TRY(launch_track_init(pose_init(b, T), sc->stream));
    const IcpArgs a = icp_args(b, depth, K, level, ref_pts, ref_normals, T_ref, dist_thresh);
    HIP_TRY(launch_icp_step(a, icp_grid(b, a), sc->stream));
    HIP_TRY(hipMemcpyAsync(sys, b.pose + 16, sizeof(double) * kIcpSums, hipMemcpyDeviceToHost, sc->stream));
    HIP_TRY(hipStreamSynchronize(sc->stream));
    return ITM_OK;
}


}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free tracking: the sums, pose and flags in a file-scope device
// array instead of the scene's lazily allocated scratch
// ---------------------------------------------------------------------------
namespace {

constexpr int kStaticParts = 1024;   // most sum workgroups (one per CU is used)
constexpr size_t kScrPartBytes = sizeof(float) * kIcpSums * kStaticParts;
constexpr size_t kScratchBytes = (kScrPartBytes + kTrackStateBytes + 255) / 256 * 256;
static_assert(kScrPartBytes % 8 == 0, "the pose must stay 8-byte aligned");

// Each GPU the library runs on holds its own copy until the process ends; in
// host code the name is not a device address, so it is only ever reached through
// the per-device address from hipGetSymbolAddress below.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// the current device's scratch address, looked up once per device
itm_status static_scratch(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ITM_ERR_ARG, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(ITM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return ITM_OK;
}

}  // namespace

extern "C" {

itm_status itm_track_noalloc(itm_scene *sc, const float *depth, const itm_intrinsics *K, const float *ref_pts,
                             const float *ref_normals, const double *T_ref, const double *T_init,
                             const itm_track_params *params, double *T_out, itm_track_info *info)
{
    if (itm_status st = track_check(sc, depth, K, ref_pts, ref_normals, T_ref, T_init)) return st;
    // the scene's stream must run on the current device, whose copy of the array is used
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != sc->device)
        return fail(ITM_ERR_ARG, "the scene lives on device %d but device %d is current", sc->device, dev);
    if (sc->num_cu > kStaticParts)
        return fail(ITM_ERR_ARG, "%d compute units need more workgroup partials than the %d of the static scratch",
                    sc->num_cu, kStaticParts);
    void *base = nullptr;
    if (itm_status st = static_scratch(&base)) return st;
    TrackBufs b;
    b.part = reinterpret_cast<float *>(base);
    b.cap = sc->num_cu;   // the grid of itm_track, so both give the same sums bit for bit
    b.pose = reinterpret_cast<double *>(static_cast<unsigned char *>(base) + kScrPartBytes);
    b.flags = reinterpret_cast<int32_t *>(b.pose + 48);
    return track_run(sc, b, depth, K, ref_pts, ref_normals, T_ref, T_init, params, T_out, info);
}
}  // extern "C"

// ---------------------------------------------------------------------------
// learned refiner
// ---------------------------------------------------------------------------
static void refiner_free(itm_refiner *r)
{
    if (!r) return;
    (void)hipStreamSynchronize(r->stream);
    for (void *p : {(void *)r->master, (void *)r->m, (void *)r->v, (void *)r->grad, (void *)r->loss,
                    (void *)r->bias, (void *)r->Wf, (void *)r->Wt, (void *)r->grad_part, (void *)r->loss_part})
        (void)hipFree(p);
    delete r;
}

itm_refiner *itm_refiner_create(const float *params, void *hip_stream)
{
    if (!params) {
        fail(ITM_ERR_ARG, "NULL parameter vector");
        return nullptr;
    }
    itm_refiner *r = new (std::nothrow) itm_refiner();
    if (!r) {
        fail(ITM_ERR_OOM, "host allocation failed");
        return nullptr;
    }
    r->stream = (hipStream_t)hip_stream;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        fail(ITM_ERR_HIP, "no HIP device");
        refiner_free(r);
        return nullptr;
    }
    r->num_cu = prop.multiProcessorCount;
    const size_t P = sizeof(float) * kRefineParams;
    if (dev_alloc((void **)&r->master, P, "refiner master") || dev_alloc((void **)&r->m, P, "adam m") ||
        dev_alloc((void **)&r->v, P, "adam v") || dev_alloc((void **)&r->grad, P, "gradient") ||
        dev_alloc((void **)&r->loss, sizeof(float), "loss") ||
        dev_alloc((void **)&r->bias, sizeof(float) * 4 * 16, "bias") ||
        dev_alloc((void **)&r->Wf, sizeof(uint16_t) * kRefineWeights, "bf16 weights") ||
        dev_alloc((void **)&r->Wt, sizeof(uint16_t) * kRefineWeights, "bf16 weights^T")) {
        refiner_free(r);
        return nullptr;
    }
    hipError_t e = hipMemcpyAsync(r->master, params, P, hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess) e = hipMemsetAsync(r->m, 0, P, r->stream);
    if (e == hipSuccess) e = hipMemsetAsync(r->v, 0, P, r->stream);
    if (e == hipSuccess) e = launch_refine_cast(r->master, r->Wf, r->Wt, r->bias, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) {
        fail(ITM_ERR_HIP, "refiner initialisation failed: %s", hipGetErrorString(e));
        refiner_free(r);
        return nullptr;
    }
    return r;
}

void itm_refiner_destroy(itm_refiner *r) { refiner_free(r); }

itm_status itm_refiner_set_stream(itm_refiner *r, void *hip_stream)
{
    if (!r) return fail(ITM_ERR_ARG, "NULL refiner");
    r->stream = (hipStream_t)hip_stream;
    return ITM_OK;
}

itm_status itm_refiner_get_params(itm_refiner *r, float *params)
{
    if (!r || !params) return fail(ITM_ERR_ARG, "NULL argument");
    HIP_TRY(hipMemcpyAsync(params, r->master, sizeof(float) * kRefineParams, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return ITM_OK;
}

static RefineParams refiner_params(const itm_refiner *r)
{
    RefineParams P;
    P.Wf = r->Wf;
    P.Wt = r->Wt;
    P.bias = r->bias;
    return P;
}

itm_status itm_refiner_forward(itm_refiner *r, const float *in, int64_t n, float *out)
{
    if (!r || (n > 0 && (!in || !out)) || n < 0) return fail(ITM_ERR_ARG, "bad refiner forward arguments");
    if (n == 0) return ITM_OK;
    RefineArgs a = {};
    a.P = refiner_params(r);
    a.in = in;
    a.n = n;
    a.out = out;
    HIP_TRY(launch_refine(a, false, (int)std::min<int64_t>(n, (int64_t)r->num_cu * 3), r->stream));
    return ITM_OK;
}

// the mean gradient into grad and the loss into loss (device pointers), with
// one Adam step in the same launch where adam is given
static itm_status refiner_grad(itm_refiner *r, const float *in, const float *target, const uint8_t *mask,
                               int64_t n, float *grad, float *loss, const AdamStep *adam)
{
    if (!r || n <= 0 || !in || !target || !mask) return fail(ITM_ERR_ARG, "bad refiner gradient arguments");
    if (n > r->part_cap) {
        HIP_TRY(hipStreamSynchronize(r->stream));
        (void)hipFree(r->grad_part);
        (void)hipFree(r->loss_part);
        r->grad_part = nullptr;
        r->loss_part = nullptr;
        r->part_cap = 0;
        if (dev_alloc((void **)&r->grad_part, sizeof(float) * kRefineParams * (size_t)n, "gradient partials") ||
            dev_alloc((void **)&r->loss_part, sizeof(float) * 2 * (size_t)n, "loss partials"))
            return ITM_ERR_OOM;
        r->part_cap = n;
    }
    RefineArgs a = {};
    a.P = refiner_params(r);
    a.in = in;
    a.n = n;
    a.target = target;
    a.mask = mask;
    a.grad_part = r->grad_part;
    a.loss_part = r->loss_part;
    HIP_TRY(launch_refine(a, true, (int)std::min<int64_t>(n, (int64_t)r->num_cu * 2), r->stream));
    HIP_TRY(launch_refine_reduce(r->grad_part, r->loss_part, n, grad, loss, adam, r->stream));
    return ITM_OK;
}

itm_status itm_refiner_gradient(itm_refiner *r, const float *in, const float *target, const uint8_t *mask,
                                int64_t n, float *grad, float *loss)
{
    return refiner_grad(r, in, target, mask, n, grad ? grad : r->grad, loss ? loss : r->loss, nullptr);
}

itm_status itm_refiner_train_step(itm_refiner *r, const float *in, const float *target, const uint8_t *mask,
                                  int64_t n, float lr, float *loss)
{
    if (!(lr > 0)) return fail(ITM_ERR_ARG, "learning rate must be > 0");
    AdamStep ad;
    ad.master = r->master;
    ad.m = r->m;
    ad.v = r->v;
    ad.Wf = r->Wf;
    ad.Wt = r->Wt;
    ad.bias = r->bias;
    ad.lr = lr;
    ad.step = r->step + 1;
    if (itm_status st = refiner_grad(r, in, target, mask, n, r->grad, loss ? loss : r->loss, &ad)) return st;
    r->step++;
    return ITM_OK;
}

itm_status itm_gather_blocks(itm_scene *sc, const int32_t *coords, int64_t n, float *out)
{
    if (!sc || n < 0 || (n > 0 && (!coords || !out))) return fail(ITM_ERR_ARG, "bad gather arguments");
    HIP_TRY(launch_refine_gather(sc->fmt, hash_view(sc), sc->sdf, sc->w, coords, n, 1.0f / (float)sc->max_w, out,
                                 sc->stream));
    return ITM_OK;
}

itm_status itm_scene_set_refiner(itm_scene *sc, itm_refiner *r, float w_threshold)
{
    if (!sc) return fail(ITM_ERR_ARG, "NULL scene");
    if (r && !(w_threshold > 0)) return fail(ITM_ERR_ARG, "weight threshold must be > 0");
    if (r && sc->swap) return fail(ITM_ERR_STATE, "a refiner does not combine with swapping");
    if (r && !sc->refined) {
        if (dev_alloc((void **)&sc->refined, sizeof(__half) * kBlockVox * (size_t)sc->vba_cap, "refined F") ||
            dev_alloc((void **)&sc->stamp, sizeof(int32_t) * (size_t)sc->vba_cap, "refine stamps"))
            return ITM_ERR_OOM;
        HIP_TRY(hipMemsetAsync(sc->stamp, 0, sizeof(int32_t) * (size_t)sc->vba_cap, sc->stream));
    }
    sc->refiner = r;
    sc->refine_w_threshold = w_threshold;
    return ITM_OK;
}

itm_status itm_refine_visible(itm_scene *sc)
{
    if (!sc) return fail(ITM_ERR_ARG, "NULL scene");
    if (!sc->refiner) return fail(ITM_ERR_STATE, "no refiner attached (itm_scene_set_refiner)");
    if (sc->frame == 0) return fail(ITM_ERR_STATE, "no frame integrated or loaded yet");
    return refine_visible(sc);
}

itm_status itm_export_blocks_refined(itm_scene *sc, int32_t *coords, float *sdf, uint8_t *refined,
                                     int64_t capacity, int64_t *n_blocks)
{
    if (!sc || !n_blocks) return fail(ITM_ERR_ARG, "NULL scene or n_blocks");
    if (itm_status st = itm_export_blocks(sc, coords, sdf, nullptr, capacity, n_blocks)) return st;
    if (!coords || !sdf || !sc->refined || *n_blocks == 0) {
        if (refined && coords) std::memset(refined, 0, (size_t)*n_blocks);
        return ITM_OK;
    }
    // voxel blocks of the exported (sorted) blocks
    std::vector<BlockRec> recs;
    if (itm_status st = collect_blocks(sc, recs)) return st;
    std::vector<int32_t> stamps(sc->vba_cap);
    HIP_TRY(hipMemcpyAsync(stamps.data(), sc->stamp, sizeof(int32_t) * sc->vba_cap, hipMemcpyDeviceToHost,
                           sc->stream));
    HIP_TRY(hipStreamSynchronize(sc->stream));
    std::vector<__half> blk(kBlockVox);
    for (int64_t i = 0; i < *n_blocks; i++) {
        const int32_t p = recs[i].blk;
        const bool r = p >= 0 && stamps[p] == sc->frame && sc->frame > 0;
        if (refined) refined[i] = r ? 1 : 0;
        if (!r) continue;
        HIP_TRY(hipMemcpy(blk.data(), sc->refined + (size_t)p * kBlockVox, sizeof(__half) * kBlockVox,
                          hipMemcpyDeviceToHost));
        for (int l = 0; l < kBlockVox; l++) sdf[i * kBlockVox + l] = __half2float(blk[l]);
    }
    return ITM_OK;
}

}  // extern "C"
