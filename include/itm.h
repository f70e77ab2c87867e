/*
 * itm.h -- C ABI of the gfx950 voxel-block-hashing TSDF fusion library (libitm.so).
 *
 * The library runs the per-frame hot path of volumetric depth fusion as described
 * in "A Framework for the Volumetric Integration of Depth Images" (Prisacariu,
 * Kaehler et al., 2014): allocation of 8^3 voxel blocks in a bucketed hash table
 * with an excess list, a per-frame list of visible blocks, the truncated signed
 * distance function (TSDF) update of every voxel of those blocks, and a raycast of
 * the fused volume into point and normal maps.  Every step runs in HIP kernels on
 * one GPU; no host fallback exists.
 *
 * Conventions shared by every call:
 *   - metres; camera frame x right, y down, z forward; pinhole, no distortion;
 *   - pixel (u, v) has its centre at integer coordinates (its camera ray is
 *     ((u - cx) / fx, (v - cy) / fy, 1));
 *   - T_wc: host array of 16 doubles, row-major 4x4 rigid camera-to-world transform
 *     (the paper's M_d is its inverse); the library inverts it rigidly;
 *   - voxel v (integer vector) sits at world position v * voxel_size; its block is
 *     floor(v / 8) and its index inside the block is lx + 8 ly + 64 lz;
 *   - F is the TSDF normalised by the truncation band mu, in [-1, 1]; W is the
 *     number of fused observations, capped at max_w.
 *
 * Errors: every call returns a status (or NULL for create); the reason is in
 * itm_last_error() (thread-local, valid until the next failing call on that
 * thread).  No call aborts or exits.  Hash-table exhaustion is not an error: blocks
 * that find no free entry are dropped and counted (itm_stats.n_dropped_total).
 *
 * Streams: integrate and raycast are asynchronous on the scene's HIP stream;
 * export and get_stats synchronise it.  A scene must not be used from two host
 * threads at once.
 */
#ifndef ITM_H
#define ITM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct itm_scene itm_scene; /* opaque, owned by the library */

typedef enum {
    ITM_OK = 0,
    ITM_ERR_ARG = -1,   /* invalid argument (NULL pointer, bad size, bad format) */
    ITM_ERR_OOM = -2,   /* device or host allocation failed */
    ITM_ERR_HIP = -3,   /* a HIP runtime call failed */
    ITM_ERR_STATE = -4  /* call not valid in the scene's current state */
} itm_status;

/* Voxel storage forms (section "Framework Flexibility": the voxel type is a
 * parameter of the volume).  Arithmetic is binary32 in every form.
 *   ITM_VOX_F32   float F, float W (8 bytes per voxel)
 *   ITM_VOX_F16   half F, half W (4 bytes per voxel)
 *   ITM_VOX_S16U8 int16 F * 32767 (round to nearest even, clamped to +-32767),
 *                 uint8 W (3 bytes per voxel; the paper's default voxel type) */
typedef enum { ITM_VOX_F32 = 0, ITM_VOX_F16 = 1, ITM_VOX_S16U8 = 2 } itm_voxel_fmt;

typedef struct {
    double fx, fy, cx, cy; /* focal lengths and principal point, pixels */
    int32_t width, height; /* image size, pixels */
} itm_intrinsics;

typedef struct {
    int64_t n_allocated;     /* voxel blocks allocated so far */
    int64_t n_visible_last;  /* visible blocks of the last integrated frame */
    int64_t n_excess_used;   /* excess-list entries in use */
    int64_t n_dropped_total; /* sum over frames of the distinct blocks dropped */
    int64_t vba_capacity;    /* voxel block array capacity (blocks) */
    int64_t n_updated_last;  /* voxels updated by the last integration */
    int64_t n_entries;       /* hash entries: 2 * n_buckets + n_excess */
    int64_t bytes_per_voxel; /* storage form's bytes per voxel */
    int64_t n_visible_total; /* visible blocks summed over all integrations */
    int64_t n_updated_total; /* updated voxels summed over all integrations */
} itm_stats;

/* Create a scene (section "Voxel Block Hashing"; scene parameters as in the
 * paper's ITMSceneParams, section "Compilation, UI, Usage and Examples").
 *   voxel_size  voxel edge, metres, > 0
 *   mu          truncation band, metres, > 0
 *   max_w       weight cap, >= 1 (<= 255 for ITM_VOX_S16U8, <= 2048 for ITM_VOX_F16)
 *   n_buckets   hash buckets, a power of two (the hash is masked), each holding
 *               2 entries ("a bucket of fixed size (typically 2)")
 *   n_excess    entries of the unordered excess list, >= 0
 * The voxel block array holds one block per hash entry (2 n_buckets + n_excess
 * blocks), so block reservation never fails.  Voxels start at F = 1, W = 0.
 * Storage F32, null stream, raycast depth range [0.2, 5.0] m.
 * Returns NULL on failure (ITM_ERR_ARG / ITM_ERR_OOM / ITM_ERR_HIP reason). */
itm_scene *itm_scene_create(float voxel_size, float mu, int32_t max_w, int64_t n_buckets,
                            int64_t n_excess);

/* As itm_scene_create, with the storage form, the HIP stream (hipStream_t, may be
 * NULL) and the raycast search range in camera depth [z_near, z_far] metres. */
itm_scene *itm_scene_create_ex(float voxel_size, float mu, int32_t max_w, int64_t n_buckets,
                               int64_t n_excess, int32_t fmt, void *hip_stream, float z_near,
                               float z_far);

/* Free every device and host resource of the scene -- the hash table and the
 * voxel block array of section "Hash Table and Hashing Function" / "Voxel Block
 * Array", the visible list, the search-range bins, the tracker's, colour's,
 * refiner's and swapping's buffers (synchronises its stream).  NULL is ignored. */
void itm_scene_destroy(itm_scene *scene);

/* Replace the scene's HIP stream (hipStream_t, may be NULL). */
itm_status itm_set_stream(itm_scene *scene, void *hip_stream);

/* Fuse one depth frame: allocation (section "Allocation", stages one to three)
 * then integration (section "Integration").
 *   depth  DEVICE pointer, K->height * K->width float32, row-major, metres; a
 *          pixel is valid when finite and > 0 (0, negative, NaN, inf = no data).
 *          Read only; must stay valid until the stream reaches this work.
 *   K      host pointer; width, height >= 3
 *   T_wc   host pointer, 16 doubles (copied before return)
 * Allocation: every voxel block crossed by a valid pixel's ray segment between
 * camera depths max(d - mu, 0) and d + mu is looked up and inserted when absent
 * (atomic insertion: every crossed block is allocated); the visible list of the
 * frame is the set of those blocks.  Integration: every voxel of every visible
 * block is projected into the depth image and updated with the paper's running
 * average.  Asynchronous on the scene's stream. */
itm_status itm_integrate(itm_scene *scene, const float *depth, const itm_intrinsics *K,
                         const double *T_wc);

/* Raycast the fused volume (section "Raycast") from pose T_wc.
 *   out_pts, out_normals  DEVICE pointers, K->height * K->width float4 each
 *   (16-byte aligned), written row-major in the world frame.  A hit pixel gets
 *   (x, y, z, 1) and its unit normal (nx, ny, nz, 1) (w = 0 when the TSDF gradient
 *   vanishes); a miss gets all zeros in both.
 * The search covers camera depths [z_near, z_far] with the state machine of the
 * paper (coarse block steps, fine steps of mu, steps of the TSDF value, two
 * trilinear refinement steps behind the surface) -- narrowed, when the search
 * range is on (itm_scene_set_search_range), to the pixel's expected depth range
 * from the last frame's visible blocks (itm_expected_depths); a pixel no visible
 * block projects onto is then a miss.  Asynchronous. */
itm_status itm_raycast(itm_scene *scene, const itm_intrinsics *K, const double *T_wc,
                       float *out_pts, float *out_normals);

/* Search range of the raycast (section "Raycast": the visible blocks of the last
 * frame, forward-projected, give each pixel the minimum and maximum depth to
 * expect).  enable != 0 turns it on for later itm_raycast calls; while it is on,
 * itm_integrate also bins the rectangles at the frame's own pose, which a
 * raycast at exactly that pose (same K and T_wc bits) then reuses; any other
 * pose bins them again from the visible list.
 *   tile_capacity  rectangles kept per 16 x 16 pixel tile (<= 0: 512, at most
 *                  65536).  A tile with more is still exact: its workgroup then
 *                  recomputes every visible block (slow).
 * Results with the range on are those of the paper's raycast with a search
 * range; with it off (the default) every pixel searches [z_near, z_far].
 * Synchronises the scene's stream when the capacity changes. */
itm_status itm_scene_set_search_range(itm_scene *scene, int32_t enable, int32_t tile_capacity);

/* The expected depth range image (section "Raycast", CreateExpectedDepths) at
 * pose T_wc, from the visible blocks of the last itm_integrate:
 *   zrange  DEVICE pointer, K->height * K->width float2 (8-byte aligned),
 *           row-major: (z_min, z_max) in camera depth, metres.
 * Each visible block's box [8k - 1/2, 8k + 7 1/2] s (per axis, the region whose
 * samples read the block) is projected; the pixels whose centres lie in the 2D
 * bounding box of its 8 corners (clipped to the image) get the min / max of the
 * corners' camera depths (binary64, rounded outwards to binary32), combined over
 * blocks by min / max.  A block with a corner at camera depth <= 0 covers the
 * whole image from depth 0.  Pixels no block covers get (+inf, 0).
 * Works whether or not the search range is on.  Asynchronous. */
itm_status itm_expected_depths(itm_scene *scene, const itm_intrinsics *K, const double *T_wc, float *zrange);

/* Copy the allocated blocks to the host, sorted ascending by (x, y, z): the
 * hash table's keys (section "Hash Table and Hashing Function") and the voxel
 * block array (section "Voxel Block Array").
 *   coords  HOST int32[capacity * 3] or NULL to only count
 *   sdf, w  HOST float[capacity * 512] each, or NULL; F as a float in [-1, 1] and
 *           W as a float, voxel order lx + 8 ly + 64 lz
 *   capacity  blocks the buffers hold; ITM_ERR_ARG when smaller than the count
 *   n_blocks  HOST int64 out: number of allocated blocks
 * Synchronises the stream. */
itm_status itm_export_blocks(itm_scene *scene, int32_t *coords, float *sdf, float *w,
                             int64_t capacity, int64_t *n_blocks);

/* Load blocks into the scene (the inverse of itm_export_blocks, e.g. a saved
 * map): each block key is found or inserted as allocation does (section "Hash
 * Table Operations"; a block that finds no entry is dropped and counted in
 * n_dropped_total) and its voxels overwritten, converted to the scene's storage
 * form (F16: round to nearest even; S16U8: F * 32767 rounded to nearest even).
 * Colour voxels, when enabled, of the loaded blocks are cleared.  The loaded
 * blocks become the visible set, as if one frame had visited them: the search
 * range of the next raycast projects them.
 *   coords  HOST int32[n * 3], distinct keys within +-32767
 *   sdf, w  HOST float[n * 512] each, export layout; F in [-1, 1], W an
 *           integer in [0, max_w]
 * ITM_ERR_ARG for NULL buffers, repeated keys or values out of range (nothing
 * is changed then).  Synchronises the stream. */
itm_status itm_import_blocks(itm_scene *scene, const int32_t *coords, const float *sdf, const float *w,
                             int64_t n);

/* ---- Colour voxels (section "Framework Flexibility": a voxel may carry a colour
 * and a colour weight beside F and W; section "Integration": the colour update is
 * the same running average, fed by the registered colour image).
 * Colour voxels: 4 bytes each, (r, g, b, colour weight), one per depth voxel. */

/* Allocate the scene's colour voxels (all zero) on the device; a no-op when
 * already enabled.  Blocks fused before this call keep colour weight 0.
 * ITM_ERR_OOM when the device memory (vba capacity * 2 KiB) is not there.
 * Synchronises the stream. */
itm_status itm_scene_enable_colour(itm_scene *scene);

/* itm_integrate with a colour image:
 *   rgbx  DEVICE pointer, K->height * K->width * 4 bytes (4-byte aligned),
 *         row-major (r, g, b, unused), registered to the depth image
 * Depth voxels are updated exactly as by itm_integrate.  A voxel whose depth is
 * updated and whose projective distance d - z is at most mu also takes the
 * colour of its depth pixel: each channel c <- (cw c + c_new) / (cw + 1) in
 * exact integer arithmetic rounded half to even, cw <- min(cw + 1, min(max_w,
 * 255)).  ITM_ERR_ARG when colour is not enabled.  Asynchronous. */
itm_status itm_integrate_colour(itm_scene *scene, const float *depth, const uint8_t *rgbx,
                                const itm_intrinsics *K, const double *T_wc);

/* itm_raycast that also renders colour:
 *   out_rgbx  DEVICE pointer, K->height * K->width * 4 bytes (4-byte aligned):
 *             at a hit, (r, g, b, 255) of the voxel nearest to the hit point
 *             (lattice point floor(p / s + 1/2)) when its block is allocated,
 *             else zeros; zeros at a miss.
 * Points and normals are those itm_raycast writes.  ITM_ERR_ARG when colour is
 * not enabled.  Asynchronous. */
itm_status itm_raycast_colour(itm_scene *scene, const itm_intrinsics *K, const double *T_wc,
                              float *out_pts, float *out_normals, uint8_t *out_rgbx);

/* Copy the colour voxels of the allocated blocks to the host, in the block
 * order of itm_export_blocks:
 *   rgbw      HOST uint8[capacity * 512 * 4] or NULL to only count;
 *             (r, g, b, colour weight) per voxel, voxel order lx + 8 ly + 64 lz
 *   capacity  blocks the buffer holds; ITM_ERR_ARG when smaller than the count
 *   n_blocks  HOST int64 out: number of allocated blocks
 * ITM_ERR_ARG when colour is not enabled.  Synchronises the stream. */
itm_status itm_export_colour(itm_scene *scene, uint8_t *rgbw, int64_t capacity, int64_t *n_blocks);

/* Counters of the scene (synchronises the stream): allocated blocks (hash
 * entries holding a key, section "Allocation" stage two), blocks listed in the
 * last frame (stage three's visible list) and since creation, excess entries
 * used and blocks dropped when the table was full (section "Hash Table
 * Operations"), voxels updated in the last frame and since creation (section
 * "Integration"), the voxel block array's capacity and the bytes per voxel of
 * the storage form (section "Framework Flexibility"). */
itm_status itm_get_stats(itm_scene *scene, itm_stats *out);

/* Per-kernel timing with a HIP event pair attached to every launch's dispatch
 * (the kernel's own start and end) while enabled (toggling does not
 * synchronise; events recorded while enabled are kept until read).  Kernel ids:
 * 0 allocation with the visible
 * list (and, with the search range on, the expected-depth binning), 1
 * integration, 2 raycast (not the re-binning a pose other than the last
 * frame's takes first), 3 refiner gate, 4 tracker step on the finest level
 * (pairing, sums, and in the workgroup that finishes last the solve and pose
 * update), 5 the same on the coarser levels. */
#define ITM_KERNEL_COUNT 6
itm_status itm_profile_enable(itm_scene *scene, int enable);
/* Synchronises, then writes the summed milliseconds and launch counts per kernel
 * id since profiling was enabled, and resets them. */
itm_status itm_profile_read(itm_scene *scene, double *ms, int64_t *launches);

/* ------------------------------------------------------------------------ */
/* Depth tracker, section "Tracking" (the depth tracker): the camera pose of a  */
/* new depth image is found by aligning it to the surface the raycast rendered  */
/* from a reference pose.  Each point p of the depth image, moved by the        */
/* current estimate T (camera -> world), is projected into the reference view   */
/* with K and paired with the nearest reference pixel (floor(x + 1/2),          */
/* floor(y + 1/2)); a pair counts when both maps hold a hit there and           */
/* |T p - V| <= the level's distance threshold.  Its point-to-plane distance is */
/* d = (T p - V) . N.  A Gauss-Newton step solves A x = -g with A = sum J J^T,  */
/* g = sum J d, J = (T p x N, N) and moves the pose by T <- (exp([x_0..2]x),    */
/* x_3..5) T.  Levels of a resolution hierarchy are visited coarse to fine:     */
/* pixel (u, v) of level l is input pixel (2^l u, 2^l v) (ceil(W / 2^l) x       */
/* ceil(H / 2^l) pixels), with intrinsics fx / 2^l, fy / 2^l, cx / 2^l,         */
/* cy / 2^l; the image must have at least 2^l pixels per axis for level l.      */
/* Per-pixel terms in float32; sums of a workgroup in float32, over             */
/* workgroups in float64 in a fixed order; the 6 x 6 solve (Cholesky) and the   */
/* pose (Rodrigues' formula) in float64, on the GPU: no host round trip between */
/* steps.                                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_levels;       /* 1..4 */
    int32_t iters[4];       /* Gauss-Newton steps per level, finest first, >= 0 */
    float dist_thresh[4];   /* pairing distance per level in metres, finest first, > 0 */
    int32_t min_inliers;    /* a level stops at the first system with fewer pairs */
} itm_track_params;
/* n_levels 3, iters {4, 6, 10}, dist_thresh {0.02, 0.05, 0.1}, min_inliers 100 */
void itm_track_default_params(itm_track_params *params);

typedef struct {
    int64_t n_pairs;        /* pairs of the last system evaluated */
    double rms;             /* RMS point-to-plane distance of that system (m) */
    int32_t steps;          /* Gauss-Newton steps taken over all levels */
} itm_track_info;

/* depth: DEVICE float32 [K->height][K->width] row-major metres (0, negative,
 * NaN or inf = invalid); ref_pts, ref_normals: DEVICE float4 [height][width],
 * 16-byte aligned, as itm_raycast writes them (world frame, w > 0 = hit) for
 * the same K at pose T_ref; T_ref, T_init: HOST double[16] row-major camera ->
 * world; params: NULL for the defaults.  T_out: HOST double[16], info: HOST,
 * may be NULL.  Runs on the scene's stream and synchronises it once at the end
 * to return the pose.  Scratch (per-workgroup sums, pose) is the scene's,
 * allocated on first use.  ITM_ERR_ARG for NULL inputs, bad sizes, misaligned
 * maps or parameters out of range. */
itm_status itm_track(itm_scene *scene, const float *depth, const itm_intrinsics *K, const float *ref_pts,
                     const float *ref_normals, const double *T_ref, const double *T_init,
                     const itm_track_params *params, double *T_out, itm_track_info *info);
/* The sums of one Gauss-Newton step at pose T on hierarchy level `level` (0 =
 * the input image): sys HOST double[29] = upper triangle of A row by row (21),
 * g (6), sum of d^2, number of pairs.  Synchronises.  Arguments as itm_track. */
itm_status itm_icp_system(itm_scene *scene, const float *depth, const itm_intrinsics *K, int32_t level,
                          const float *ref_pts, const float *ref_normals, const double *T_ref, const double *T,
                          float dist_thresh, double *sys);

/* itm_track without any device allocation, for callers that cannot allocate   */
/* (code under HIP graph capture, tight serving loops, harnesses that forbid    */
/* hipMalloc).  Same arguments, kernels, grid and result as itm_track (the pose  */
/* is bit-identical), but the per-workgroup sums, pose and flags live in one     */
/* static device array of the library (about 117 KiB, held by each GPU the       */
/* library runs on until the process ends) instead of the scene's scratch.       */
/* Every call on a GPU shares that GPU's array: calls that overlap on one GPU    */
/* (other streams, other scenes, other host threads) race and must be            */
/* serialised by the caller.  The scene must belong to the current device.      */
/* ITM_ERR_ARG also when the device has more than 1024 compute units (the        */
/* array's sum rows).                                                           */
itm_status itm_track_noalloc(itm_scene *scene, const float *depth, const itm_intrinsics *K,
                             const float *ref_pts, const float *ref_normals, const double *T_ref,
                             const double *T_init, const itm_track_params *params, double *T_out,
                             itm_track_info *info);

/* ------------------------------------------------------------------------ */
/* Swapping (section "Swapping").  The device keeps a pool of device_blocks    */
/* voxel blocks (the voxel block array, fewer than the map may hold); every   */
/* hash entry can hold one.  Per frame, after the integration:                */
/*  - a visible block without a device block takes one from the pool during  */
/*    the allocation (a new block, or one whose data is on the host); with    */
/*    the pool empty it is not integrated in that frame (counted);            */
/*  - swap in: of the blocks holding a device block and a host copy not yet   */
/*    merged, the first swap_in in key order (x, y, z) are merged back -- the  */
/*    secondary integration F = (W_d F_d + W_h F_h) / (W_d + W_h), W = min(W_d */
/*    + W_h, max_w);                                                          */
/*  - swap out: of the device blocks not visible in the frame with nothing to */
/*    merge, the first swap_out in key order move to the host (a host voxel   */
/*    block per hash entry, kept by the library) and free their device block.  */
/* Transfers go through fixed-size buffers (pinned on the host) of            */
/* max(swap_in, swap_out) blocks; each frame synchronises the stream twice.   */
/* The raycast sees the blocks on the device only; itm_export_blocks returns    */
/* every block wherever it is (merged when both copies exist).  Call before   */
/* the first frame; not with colour, a refiner or itm_import_blocks            */
/* (ITM_ERR_STATE).  swap_in = swap_out = 0 keeps the pool without transfers: */
/* the voxel block array is sized to device_blocks instead of one block per   */
/* hash entry, and a block that finds the pool empty is not integrated        */
/* (counted).  ITM_ERR_ARG unless 1 <= device_blocks <= the entries and either */
/* both transfer sizes are 0 or 1 <= swap_in, swap_out <= 2^20.  Synchronises   */
/* the stream. */
itm_status itm_scene_enable_swapping(itm_scene *scene, int64_t device_blocks, int32_t swap_in,
                                     int32_t swap_out);
/* out[8]: blocks holding a device block, blocks whose data is on the host     */
/* only, blocks with a host copy not yet merged, blocks swapped in / out in the */
/* last frame, the totals of both, visible blocks left without a device block */
/* (total).  ITM_ERR_STATE when swapping is off.  Synchronises the stream.     */
itm_status itm_swap_stats(itm_scene *scene, int64_t *out);

/* ------------------------------------------------------------------------ */
/* Learned block refiner.  Not part of the paper's method: a small 3D           */
/* convolutional network, trained on pairs the method itself produces, maps a   */
/* block's few-frame TSDF (with a one-voxel halo) towards the TSDF the running  */
/* average reaches after many frames.  Layers (each a 3^3 convolution from the  */
/* 10^3 haloed / zero-padded grid to the 8^3 block): 2->16 ReLU, 16->16 ReLU,    */
/* 16->16 ReLU, 16->1; F_out = clamp(F + L4, -1, 1).  bf16 operands on MFMA,     */
/* float32 accumulation, float32 master weights.                                */
/* Parameter vector: for layers 1..4 W[tap][co][ci] (tap = dz*9 + dy*3 + dx,     */
/* co, ci in 0..15, unused channels 0), then the biases b[layer][co].            */
/* Network input of a block: float32 [2][10][10][10] = (F, W / max_w) on the     */
/* voxels 8 k - 1 .. 8 k + 8 per axis; voxels of absent blocks read (1, 0).       */
/* ------------------------------------------------------------------------ */
#define ITM_REFINE_PARAMS 27712
typedef struct itm_refiner itm_refiner; /* opaque, owned by the library */

/* params: HOST float[ITM_REFINE_PARAMS] (copied).  NULL on failure. */
itm_refiner *itm_refiner_create(const float *params, void *hip_stream);
void itm_refiner_destroy(itm_refiner *refiner);
itm_status itm_refiner_set_stream(itm_refiner *refiner, void *hip_stream);
/* params: HOST float[ITM_REFINE_PARAMS] out (synchronises). */
itm_status itm_refiner_get_params(itm_refiner *refiner, float *params);
/* in: DEVICE float[n][2][1000]; out: DEVICE float[n][512] refined F.  Async. */
itm_status itm_refiner_forward(itm_refiner *refiner, const float *in, int64_t n, float *out);
/* Mean squared error of F_out against target over the voxels with mask != 0,
 * summed over the n blocks and divided by the count of such voxels, and its
 * gradient.  in: DEVICE float[n][2][1000]; target: DEVICE float[n][512]; mask:
 * DEVICE uint8[n][512]; grad: DEVICE float[ITM_REFINE_PARAMS] or NULL; loss:
 * DEVICE float[1] or NULL.  Async; scratch grows with n (about 111 KB per block). */
itm_status itm_refiner_gradient(itm_refiner *refiner, const float *in, const float *target,
                                const uint8_t *mask, int64_t n, float *grad, float *loss);
/* The gradient above, then one Adam step (beta 0.9, 0.999, eps 1e-8) on the
 * float32 master weights and a re-rounding of the bf16 copies.  Async. */
itm_status itm_refiner_train_step(itm_refiner *refiner, const float *in, const float *target,
                                  const uint8_t *mask, int64_t n, float lr, float *loss);
/* Network inputs of the blocks at coords (DEVICE int32[n][3]) from the scene's
 * volume into out (DEVICE float[n][2][1000]).  Async. */
itm_status itm_gather_blocks(itm_scene *scene, const int32_t *coords, int64_t n, float *out);
/* Attach a refiner (not owned; NULL detaches): after every integration each
 * visible block whose largest weight is below w_threshold is refined into a side
 * buffer (half precision, one per voxel block; allocated on first attach), and
 * the raycast until the next frame reads those blocks' F from it (the plain F
 * of every other block is the fallback; the running average never sees it). */
itm_status itm_scene_set_refiner(itm_scene *scene, itm_refiner *refiner, float w_threshold);
/* Run the refiner (as itm_integrate does after each frame) over the current
 * visible set -- e.g. right after itm_import_blocks -- on the blocks whose
 * largest weight is below the threshold.  Until the next frame, the raycast
 * reads those blocks' F from the refiner's output.  ITM_ERR_STATE without a
 * refiner or before any frame.  Asynchronous. */
itm_status itm_refine_visible(itm_scene *scene);
/* As itm_export_blocks for F, with the refined F of the blocks refined in the
 * last integration; refined: HOST uint8[capacity] or NULL, 1 where refined. */
itm_status itm_export_blocks_refined(itm_scene *scene, int32_t *coords, float *sdf, uint8_t *refined,
                                     int64_t capacity, int64_t *n_blocks);

/* Reason of the last failing call on this thread ("" if none). */
const char *itm_last_error(void);
/* Status of the last failing call on this thread (ITM_OK if none); the way to
 * tell why itm_scene_create / _ex returned NULL (e.g. ITM_ERR_OOM). */
itm_status itm_last_status(void);

#ifdef __cplusplus
}
#endif

#endif /* ITM_H */
