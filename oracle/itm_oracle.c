/*
 * oracle/itm_oracle.c -- plain, slow, obviously-correct CPU implementation of the
 * per-frame volumetric fusion path of "A Framework for the Volumetric Integration
 * of Depth Images" (Prisacariu, Kaehler et al., 2014).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant generator with the
 * GPU library.
 *
 * Precision: values (camera-space depth difference, truncated SDF, running
 * average) are binary64.  Where floating point decides an integer -- which voxel
 * blocks a band segment crosses, which pixel a voxel projects to, whether a voxel
 * is skipped -- the decision is taken in binary32 along a fixed evaluation order,
 * which is the precision of the paper's own listings (float vectors and
 * matrices).  The fixed order is stated next to each decision below.
 *
 * Parts and the passages they follow:
 *   hashIndex ............................ section "Hash Table and Hashing Function"
 *   retrieval (bucket, then excess chain)  section "Hash Table Operations" (readVoxel)
 *   insertion (bucket slot, else append to
 *     the excess list, reserve a block) .. section "Hash Table Operations"
 *   allocation (band segment, blocks it
 *     crosses, visible flags) ............ section "Allocation", stages one to three
 *   voxel update ......................... section "Integration"
 *                                          (computeUpdatedVoxelDepthInfo)
 *   dense volume ......................... section "Dense Volumes"
 *   raycast state machine ................ section "Raycast"
 *   expected depth range per pixel ....... section "Raycast" (search range,
 *                                          CreateExpectedDepths)
 *   depth tracker (point-to-plane ICP over
 *     a resolution hierarchy) ............ section "Tracking" (ITMDepthTracker)
 *   colour voxels (RGB and a colour weight
 *     per voxel, fused with the depth) ... section "Framework Flexibility"
 *                                          (ITMVoxel_s_rgb) and "Integration" 
 * Readings where the paper is silent are noted beside the code that takes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SDF_BLOCK 8
#define SDF_BLOCK3 512
#define ENTRIES_PER_BUCKET 2 /* "a bucket of fixed size (typically 2)" */

/* ------------------------------------------------------------------------- */
/* hash entry: block position, excess-list offset (index + 1, 0 = end of list) */
/* and pointer into the voxel block array (>= 0 allocated, < -1 unallocated).  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int16_t x, y, z;
    int32_t offset;
    int32_t ptr;
} orc_entry;

typedef struct {
    double s;          /* voxel size, metres */
    float mu_f;        /* truncation band, binary32 as given */
    double mu;         /* same value, binary64 */
    int max_w;
    int64_t n_buckets, n_excess, n_entries;
    uint32_t mask;
    orc_entry *e;
    int64_t excess_used; /* prepopulated excess free list: next unused index */
    /* voxel block array, grown on demand; F in [-1,1] (binary64), W integer */
    double *F;
    int32_t *W;
    uint8_t *C;        /* colour (r, g, b, colour weight) per voxel, NULL until enabled */
    int64_t n_blocks, cap_blocks;
    /* per-frame visibility (one flag per hash entry) and statistics */
    uint8_t *vis;
    int64_t n_vis;
    int64_t dropped_total; /* sum over frames of the distinct blocks dropped */
    int32_t *drop_keys;    /* blocks dropped in the current frame (with repeats) */
    int64_t n_drop, cap_drop;
    int64_t updated_last;
    float z_near, z_far;
} orc_scene;

/* ------------------------------------------------------------------------- */
/* hashIndex: ((x * 73856093) ^ (y * 19349669) ^ (z * 83492791)) & mask,      */
/* each coordinate converted to unsigned 32-bit, products wrap modulo 2^32.    */
/* ------------------------------------------------------------------------- */
uint32_t orc_hash_index(int32_t x, int32_t y, int32_t z, uint32_t mask)
{
    uint32_t hx = (uint32_t)x * 73856093u;
    uint32_t hy = (uint32_t)y * 19349669u;
    uint32_t hz = (uint32_t)z * 83492791u;
    return (hx ^ hy ^ hz) & mask;
}

orc_scene *orc_scene_create(float voxel_size, float mu, int32_t max_w, int64_t n_buckets,
                            int64_t n_excess)
{
    if (!(voxel_size > 0) || !(mu > 0) || max_w < 1 || n_buckets < 1 || n_excess < 0)
        return NULL;
    if ((n_buckets & (n_buckets - 1)) != 0 || n_buckets > ((int64_t)1 << 30))
        return NULL;
    orc_scene *sc = (orc_scene *)calloc(1, sizeof(orc_scene));
    if (!sc) return NULL;
    sc->s = (double)voxel_size;
    sc->mu_f = mu;
    sc->mu = (double)mu;
    sc->max_w = max_w;
    sc->n_buckets = n_buckets;
    sc->n_excess = n_excess;
    sc->n_entries = ENTRIES_PER_BUCKET * n_buckets + n_excess;
    sc->mask = (uint32_t)(n_buckets - 1);
    sc->e = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)sc->n_entries);
    sc->vis = (uint8_t *)calloc((size_t)sc->n_entries, 1);
    if (!sc->e || !sc->vis) { free(sc->e); free(sc->vis); free(sc); return NULL; }
    for (int64_t i = 0; i < sc->n_entries; i++) {
        sc->e[i].x = sc->e[i].y = sc->e[i].z = 0;
        sc->e[i].offset = 0;
        sc->e[i].ptr = -2;
    }
    sc->z_near = 0.2f;
    sc->z_far = 5.0f;
    return sc;
}

void orc_scene_destroy(orc_scene *sc)
{
    if (!sc) return;
    free(sc->e); free(sc->vis); free(sc->F); free(sc->W); free(sc->C); free(sc->drop_keys); free(sc);
}

int orc_set_range(orc_scene *sc, float z_near, float z_far)
{
    if (!(z_near > 0) || !(z_far > z_near)) return -1;
    sc->z_near = z_near;
    sc->z_far = z_far;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* retrieval: look through the bucket, then follow the excess chain whose head */
/* offset is the one held by the bucket's last entry; an entry matches when    */
/* its position equals the block and its pointer is >= 0.                      */
/* ------------------------------------------------------------------------- */
int64_t orc_find(const orc_scene *sc, int32_t x, int32_t y, int32_t z)
{
    int64_t base = (int64_t)orc_hash_index(x, y, z, sc->mask) * ENTRIES_PER_BUCKET;
    int32_t off = 0;
    for (int i = 0; i < ENTRIES_PER_BUCKET; i++) {
        const orc_entry *h = &sc->e[base + i];
        off = h->offset - 1;
        if (h->x == x && h->y == y && h->z == z && h->ptr >= 0) return base + i;
    }
    while (off >= 0) {
        int64_t idx = ENTRIES_PER_BUCKET * sc->n_buckets + off;
        const orc_entry *h = &sc->e[idx];
        if (h->x == x && h->y == y && h->z == z && h->ptr >= 0) return idx;
        off = h->offset - 1;
    }
    return -1;
}

/* reserve the next block of the voxel block array (fresh voxels: F = 1, W = 0,
 * the initial value of the paper's voxel types) */
static int32_t orc_reserve_block(orc_scene *sc)
{
    if (sc->n_blocks == sc->cap_blocks) {
        int64_t nc = sc->cap_blocks ? sc->cap_blocks * 2 : 1024;
        double *F = (double *)realloc(sc->F, sizeof(double) * SDF_BLOCK3 * (size_t)nc);
        if (!F) return -2;
        sc->F = F;
        int32_t *W = (int32_t *)realloc(sc->W, sizeof(int32_t) * SDF_BLOCK3 * (size_t)nc);
        if (!W) return -2;
        sc->W = W;
        if (sc->C) {
            uint8_t *C = (uint8_t *)realloc(sc->C, 4 * SDF_BLOCK3 * (size_t)nc);
            if (!C) return -2;
            sc->C = C;
        }
        sc->cap_blocks = nc;
    }
    int64_t b = sc->n_blocks++;
    for (int i = 0; i < SDF_BLOCK3; i++) {
        sc->F[b * SDF_BLOCK3 + i] = 1.0;
        sc->W[b * SDF_BLOCK3 + i] = 0;
    }
    if (sc->C) memset(sc->C + 4 * b * SDF_BLOCK3, 0, 4 * SDF_BLOCK3);
    return (int32_t)b;
}

/* insertion: if the block is present return its entry; else take the first
 * unallocated entry of the bucket; else append a new entry from the excess
 * list and link it from the last entry of the chain.  Returns the entry index,
 * or -1 when the excess list is exhausted (the block is dropped and counted). */
int64_t orc_insert(orc_scene *sc, int32_t x, int32_t y, int32_t z)
{
    int64_t found = orc_find(sc, x, y, z);
    if (found >= 0) return found;
    int64_t base = (int64_t)orc_hash_index(x, y, z, sc->mask) * ENTRIES_PER_BUCKET;
    for (int i = 0; i < ENTRIES_PER_BUCKET; i++) {
        orc_entry *h = &sc->e[base + i];
        if (h->ptr < -1) {
            int32_t p = orc_reserve_block(sc);
            if (p < 0) return -1;
            h->x = (int16_t)x; h->y = (int16_t)y; h->z = (int16_t)z;
            h->ptr = p;
            return base + i;
        }
    }
    int64_t prev = base + ENTRIES_PER_BUCKET - 1;
    while (sc->e[prev].offset > 0) prev = ENTRIES_PER_BUCKET * sc->n_buckets + sc->e[prev].offset - 1;
    if (sc->excess_used >= sc->n_excess) {
        if (sc->n_drop == sc->cap_drop) {
            int64_t nc = sc->cap_drop ? 2 * sc->cap_drop : 1024;
            int32_t *nk = (int32_t *)realloc(sc->drop_keys, sizeof(int32_t) * 3 * (size_t)nc);
            if (!nk) return -1;
            sc->drop_keys = nk;
            sc->cap_drop = nc;
        }
        sc->drop_keys[3 * sc->n_drop] = x;
        sc->drop_keys[3 * sc->n_drop + 1] = y;
        sc->drop_keys[3 * sc->n_drop + 2] = z;
        sc->n_drop++;
        return -1;
    }
    int64_t xi = sc->excess_used++;
    int64_t idx = ENTRIES_PER_BUCKET * sc->n_buckets + xi;
    int32_t p = orc_reserve_block(sc);
    if (p < 0) return -1;
    orc_entry *h = &sc->e[idx];
    h->x = (int16_t)x; h->y = (int16_t)y; h->z = (int16_t)z;
    h->offset = 0;
    h->ptr = p;
    sc->e[prev].offset = (int32_t)(xi + 1);
    return idx;
}

/* ------------------------------------------------------------------------- */
/* blocks crossed by a segment, in block units (binary32 end points).          */
/* Fixed order: start at floor(P0); per axis the number of boundary crossings  */
/* is |floor(P1) - floor(P0)|; the parameter of the next crossing on axis a is */
/* t_a = (B_a - P0_a) / (P1_a - P0_a) in binary32, B_a the next integer plane   */
/* in the direction of travel, recomputed from B_a after every step; each step */
/* crosses the axis with the smallest t_a (ties: x, then y, then z).           */
/* Returns the number of blocks written (capped at cap, total always counted). */
/* ------------------------------------------------------------------------- */
int64_t orc_dda_blocks(const float *P0, const float *P1, int32_t *out, int64_t cap)
{
    int32_t b[3], n[3], st[3];
    float D[3], t[3];
    for (int a = 0; a < 3; a++) {
        int32_t b0 = (int32_t)floorf(P0[a]);
        int32_t b1 = (int32_t)floorf(P1[a]);
        b[a] = b0;
        n[a] = b1 > b0 ? b1 - b0 : b0 - b1;
        st[a] = b1 > b0 ? 1 : (b1 < b0 ? -1 : 0);
        D[a] = P1[a] - P0[a];
        if (n[a] > 0) {
            float B = (float)(b[a] + (st[a] > 0 ? 1 : 0));
            t[a] = (B - P0[a]) / D[a];
        } else {
            t[a] = 0.0f;
        }
    }
    int64_t k = 0;
    if (k < cap) { out[3 * k] = b[0]; out[3 * k + 1] = b[1]; out[3 * k + 2] = b[2]; }
    k++;
    while (n[0] + n[1] + n[2] > 0) {
        int a = -1;
        for (int c = 0; c < 3; c++)
            if (n[c] > 0 && (a < 0 || t[c] < t[a])) a = c;
        b[a] += st[a];
        n[a]--;
        if (n[a] > 0) {
            float B = (float)(b[a] + (st[a] > 0 ? 1 : 0));
            t[a] = (B - P0[a]) / D[a];
        }
        if (k < cap) { out[3 * k] = b[0]; out[3 * k + 1] = b[1]; out[3 * k + 2] = b[2]; }
        k++;
    }
    return k;
}

/* ------------------------------------------------------------------------- */
/* band segment of one pixel, section "Allocation": the ray through pixel      */
/* (u, v) between camera depths max(d - mu, 0) and d + mu (a camera-z range),  */
/* in world coordinates, divided by the block edge 8 * voxel_size.             */
/* binary64, fixed order, no fused operations:                                 */
/*   r = ((u - cx) * (1/fx), (v - cy) * (1/fy), 1), 1/fx and 1/fy rounded once   */
/*   q = z * r;  P_a = ((R_a0 q_0 + R_a1 q_1) + R_a2 q_2) + t_a                 */
/*   end point = (float)(P_a * (1 / (8 s))), 1/(8 s) rounded once               */
/* Returns 0 when the pixel has no valid depth (not finite or not > 0) or the  */
/* segment leaves the range of 16-bit block coordinates.                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    int W, H;
    double fx, fy, cx, cy, inv_fx, inv_fy;
    double Rwc[9], twc[3];
    double Rcw[9], tcw[3];
} orc_cam;

static void orc_cam_setup(orc_cam *c, int W, int H, const double *K, const double *T_wc)
{
    c->W = W; c->H = H;
    c->fx = K[0]; c->fy = K[1]; c->cx = K[2]; c->cy = K[3];
    c->inv_fx = 1.0 / K[0];
    c->inv_fy = 1.0 / K[1];
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) c->Rwc[3 * i + j] = T_wc[4 * i + j];
        c->twc[i] = T_wc[4 * i + 3];
    }
    /* rigid inverse: R_cw = R_wc^T, t_cw = -R_wc^T t_wc (fixed order) */
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) c->Rcw[3 * i + j] = c->Rwc[3 * j + i];
        double acc = c->Rwc[0 * 3 + i] * c->twc[0];
        acc = acc + c->Rwc[1 * 3 + i] * c->twc[1];
        acc = acc + c->Rwc[2 * 3 + i] * c->twc[2];
        c->tcw[i] = -acc;
    }
}

static int orc_band_segment(const orc_scene *sc, const orc_cam *c, int u, int v, float depth,
                            float *P0, float *P1)
{
    if (!(depth > 0.0f) || isinf(depth)) return 0;
    double d = (double)depth;
    double z0 = d - sc->mu;
    if (z0 < 0.0) z0 = 0.0;
    double z1 = d + sc->mu;
    double rx = ((double)u - c->cx) * c->inv_fx;
    double ry = ((double)v - c->cy) * c->inv_fy;
    double inv_bs = 1.0 / (8.0 * sc->s);
    for (int k = 0; k < 2; k++) {
        double z = k ? z1 : z0;
        double q0 = z * rx, q1 = z * ry, q2 = z;
        float *P = k ? P1 : P0;
        for (int a = 0; a < 3; a++) {
            double w = c->Rwc[3 * a + 0] * q0;
            w = w + c->Rwc[3 * a + 1] * q1;
            w = w + c->Rwc[3 * a + 2] * q2;
            w = w + c->twc[a];
            P[a] = (float)(w * inv_bs);
            if (!(P[a] >= -32767.0f && P[a] < 32767.0f)) return 0;
        }
    }
    return 1;
}

/* exposed for tests: the two end points (block units) of a pixel's segment */
int orc_segment(const orc_scene *sc, int W, int H, const double *K, const double *T_wc, int u,
                int v, float depth, float *P0, float *P1)
{
    orc_cam c;
    orc_cam_setup(&c, W, H, K, T_wc);
    return orc_band_segment(sc, &c, u, v, depth, P0, P1);
}

/* ------------------------------------------------------------------------- */
/* allocation, stages one to three: every block crossed by a valid pixel's band */
/* segment is looked up, inserted when absent, and flagged visible.  Pixels     */
/* are visited in row-major order; the visible set is the set of flagged        */
/* entries.  Every crossed block is allocated (atomic insertion), not only the  */
/* last request per bucket.  Returns the number of visible entries.             */
/* ------------------------------------------------------------------------- */
static int orc_key_cmp3(const void *a, const void *b)
{
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    for (int i = 0; i < 3; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

int64_t orc_allocate(orc_scene *sc, const float *depth, int W, int H, const double *K,
                     const double *T_wc)
{
    sc->n_drop = 0;
    orc_cam c;
    orc_cam_setup(&c, W, H, K, T_wc);
    memset(sc->vis, 0, (size_t)sc->n_entries);
    int64_t cap = 1 << 16;
    int32_t *blk = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)cap);
    if (!blk) return -1;
    for (int v = 0; v < H; v++) {
        for (int u = 0; u < W; u++) {
            float P0[3], P1[3];
            if (!orc_band_segment(sc, &c, u, v, depth[(int64_t)v * W + u], P0, P1)) continue;
            int64_t nb = orc_dda_blocks(P0, P1, blk, cap);
            if (nb > cap) {
                int32_t *nbk = (int32_t *)realloc(blk, sizeof(int32_t) * 3 * (size_t)nb);
                if (!nbk) { free(blk); return -1; }
                blk = nbk;
                cap = nb;
                nb = orc_dda_blocks(P0, P1, blk, cap);
            }
            for (int64_t i = 0; i < nb; i++) {
                int64_t e = orc_insert(sc, blk[3 * i], blk[3 * i + 1], blk[3 * i + 2]);
                if (e >= 0) sc->vis[e] = 1;
            }
        }
    }
    free(blk);
    if (sc->n_drop > 0) {
        qsort(sc->drop_keys, (size_t)sc->n_drop, sizeof(int32_t) * 3, orc_key_cmp3);
        int64_t u = 1;
        for (int64_t i = 1; i < sc->n_drop; i++)
            u += orc_key_cmp3(sc->drop_keys + 3 * i, sc->drop_keys + 3 * (i - 1)) != 0;
        sc->dropped_total += u;
    }
    int64_t n = 0;
    for (int64_t i = 0; i < sc->n_entries; i++) n += sc->vis[i];
    sc->n_vis = n;
    return n;
}

/* ------------------------------------------------------------------------- */
/* voxel update, section "Integration" (computeUpdatedVoxelDepthInfo), for     */
/* voxel v = 8 k + l of block k, at world position v * s.                       */
/* Decisions in binary32, fixed order (no fused operations):                    */
/*   c  = R_cw (8 k s) + t_cw      binary64: ((R_a0 o_0 + R_a1 o_1) + R_a2 o_2) + t_a */
/*   hi = (float)c, lo = (float)(c - hi)                                        */
/*   g_j = (float)(R_cw[:, j] * s)  camera-frame step of one voxel along axis j  */
/*   dl = (l_x g_x + l_y g_y) + l_z g_z;  p = hi + (lo + dl)                     */
/*   skip if p_z <= 0; x = fx p_x / p_z + cx, y = fy p_y / p_z + cy;            */
/*   skip if x < 1, x > W - 2, y < 1 or y > H - 2;                              */
/*   d = depth[(int)(x + 0.5) + (int)(y + 0.5) W]; skip unless d finite, > 0;   */
/*   eta32 = (d - hi_z) - (lo_z + dl_z); skip if eta32 < -mu.                   */
/* Value in binary64 from the plain definition: p_z = R_cw row z . (v s) + t_z, */
/*   eta = d - p_z, f = min(1, eta / mu), F <- (W F + f) / (W + 1),             */
/*   W <- min(W + 1, max_w)   (the average uses W + 1 before the cap).          */
/* ------------------------------------------------------------------------- */
typedef struct {
    orc_cam c;
    float fx, fy, cx, cy;  /* binary32 intrinsics for the projection decision */
    float g[3][3];         /* g[j][a]: step along world axis j, camera component a */
    const float *depth;
    const uint8_t *rgbx;   /* registered colour image, 4 bytes per pixel, or NULL */
    float mu_f;
    double mu, s;
    int max_w;
} orc_frame;

static void orc_frame_setup(orc_frame *fr, const orc_scene *sc, const float *depth, int W,
                            int H, const double *K, const double *T_wc)
{
    orc_cam_setup(&fr->c, W, H, K, T_wc);
    fr->fx = (float)K[0]; fr->fy = (float)K[1]; fr->cx = (float)K[2]; fr->cy = (float)K[3];
    for (int j = 0; j < 3; j++)
        for (int a = 0; a < 3; a++) fr->g[j][a] = (float)(fr->c.Rcw[3 * a + j] * sc->s);
    fr->depth = depth;
    fr->rgbx = NULL;
    fr->mu_f = sc->mu_f;
    fr->mu = sc->mu;
    fr->s = sc->s;
    fr->max_w = sc->max_w;
}

typedef struct { float hi[3], lo[3]; } orc_blockorigin;

static void orc_block_origin(const orc_frame *fr, int32_t kx, int32_t ky, int32_t kz,
                             orc_blockorigin *bo)
{
    double o[3] = {(double)(8 * kx) * fr->s, (double)(8 * ky) * fr->s, (double)(8 * kz) * fr->s};
    for (int a = 0; a < 3; a++) {
        double w = fr->c.Rcw[3 * a + 0] * o[0];
        w = w + fr->c.Rcw[3 * a + 1] * o[1];
        w = w + fr->c.Rcw[3 * a + 2] * o[2];
        w = w + fr->c.tcw[a];
        bo->hi[a] = (float)w;
        bo->lo[a] = (float)(w - (double)bo->hi[a]);
    }
}

/* returns 1 when the voxel was updated */
/* Colour (readings; the paper shows the voxel type and says a similar function
 * updates the colour): the colour image is registered with the depth image and
 * read at the same pixel; a voxel whose depth update ran takes a colour sample
 * when it lies inside the band, eta32 <= mu (binary32, like the other decisions);
 * each channel keeps the running average of its samples rounded to the nearest
 * integer (ties to even), new = round((w_c c + sample) / (w_c + 1)) in exact
 * integer arithmetic, and w_c <- min(w_c + 1, min(max_w, 255)). */
static uint8_t orc_colour_mean(int c, int w, int sample)
{
    const int num = w * c + sample, den = w + 1;
    int q = num / den;
    const int r2 = 2 * (num - q * den);
    if (r2 > den || (r2 == den && (q & 1))) q++;
    return (uint8_t)q;
}

static int orc_update_voxel(const orc_frame *fr, const orc_blockorigin *bo, int32_t kx,
                            int32_t ky, int32_t kz, int lx, int ly, int lz, double *F,
                            int32_t *Wt, uint8_t *C)
{
    float fl[3] = {(float)lx, (float)ly, (float)lz};
    float dl[3], p[3];
    for (int a = 0; a < 3; a++) {
        float t = fl[0] * fr->g[0][a];
        t = t + fl[1] * fr->g[1][a];
        t = t + fl[2] * fr->g[2][a];
        dl[a] = t;
        p[a] = bo->hi[a] + (bo->lo[a] + dl[a]);
    }
    if (p[2] <= 0.0f) return 0;
    float x = fr->fx * p[0] / p[2] + fr->cx;
    float y = fr->fy * p[1] / p[2] + fr->cy;
    if (x < 1.0f || x > (float)(fr->c.W - 2) || y < 1.0f || y > (float)(fr->c.H - 2)) return 0;
    const int pix = (int)(x + 0.5f) + (int)(y + 0.5f) * fr->c.W;
    float d = fr->depth[pix];
    if (!(d > 0.0f) || isinf(d)) return 0;
    float eta32 = (d - bo->hi[2]) - (bo->lo[2] + dl[2]);
    if (eta32 < -fr->mu_f) return 0;
    if (C && fr->rgbx && eta32 <= fr->mu_f) {
        const int wc = C[3];
        for (int ch = 0; ch < 3; ch++) C[ch] = orc_colour_mean(C[ch], wc, fr->rgbx[4 * pix + ch]);
        const int cap = fr->max_w < 255 ? fr->max_w : 255;
        C[3] = (uint8_t)(wc + 1 < cap ? wc + 1 : cap);
    }

    double vs[3] = {(double)(8 * kx + lx) * fr->s, (double)(8 * ky + ly) * fr->s,
                    (double)(8 * kz + lz) * fr->s};
    double pz = fr->c.Rcw[6] * vs[0] + fr->c.Rcw[7] * vs[1] + fr->c.Rcw[8] * vs[2] + fr->c.tcw[2];
    double eta = (double)d - pz;
    double f = eta / fr->mu;
    if (f > 1.0) f = 1.0;
    double w = (double)(*Wt);
    *F = (w * (*F) + f) / (w + 1.0);
    int nw = *Wt + 1;
    *Wt = nw < fr->max_w ? nw : fr->max_w;
    return 1;
}

/* integration over the visible blocks of the current frame */
static int64_t orc_integrate_visible(orc_scene *sc, const orc_frame *fr)
{
    int64_t n = 0;
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(sc->n_vis + 1));
    if (!list) return -1;
    for (int64_t i = 0; i < sc->n_entries; i++)
        if (sc->vis[i]) list[n++] = i;
    int64_t updated = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : updated)
    for (int64_t j = 0; j < n; j++) {
        const orc_entry *h = &sc->e[list[j]];
        orc_blockorigin bo;
        orc_block_origin(fr, h->x, h->y, h->z, &bo);
        double *F = sc->F + (int64_t)h->ptr * SDF_BLOCK3;
        int32_t *W = sc->W + (int64_t)h->ptr * SDF_BLOCK3;
        uint8_t *Cb = sc->C ? sc->C + 4 * (int64_t)h->ptr * SDF_BLOCK3 : NULL;
        for (int lz = 0; lz < 8; lz++)
            for (int ly = 0; ly < 8; ly++)
                for (int lx = 0; lx < 8; lx++) {
                    int li = lx + 8 * ly + 64 * lz;
                    updated += orc_update_voxel(fr, &bo, h->x, h->y, h->z, lx, ly, lz, &F[li], &W[li],
                                                Cb ? Cb + 4 * li : NULL);
                }
    }
    free(list);
    sc->updated_last = updated;
    return updated;
}

/* one frame: allocation then integration.  Returns the number of updated voxels. */
int64_t orc_integrate(orc_scene *sc, const float *depth, int W, int H, const double *K,
                      const double *T_wc)
{
    if (orc_allocate(sc, depth, W, H, K, T_wc) < 0) return -1;
    orc_frame fr;
    orc_frame_setup(&fr, sc, depth, W, H, K, T_wc);
    return orc_integrate_visible(sc, &fr);
}

/* colour voxels: storage for every block, present and future (colour (0, 0, 0),
   weight 0) */
int orc_enable_colour(orc_scene *sc)
{
    if (sc->C) return 0;
    sc->C = (uint8_t *)calloc(4 * SDF_BLOCK3 * (size_t)(sc->cap_blocks ? sc->cap_blocks : 1), 1);
    return sc->C ? 0 : -1;
}

/* a frame with its registered colour image (4 bytes per pixel: r, g, b, unused) */
int64_t orc_integrate_colour(orc_scene *sc, const float *depth, const uint8_t *rgbx, int W, int H,
                             const double *K, const double *T_wc)
{
    if (!sc->C) return -1;
    if (orc_allocate(sc, depth, W, H, K, T_wc) < 0) return -1;
    orc_frame fr;
    orc_frame_setup(&fr, sc, depth, W, H, K, T_wc);
    fr.rgbx = rgbx;
    return orc_integrate_visible(sc, &fr);
}

/* keys of the current frame's visible blocks (entry order) */
int64_t orc_visible_keys(const orc_scene *sc, int32_t *out, int64_t cap)
{
    int64_t n = 0;
    for (int64_t i = 0; i < sc->n_entries; i++) {
        if (!sc->vis[i]) continue;
        if (n < cap) {
            out[3 * n] = sc->e[i].x; out[3 * n + 1] = sc->e[i].y; out[3 * n + 2] = sc->e[i].z;
        }
        n++;
    }
    return n;
}

/* stats: n_allocated, n_visible (last frame), excess used, dropped total,
 * excess demand D = sum over buckets of max(0, keys in bucket - 2), updated
 * voxels (last frame) */
void orc_stats(const orc_scene *sc, int64_t *out)
{
    out[0] = sc->n_blocks;
    out[1] = sc->n_vis;
    out[2] = sc->excess_used;
    out[3] = sc->dropped_total;
    int64_t D = 0;
    /* keys per bucket: bucket entries in use plus the chain length */
    for (int64_t b = 0; b < sc->n_buckets; b++) {
        int64_t nb = 0;
        for (int i = 0; i < ENTRIES_PER_BUCKET; i++) nb += sc->e[b * ENTRIES_PER_BUCKET + i].ptr >= 0;
        int32_t off = sc->e[b * ENTRIES_PER_BUCKET + ENTRIES_PER_BUCKET - 1].offset - 1;
        while (off >= 0) {
            nb++;
            off = sc->e[ENTRIES_PER_BUCKET * sc->n_buckets + off].offset - 1;
        }
        if (nb > ENTRIES_PER_BUCKET) D += nb - ENTRIES_PER_BUCKET;
    }
    out[4] = D;
    out[5] = sc->updated_last;
}

/* raw hash table, for the structure invariants */
void orc_entries(const orc_scene *sc, int16_t *pos, int32_t *offset, int32_t *ptr)
{
    for (int64_t i = 0; i < sc->n_entries; i++) {
        pos[3 * i] = sc->e[i].x; pos[3 * i + 1] = sc->e[i].y; pos[3 * i + 2] = sc->e[i].z;
        offset[i] = sc->e[i].offset;
        ptr[i] = sc->e[i].ptr;
    }
}

static int orc_key_cmp(const void *a, const void *b)
{
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    for (int i = 0; i < 3; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

/* allocated blocks sorted by (x, y, z); F and W per voxel, order lx + 8 ly + 64 lz.
 * coords may be NULL to count.  Returns the number of allocated blocks. */
int64_t orc_export(const orc_scene *sc, int32_t *coords, double *F, int32_t *Wt, int64_t cap)
{
    int64_t n = sc->n_blocks;
    if (!coords || cap < n) return n;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(n + 1));
    if (!tmp) return -1;
    int64_t k = 0;
    for (int64_t i = 0; i < sc->n_entries; i++) {
        if (sc->e[i].ptr < 0) continue;
        tmp[4 * k] = sc->e[i].x; tmp[4 * k + 1] = sc->e[i].y; tmp[4 * k + 2] = sc->e[i].z;
        tmp[4 * k + 3] = sc->e[i].ptr;
        k++;
    }
    qsort(tmp, (size_t)k, sizeof(int32_t) * 4, orc_key_cmp);
    for (int64_t i = 0; i < k; i++) {
        coords[3 * i] = tmp[4 * i]; coords[3 * i + 1] = tmp[4 * i + 1]; coords[3 * i + 2] = tmp[4 * i + 2];
        if (F) memcpy(F + i * SDF_BLOCK3, sc->F + (int64_t)tmp[4 * i + 3] * SDF_BLOCK3, sizeof(double) * SDF_BLOCK3);
        if (Wt) memcpy(Wt + i * SDF_BLOCK3, sc->W + (int64_t)tmp[4 * i + 3] * SDF_BLOCK3, sizeof(int32_t) * SDF_BLOCK3);
    }
    free(tmp);
    return k;
}

/* colours of the allocated blocks, in the order of orc_export */
int64_t orc_export_colour(const orc_scene *sc, uint8_t *rgbw, int64_t cap)
{
    int64_t n = sc->n_blocks;
    if (!sc->C) return -1;
    if (!rgbw || cap < n) return n;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(n + 1));
    if (!tmp) return -1;
    int64_t k = 0;
    for (int64_t i = 0; i < sc->n_entries; i++) {
        if (sc->e[i].ptr < 0) continue;
        tmp[4 * k] = sc->e[i].x; tmp[4 * k + 1] = sc->e[i].y; tmp[4 * k + 2] = sc->e[i].z;
        tmp[4 * k + 3] = sc->e[i].ptr;
        k++;
    }
    qsort(tmp, (size_t)k, sizeof(int32_t) * 4, orc_key_cmp);
    for (int64_t i = 0; i < k; i++)
        memcpy(rgbw + 4 * i * SDF_BLOCK3, sc->C + 4 * (int64_t)tmp[4 * i + 3] * SDF_BLOCK3, 4 * SDF_BLOCK3);
    free(tmp);
    return k;
}

/* colour at surface points (the raycast's colour read; reading: the colour of
   the nearest lattice voxel floor(p / s + 1/2), as the march's own reads):
   (r, g, b, 255) when that voxel's block is allocated, zeros otherwise or where
   the point is not a hit (w <= 0) */
int orc_colour_at(const orc_scene *sc, const float *pts, int64_t n, uint8_t *out)
{
    if (!sc->C) return -1;
    for (int64_t i = 0; i < n; i++) {
        uint8_t *o = out + 4 * i;
        o[0] = o[1] = o[2] = o[3] = 0;
        if (!(pts[4 * i + 3] > 0.0f)) continue;
        int32_t v[3], k[3], l[3];
        for (int a = 0; a < 3; a++) {
            v[a] = (int32_t)floor((double)pts[4 * i + a] / sc->s + 0.5);
            k[a] = v[a] >= 0 ? v[a] / SDF_BLOCK : -((-v[a] + SDF_BLOCK - 1) / SDF_BLOCK);
            l[a] = v[a] - SDF_BLOCK * k[a];
        }
        if (k[0] < -32768 || k[0] > 32767 || k[1] < -32768 || k[1] > 32767 || k[2] < -32768 || k[2] > 32767)
            continue;
        const int64_t e = orc_find(sc, k[0], k[1], k[2]);
        if (e < 0) continue;
        const uint8_t *c = sc->C + 4 * ((int64_t)sc->e[e].ptr * SDF_BLOCK3 + l[0] + 8 * l[1] + 64 * l[2]);
        o[0] = c[0]; o[1] = c[1]; o[2] = c[2]; o[3] = 255;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* sampled voxels: the same update applied to a list of individual voxels,     */
/* for checks of full-size runs voxel by voxel.  active[i] != 0 when voxel i's  */
/* block is visible in this frame.  Returns the number updated.                 */
/* ------------------------------------------------------------------------- */
int64_t orc_update_voxels(const orc_scene *sc, const float *depth, int W, int H, const double *K,
                          const double *T_wc, const int32_t *vox, const uint8_t *active,
                          int64_t n, double *F, int32_t *Wt)
{
    orc_frame fr;
    orc_frame_setup(&fr, sc, depth, W, H, K, T_wc);
    int64_t upd = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!active[i]) continue;
        int32_t v[3] = {vox[3 * i], vox[3 * i + 1], vox[3 * i + 2]};
        int32_t k[3], l[3];
        for (int a = 0; a < 3; a++) {
            k[a] = (int32_t)floor((double)v[a] / 8.0);
            l[a] = v[a] - 8 * k[a];
        }
        orc_blockorigin bo;
        orc_block_origin(&fr, k[0], k[1], k[2], &bo);
        upd += orc_update_voxel(&fr, &bo, k[0], k[1], k[2], l[0], l[1], l[2], &F[i], &Wt[i], NULL);
    }
    return upd;
}

/* ------------------------------------------------------------------------- */
/* dense volume, section "Dense Volumes": one grid of nx*ny*nz voxels whose     */
/* first voxel is at integer voxel coordinates (ox, oy, oz); the same update    */
/* for every voxel (no allocation).  A voxel's block and in-block index come   */
/* from its absolute voxel coordinates, exactly as in the hashed volume.  An   */
/* optional block mask restricts the update to voxels whose block is listed.   */
/* frames[i] collects a bit per frame that updated voxel i (first 64 frames).  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t o[3], n[3];
    double s, mu;
    float mu_f;
    int max_w;
    double *F;
    int32_t *W;
    uint64_t *frames;
    int frame_no;
} orc_dense;

orc_dense *orc_dense_create(int64_t ox, int64_t oy, int64_t oz, int64_t nx, int64_t ny, int64_t nz,
                            float voxel_size, float mu, int32_t max_w)
{
    if (nx <= 0 || ny <= 0 || nz <= 0) return NULL;
    orc_dense *dv = (orc_dense *)calloc(1, sizeof(orc_dense));
    if (!dv) return NULL;
    dv->o[0] = ox; dv->o[1] = oy; dv->o[2] = oz;
    dv->n[0] = nx; dv->n[1] = ny; dv->n[2] = nz;
    dv->s = (double)voxel_size; dv->mu = (double)mu; dv->mu_f = mu; dv->max_w = max_w;
    size_t N = (size_t)(nx * ny * nz);
    dv->F = (double *)malloc(sizeof(double) * N);
    dv->W = (int32_t *)calloc(N, sizeof(int32_t));
    dv->frames = (uint64_t *)calloc(N, sizeof(uint64_t));
    if (!dv->F || !dv->W || !dv->frames) {
        free(dv->F); free(dv->W); free(dv->frames); free(dv); return NULL;
    }
    for (size_t i = 0; i < N; i++) dv->F[i] = 1.0;
    return dv;
}

void orc_dense_destroy(orc_dense *dv)
{
    if (!dv) return;
    free(dv->F); free(dv->W); free(dv->frames); free(dv);
}

static int64_t fdiv8(int64_t v) { return v >= 0 ? v / 8 : -((-v + 7) / 8); }

int64_t orc_dense_integrate(orc_dense *dv, const float *depth, int W, int H, const double *K,
                            const double *T_wc, const int32_t *mask_keys, int64_t n_mask)
{
    orc_frame fr;
    orc_cam_setup(&fr.c, W, H, K, T_wc);
    fr.fx = (float)K[0]; fr.fy = (float)K[1]; fr.cx = (float)K[2]; fr.cy = (float)K[3];
    for (int j = 0; j < 3; j++)
        for (int a = 0; a < 3; a++) fr.g[j][a] = (float)(fr.c.Rcw[3 * a + j] * dv->s);
    fr.depth = depth; fr.mu_f = dv->mu_f; fr.mu = dv->mu; fr.s = dv->s; fr.max_w = dv->max_w;
    /* block-level mask over the block range the grid spans */
    int64_t kb0[3], kn[3];
    for (int a = 0; a < 3; a++) {
        kb0[a] = fdiv8(dv->o[a]);
        kn[a] = fdiv8(dv->o[a] + dv->n[a] - 1) - kb0[a] + 1;
    }
    uint8_t *bm = NULL;
    if (mask_keys) {
        bm = (uint8_t *)calloc((size_t)(kn[0] * kn[1] * kn[2]), 1);
        if (!bm) return -1;
        for (int64_t m = 0; m < n_mask; m++) {
            int64_t q[3];
            int inside = 1;
            for (int a = 0; a < 3; a++) {
                q[a] = mask_keys[3 * m + a] - kb0[a];
                inside &= q[a] >= 0 && q[a] < kn[a];
            }
            if (inside) bm[q[0] + kn[0] * (q[1] + kn[1] * q[2])] = 1;
        }
    }
    int64_t updated = 0;
    int fbit = dv->frame_no;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : updated)
    for (int64_t iz = 0; iz < dv->n[2]; iz++) {
        for (int64_t iy = 0; iy < dv->n[1]; iy++) {
            for (int64_t ix = 0; ix < dv->n[0]; ix++) {
                int64_t v[3] = {dv->o[0] + ix, dv->o[1] + iy, dv->o[2] + iz};
                int32_t k[3], l[3];
                for (int a = 0; a < 3; a++) {
                    k[a] = (int32_t)fdiv8(v[a]);
                    l[a] = (int32_t)(v[a] - 8 * (int64_t)k[a]);
                }
                if (bm && !bm[(k[0] - kb0[0]) + kn[0] * ((k[1] - kb0[1]) + kn[1] * (k[2] - kb0[2]))])
                    continue;
                orc_blockorigin bo;
                orc_block_origin(&fr, k[0], k[1], k[2], &bo);
                int64_t i = ix + dv->n[0] * (iy + dv->n[1] * iz);
                int u = orc_update_voxel(&fr, &bo, k[0], k[1], k[2], l[0], l[1], l[2], &dv->F[i], &dv->W[i], NULL);
                if (u && fbit < 64) dv->frames[i] |= (uint64_t)1 << fbit;
                updated += u;
            }
        }
    }
    free(bm);
    dv->frame_no++;
    return updated;
}

void orc_dense_read(const orc_dense *dv, double *F, int32_t *Wt, uint64_t *frames)
{
    size_t N = (size_t)(dv->n[0] * dv->n[1] * dv->n[2]);
    if (F) memcpy(F, dv->F, sizeof(double) * N);
    if (Wt) memcpy(Wt, dv->W, sizeof(int32_t) * N);
    if (frames) memcpy(frames, dv->frames, sizeof(uint64_t) * N);
}

/* ------------------------------------------------------------------------- */
/* raycast, section "Raycast".  Reads from the hashed volume:                  */
/*   n(p)   = nearest lattice voxel floor(p / s + 1/2) (voxel v sits at v s);  */
/*   found  = the block of n(p) is allocated; F_n = F at n(p);                 */
/*   F_t(p) = trilinear interpolation of F over the 8 lattice voxels around    */
/*            p / s, unallocated voxels reading F = 1.                         */
/* Ray: unit world direction of pixel (u, v), from the camera centre; t is the */
/* distance along it, searched over camera depths [z_near, z_far].             */
/* State machine (step lengths are this implementation's reading):             */
/*   COARSE:     not found -> t += 8 s; found -> step back t = max(t - 8 s,    */
/*               t_near), go FINE                                              */
/*   FINE:       not found -> t += mu, and after ceil(8 s / mu) + 1 such steps  */
/*               go COARSE; F_n < 0 -> WRONG_SIDE; else -> SURFACE             */
/*   SURFACE:    not found -> COARSE; F_n < 0 -> BEHIND; else t += max(F_n mu, s) */
/*   WRONG_SIDE: not found -> COARSE; F_n > 0 -> SURFACE; else                 */
/*               t += max(-F_n mu, s)                                          */
/*   BEHIND:     two refinement steps t += F_t(o + t d) mu; the hit is o + t d. */
/* Normal: central differences of F_t at +-s along the world axes, normalised. */
/* ------------------------------------------------------------------------- */
static int orc_read_nearest(const orc_scene *sc, const double *p, double *F)
{
    int32_t n[3], k[3];
    for (int a = 0; a < 3; a++) {
        double q = floor(p[a] / sc->s + 0.5);
        if (!(q > -262000.0 && q < 262000.0)) return 0;
        n[a] = (int32_t)q;
        k[a] = (int32_t)fdiv8(n[a]);
    }
    int64_t e = orc_find(sc, k[0], k[1], k[2]);
    if (e < 0) return 0;
    int li = (n[0] - 8 * k[0]) + 8 * (n[1] - 8 * k[1]) + 64 * (n[2] - 8 * k[2]);
    *F = sc->F[(int64_t)sc->e[e].ptr * SDF_BLOCK3 + li];
    return 1;
}

static double orc_voxel_F(const orc_scene *sc, int32_t vx, int32_t vy, int32_t vz)
{
    int32_t k[3] = {(int32_t)fdiv8(vx), (int32_t)fdiv8(vy), (int32_t)fdiv8(vz)};
    int64_t e = orc_find(sc, k[0], k[1], k[2]);
    if (e < 0) return 1.0;
    int li = (vx - 8 * k[0]) + 8 * (vy - 8 * k[1]) + 64 * (vz - 8 * k[2]);
    return sc->F[(int64_t)sc->e[e].ptr * SDF_BLOCK3 + li];
}

static double orc_read_trilinear(const orc_scene *sc, const double *p)
{
    double q[3], fr[3];
    int32_t i0[3];
    for (int a = 0; a < 3; a++) {
        q[a] = p[a] / sc->s;
        double fl = floor(q[a]);
        if (!(fl > -262000.0 && fl < 262000.0)) return 1.0;
        i0[a] = (int32_t)fl;
        fr[a] = q[a] - fl;
    }
    double acc = 0.0;
    for (int c = 0; c < 8; c++) {
        int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        double w = (dx ? fr[0] : 1.0 - fr[0]) * (dy ? fr[1] : 1.0 - fr[1]) * (dz ? fr[2] : 1.0 - fr[2]);
        acc += w * orc_voxel_F(sc, i0[0] + dx, i0[1] + dy, i0[2] + dz);
    }
    return acc;
}

enum { ORC_COARSE, ORC_FINE, ORC_SURFACE, ORC_BEHIND, ORC_WRONG_SIDE };

typedef struct {
    double o[3], d[3], t_near, t_far, len;
} orc_ray;

/* zr: this pixel's expected depth range (camera depth, zr[0] = min, zr[1] = max)
 * or NULL for the fixed range [z_near, z_far].  With a range the ray searches
 * t in [max(z_min len, t_near), min(z_max len, t_far)]; an empty range (no
 * visible block projects onto the pixel) leaves nothing to search. */
static void orc_ray_setup(const orc_scene *sc, const orc_cam *c, int u, int v, const float *zr,
                          orc_ray *r)
{
    double cd[3] = {((double)u - c->cx) / c->fx, ((double)v - c->cy) / c->fy, 1.0};
    r->len = sqrt(cd[0] * cd[0] + cd[1] * cd[1] + 1.0);
    for (int a = 0; a < 3; a++) {
        r->d[a] = (c->Rwc[3 * a] * cd[0] + c->Rwc[3 * a + 1] * cd[1] + c->Rwc[3 * a + 2]) / r->len;
        r->o[a] = c->twc[a];
    }
    r->t_near = (double)sc->z_near * r->len;
    r->t_far = (double)sc->z_far * r->len;
    if (zr) {
        if (!((double)zr[0] <= (double)zr[1])) { r->t_far = r->t_near; return; }
        double a = (double)zr[0] * r->len, b = (double)zr[1] * r->len;
        if (a > r->t_near) r->t_near = a;
        if (b < r->t_far) r->t_far = b;
    }
}

/* flags bit 0: a sign decision had |F_n| < 1e-4; bit 1: iteration cap reached */
static int orc_march(const orc_scene *sc, const orc_ray *r, double *t_hit, int *flags, int *steps)
{
    double bs = 8.0 * sc->s, t = r->t_near;
    int state = ORC_COARSE, fine_miss = 0;
    int fine_budget = (int)ceil(bs / sc->mu) + 1;
    int cap = (int)((r->t_far - r->t_near) / sc->s) * 4 + 1000;
    *flags = 0;
    int it;
    for (it = 0; it < cap; it++) {
        if (!(t < r->t_far)) break;
        double p[3] = {r->o[0] + t * r->d[0], r->o[1] + t * r->d[1], r->o[2] + t * r->d[2]};
        double F = 1.0;
        int found = orc_read_nearest(sc, p, &F);
        if (found && fabs(F) < 1e-4 && state != ORC_COARSE) *flags |= 1;
        switch (state) {
        case ORC_COARSE:
            if (!found) t += bs;
            else { t = t - bs > r->t_near ? t - bs : r->t_near; state = ORC_FINE; fine_miss = 0; }
            break;
        case ORC_FINE:
            if (!found) {
                t += sc->mu;
                if (++fine_miss > fine_budget) state = ORC_COARSE;
            } else if (F < 0) state = ORC_WRONG_SIDE;
            else state = ORC_SURFACE;
            break;
        case ORC_SURFACE:
            if (!found) state = ORC_COARSE;
            else if (F < 0) state = ORC_BEHIND;
            else t += (F * sc->mu > sc->s ? F * sc->mu : sc->s);
            break;
        case ORC_WRONG_SIDE:
            if (!found) state = ORC_COARSE;
            else if (F > 0) state = ORC_SURFACE;
            else t += (-F * sc->mu > sc->s ? -F * sc->mu : sc->s);
            break;
        }
        if (state == ORC_BEHIND) break;
    }
    *steps = it;
    if (it >= cap) *flags |= 2;
    if (state != ORC_BEHIND) return 0;
    for (int k = 0; k < 2; k++) {
        double p[3] = {r->o[0] + t * r->d[0], r->o[1] + t * r->d[1], r->o[2] + t * r->d[2]};
        t += orc_read_trilinear(sc, p) * sc->mu;
    }
    *t_hit = t;
    return 1;
}

/* pts/normals: H*W*4 binary64, world frame; pts w = 1 on a hit, all zero on a
 * miss; normals w = 1 when the gradient is non-zero.  zc: camera depth of the
 * hit (0 on a miss).  flags/steps per pixel may be NULL.  zr: H*W*2 expected
 * depth ranges (see orc_expected_depths) or NULL for [z_near, z_far]. */
int orc_raycast_range(const orc_scene *sc, int W, int H, const double *K, const double *T_wc,
                      const float *zr, double *pts, double *normals, double *zc, uint8_t *flags,
                      int32_t *steps)
{
    orc_cam c;
    orc_cam_setup(&c, W, H, K, T_wc);
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < H; v++) {
        for (int u = 0; u < W; u++) {
            int64_t i = (int64_t)v * W + u;
            orc_ray r;
            orc_ray_setup(sc, &c, u, v, zr ? zr + 2 * i : NULL, &r);
            double t = 0;
            int fl = 0, st = 0;
            int hit = orc_march(sc, &r, &t, &fl, &st);
            if (flags) flags[i] = (uint8_t)fl;
            if (steps) steps[i] = st;
            for (int a = 0; a < 4; a++) { pts[4 * i + a] = 0; normals[4 * i + a] = 0; }
            if (zc) zc[i] = 0;
            if (!hit) continue;
            double p[3] = {r.o[0] + t * r.d[0], r.o[1] + t * r.d[1], r.o[2] + t * r.d[2]};
            for (int a = 0; a < 3; a++) pts[4 * i + a] = p[a];
            pts[4 * i + 3] = 1.0;
            if (zc) zc[i] = t / r.len;
            double g[3];
            for (int a = 0; a < 3; a++) {
                double pp[3] = {p[0], p[1], p[2]}, pm[3] = {p[0], p[1], p[2]};
                pp[a] += sc->s;
                pm[a] -= sc->s;
                g[a] = orc_read_trilinear(sc, pp) - orc_read_trilinear(sc, pm);
            }
            double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            if (gn > 0) {
                for (int a = 0; a < 3; a++) normals[4 * i + a] = g[a] / gn;
                normals[4 * i + 3] = 1.0;
            }
        }
    }
    return 0;
}

int orc_raycast(const orc_scene *sc, int W, int H, const double *K, const double *T_wc,
                double *pts, double *normals, double *zc, uint8_t *flags, int32_t *steps)
{
    return orc_raycast_range(sc, W, H, K, T_wc, NULL, pts, normals, zc, flags, steps);
}

/* plain-definition cross-check of the raycast: the first + to - zero crossing
 * of F_t along the ray over [t_near, t_far], sampled every s / 4 and bisected
 * to 1e-7 m.  zc: camera depth of the crossing, 0 when there is none. */
int orc_raycast_crossing(const orc_scene *sc, int W, int H, const double *K, const double *T_wc,
                         double *zc)
{
    orc_cam c;
    orc_cam_setup(&c, W, H, K, T_wc);
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < H; v++) {
        for (int u = 0; u < W; u++) {
            orc_ray r;
            orc_ray_setup(sc, &c, u, v, NULL, &r);
            double h = sc->s / 4.0, t0 = r.t_near;
            double p[3] = {r.o[0] + t0 * r.d[0], r.o[1] + t0 * r.d[1], r.o[2] + t0 * r.d[2]};
            double f0 = orc_read_trilinear(sc, p), res = 0;
            for (double t1 = t0 + h; t1 <= r.t_far; t1 += h) {
                double q[3] = {r.o[0] + t1 * r.d[0], r.o[1] + t1 * r.d[1], r.o[2] + t1 * r.d[2]};
                double f1 = orc_read_trilinear(sc, q);
                if (f0 > 0 && f1 < 0) {
                    double a = t0, b = t1;
                    while (b - a > 1e-7) {
                        double m = 0.5 * (a + b);
                        double pm[3] = {r.o[0] + m * r.d[0], r.o[1] + m * r.d[1], r.o[2] + m * r.d[2]};
                        if (orc_read_trilinear(sc, pm) > 0) a = m; else b = m;
                    }
                    res = 0.5 * (a + b) / r.len;
                    break;
                }
                t0 = t1;
                f0 = f1;
            }
            zc[(int64_t)v * W + u] = res;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Expected depth range per pixel (section "Raycast", the search range):      */
/* every block visible in the last frame is projected into the image; the     */
/* pixels inside the 2D bounding box of its projection get the minimum and     */
/* maximum camera depth of its 3D bounding box, overlapping boxes combined by  */
/* min and max.  Readings:                                                      */
/*   - a block's 3D box is the region whose samples read it in the march       */
/*     (nearest voxel): [8k - 1/2, 8k + 7 1/2] s per axis, so every sample that */
/*     finds the block lies inside the box;                                    */
/*   - the 2D box is that of the 8 projected corners; pixel (u, v), centre at  */
/*     integer coordinates, is inside when ceil(x_min) <= u <= floor(x_max),   */
/*     likewise v, clipped to the image;                                       */
/*   - a block with a corner at camera depth <= 0 cannot be projected: it      */
/*     covers the whole image with the range [0, its largest corner depth];    */
/*   - arithmetic in binary64, corners as ((R0 X0 + R1 X1) + R2 X2) + t, the   */
/*     range stored in binary32 rounded outwards (min down, max up);           */
/*   - a pixel no block covers gets the empty range (+inf, 0).                 */
/* zr: H*W*2 binary32, (z_min, z_max) per pixel.                               */
/* ------------------------------------------------------------------------- */
static float orc_round_down(double z)
{
    float f = (float)z;
    if ((double)f > z) f = nextafterf(f, -INFINITY);
    return f;
}

static float orc_round_up(double z)
{
    float f = (float)z;
    if ((double)f < z) f = nextafterf(f, INFINITY);
    return f;
}

int orc_expected_depths(const orc_scene *sc, int W, int H, const double *K, const double *T_wc,
                        float *zr)
{
    orc_cam c;
    orc_cam_setup(&c, W, H, K, T_wc);
    for (int64_t i = 0; i < (int64_t)W * H; i++) { zr[2 * i] = INFINITY; zr[2 * i + 1] = 0.0f; }
    for (int64_t e = 0; e < sc->n_entries; e++) {
        if (!sc->vis[e]) continue;
        const int32_t k[3] = {sc->e[e].x, sc->e[e].y, sc->e[e].z};
        double zlo = INFINITY, zhi = -INFINITY, xlo = INFINITY, xhi = -INFINITY;
        double ylo = INFINITY, yhi = -INFINITY;
        int behind = 0;
        for (int corner = 0; corner < 8; corner++) {
            double X[3], P[3];
            for (int a = 0; a < 3; a++) {
                int up = (corner >> a) & 1;
                X[a] = ((double)(8 * k[a]) - 0.5 + (up ? 8.0 : 0.0)) * sc->s;
            }
            for (int a = 0; a < 3; a++) {
                double w = c.Rcw[3 * a + 0] * X[0];
                w = w + c.Rcw[3 * a + 1] * X[1];
                w = w + c.Rcw[3 * a + 2] * X[2];
                P[a] = w + c.tcw[a];
            }
            if (P[2] < zlo) zlo = P[2];
            if (P[2] > zhi) zhi = P[2];
            if (P[2] <= 0.0) { behind = 1; continue; }
            double x = c.fx * P[0] / P[2] + c.cx, y = c.fy * P[1] / P[2] + c.cy;
            if (x < xlo) xlo = x;
            if (x > xhi) xhi = x;
            if (y < ylo) ylo = y;
            if (y > yhi) yhi = y;
        }
        int u0, u1, v0, v1;
        if (behind) {
            u0 = 0; u1 = W - 1; v0 = 0; v1 = H - 1;
            zlo = 0.0;
        } else {
            double a0 = ceil(xlo), a1 = floor(xhi), b0 = ceil(ylo), b1 = floor(yhi);
            if (a1 < 0.0 || b1 < 0.0 || a0 > (double)(W - 1) || b0 > (double)(H - 1) || a0 > a1 ||
                b0 > b1)
                continue;
            u0 = a0 < 0.0 ? 0 : (int)a0;
            v0 = b0 < 0.0 ? 0 : (int)b0;
            u1 = a1 > (double)(W - 1) ? W - 1 : (int)a1;
            v1 = b1 > (double)(H - 1) ? H - 1 : (int)b1;
        }
        float fz0 = orc_round_down(zlo), fz1 = orc_round_up(zhi);
        for (int v = v0; v <= v1; v++)
            for (int u = u0; u <= u1; u++) {
                float *r = zr + 2 * ((int64_t)v * W + u);
                if (fz0 < r[0]) r[0] = fz0;
                if (fz1 > r[1]) r[1] = fz1;
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* depth tracker, section "Tracking" (ITMDepthTracker): the reference maps V   */
/* (surface points) and N (normals), world frame, come from a raycast at pose  */
/* T_ref with intrinsics K at full resolution; every point p of the new depth  */
/* image, moved by the current estimate T (camera -> world), is projected into */
/* the reference view, paired with the nearest reference pixel, and scored by  */
/* its distance to the plane there, d = (T p - V)^T N.  A Gauss-Newton step     */
/* solves the linearised least squares; levels of a resolution hierarchy are   */
/* visited coarse to fine.  binary64 throughout.                               */
/* Readings (the paper gives the scheme, not these details):                   */
/*   hierarchy: level l keeps every other pixel of level l - 1 in each        */
/*     direction (pixel (u, v) of level l is pixel (2u, 2v) of level l - 1,     */
/*     W_l = ceil(W_{l-1} / 2)), so it is pixel (2^l u, 2^l v) of the input,    */
/*     with intrinsics fx / 2^l, fy / 2^l, cx / 2^l, cy / 2^l.  (A 2 x 2 mean   */
/*     would sit at the half-pixel between four input pixels: at the reference */
/*     pose every coarse point would then project exactly between two          */
/*     reference pixels, and the pairing would be decided by rounding.)        */
/*   pairing: nearest reference pixel floor(x + 1/2), floor(y + 1/2) of the     */
/*     projection with the full-resolution K; a pair counts when both maps are  */
/*     valid there (w > 0) and |T p - V| <= the level's distance threshold;     */
/*   linearisation: T <- (exp([w]x), v) T, so d(w, v) ~ d + w.(P x N) + v.N at  */
/*     P = T p: J = (P x N, N);  A = sum J J^T, g = sum J d, step A x = -g      */
/*     (Cholesky); the rotation exp by Rodrigues' formula;                      */
/*   a level stops early when fewer than min_inliers pairs remain.             */
/* ------------------------------------------------------------------------- */

/* level l of the depth hierarchy (level 0 = the input, as binary64) */
int orc_depth_level(const float *depth, int W, int H, int level, double *out, int *Wl, int *Hl)
{
    const int step = 1 << level;
    const int w = (W + step - 1) / step, h = (H + step - 1) / step;
    for (int v = 0; v < h; v++)
        for (int u = 0; u < w; u++) {
            const double d = depth[(int64_t)(v * step) * W + (int64_t)u * step];
            out[(int64_t)v * w + u] = (isfinite(d) && d > 0.0) ? d : 0.0;
        }
    *Wl = w;
    *Hl = h;
    return 0;
}

static void orc_pose_parts(const double *T, double R[9], double t[3])
{
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) R[3 * i + j] = T[4 * i + j];
        t[i] = T[4 * i + 3];
    }
}

/* sums of one Gauss-Newton step at pose T on hierarchy level `level`:
   sys[0..20] upper triangle of A row by row, sys[21..26] g, sys[27] sum d^2,
   sys[28] number of pairs */
static void orc_icp_sums(const double *dl, int Wl, int Hl, int level, int W, int H, const double *K,
                         const float *V, const float *N, const double *T_ref, const double *T,
                         double dist_thresh, double *sys)
{
    const double sc = ldexp(1.0, -level);
    const double fxl = K[0] * sc, fyl = K[1] * sc, cxl = K[2] * sc, cyl = K[3] * sc;
    double R[9], t[3], Rr[9], tr[3];
    orc_pose_parts(T, R, t);
    orc_pose_parts(T_ref, Rr, tr);
    for (int i = 0; i < 29; i++) sys[i] = 0.0;
    for (int v = 0; v < Hl; v++)
        for (int u = 0; u < Wl; u++) {
            const double d = dl[(int64_t)v * Wl + u];
            if (!(d > 0.0)) continue;
            const double p[3] = {d * (u - cxl) / fxl, d * (v - cyl) / fyl, d};
            double P[3], X[3];
            for (int a = 0; a < 3; a++) P[a] = R[3 * a] * p[0] + R[3 * a + 1] * p[1] + R[3 * a + 2] * p[2] + t[a];
            /* into the reference camera: R_ref^T (P - t_ref) */
            for (int a = 0; a < 3; a++)
                X[a] = Rr[a] * (P[0] - tr[0]) + Rr[3 + a] * (P[1] - tr[1]) + Rr[6 + a] * (P[2] - tr[2]);
            if (!(X[2] > 0.0)) continue;
            const double x = K[0] * X[0] / X[2] + K[2], y = K[1] * X[1] / X[2] + K[3];
            const double xf = floor(x + 0.5), yf = floor(y + 0.5);
            if (!(xf >= 0.0 && xf <= W - 1 && yf >= 0.0 && yf <= H - 1)) continue;
            const int64_t q = (int64_t)yf * W + (int64_t)xf;
            const float *Vq = V + 4 * q, *Nq = N + 4 * q;
            if (!(Vq[3] > 0.0f) || !(Nq[3] > 0.0f)) continue;
            const double diff[3] = {P[0] - Vq[0], P[1] - Vq[1], P[2] - Vq[2]};
            if (sqrt(diff[0] * diff[0] + diff[1] * diff[1] + diff[2] * diff[2]) > dist_thresh) continue;
            const double n[3] = {Nq[0], Nq[1], Nq[2]};
            const double r = diff[0] * n[0] + diff[1] * n[1] + diff[2] * n[2];
            const double J[6] = {P[1] * n[2] - P[2] * n[1], P[2] * n[0] - P[0] * n[2], P[0] * n[1] - P[1] * n[0],
                                 n[0], n[1], n[2]};
            int k = 0;
            for (int i = 0; i < 6; i++)
                for (int j = i; j < 6; j++) sys[k++] += J[i] * J[j];
            for (int i = 0; i < 6; i++) sys[21 + i] += J[i] * r;
            sys[27] += r * r;
            sys[28] += 1.0;
        }
}

int orc_icp_system(const float *depth, int W, int H, const double *K, int level, const float *V,
                   const float *N, const double *T_ref, const double *T, double dist_thresh, double *sys)
{
    double *dl = malloc(sizeof(double) * (size_t)W * H);
    int Wl, Hl;
    if (!dl || orc_depth_level(depth, W, H, level, dl, &Wl, &Hl)) { free(dl); return -1; }
    orc_icp_sums(dl, Wl, Hl, level, W, H, K, V, N, T_ref, T, dist_thresh, sys);
    free(dl);
    return 0;
}

/* solve A x = b, A symmetric positive definite (upper triangle packed row by
   row), by Cholesky; returns -1 when A is not positive definite */
int orc_solve6(const double *Aup, const double *b, double *x)
{
    double A[36], L[36] = {0}, y[6];
    int k = 0;
    for (int i = 0; i < 6; i++)
        for (int j = i; j < 6; j++) { A[6 * i + j] = Aup[k]; A[6 * j + i] = Aup[k]; k++; }
    for (int j = 0; j < 6; j++) {
        double s = A[6 * j + j];
        for (int m = 0; m < j; m++) s -= L[6 * j + m] * L[6 * j + m];
        if (!(s > 0.0)) return -1;
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
    return 0;
}

/* T <- (exp([w]x), v) T, the rotation by Rodrigues' formula */
void orc_pose_step(const double *xi, double *T)
{
    const double w[3] = {xi[0], xi[1], xi[2]};
    const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double Rinc[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (th > 0.0) {
        const double k[3] = {w[0] / th, w[1] / th, w[2] / th};
        const double c = cos(th), s = sin(th), C1 = 1.0 - c;
        const double Kx[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double kk = 0.0;
                for (int m = 0; m < 3; m++) kk += Kx[3 * i + m] * Kx[3 * m + j];
                Rinc[3 * i + j] = (i == j ? 1.0 : 0.0) + s * Kx[3 * i + j] + C1 * kk;
            }
    }
    double R[9], t[3], Rn[9], tn[3];
    orc_pose_parts(T, R, t);
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) {
            double acc = 0.0;
            for (int m = 0; m < 3; m++) acc += Rinc[3 * i + m] * R[3 * m + j];
            Rn[3 * i + j] = acc;
        }
        tn[i] = Rinc[3 * i] * t[0] + Rinc[3 * i + 1] * t[1] + Rinc[3 * i + 2] * t[2] + xi[3 + i];
    }
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) T[4 * i + j] = Rn[3 * i + j];
        T[4 * i + 3] = tn[i];
    }
    T[12] = T[13] = T[14] = 0.0;
    T[15] = 1.0;
}

/* the tracker: levels n_levels - 1 .. 0, iters[l] Gauss-Newton steps on level
   l with distance threshold dist[l]; info = {pairs of the last system,
   RMS distance of the last system, steps taken} */
int orc_track(const float *depth, int W, int H, const double *K, const float *V, const float *N,
              const double *T_ref, const double *T_init, int n_levels, const int *iters,
              const double *dist, int min_inliers, double *T_out, double *info)
{
    double *dl = malloc(sizeof(double) * (size_t)W * H);
    if (!dl) return -1;
    for (int i = 0; i < 16; i++) T_out[i] = T_init[i];
    double sys[29] = {0};
    int steps = 0;
    for (int l = n_levels - 1; l >= 0; l--) {
        int Wl, Hl;
        orc_depth_level(depth, W, H, l, dl, &Wl, &Hl);
        for (int it = 0; it < iters[l]; it++) {
            orc_icp_sums(dl, Wl, Hl, l, W, H, K, V, N, T_ref, T_out, dist[l], sys);
            if (sys[28] < min_inliers) break;
            double b[6], xi[6];
            for (int i = 0; i < 6; i++) b[i] = -sys[21 + i];
            if (orc_solve6(sys, b, xi)) break;
            orc_pose_step(xi, T_out);
            steps++;
        }
    }
    info[0] = sys[28];
    info[1] = sys[28] > 0 ? sqrt(sys[27] / sys[28]) : 0.0;
    info[2] = steps;
    free(dl);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
