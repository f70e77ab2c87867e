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
 * Precision: binary64 throughout, from the definitions, with two exceptions
 * stated where they occur.  (1) The blocks a band segment crosses are a walk
 * specified in binary32 (end points rounded once, crossing parameters
 * recomputed per step), so that the allocated set is one reproducible set.
 * (2) The expected depth range is stored in binary32, rounded outwards.
 * Where floating point decides an integer in the voxel update (pixel, border,
 * band) or in the raycast (nearest voxel, end of range), the binary64 value can
 * lie within the binary32 error bound of a threshold; there both outcomes are
 * correct, and the oracle keeps both (candidate voxel states, branched marches),
 * so a binary32 implementation is judged against every correct result.
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

/* other candidate states of a voxel (see "Decision margins" at the integration) */
#define ORC_MAX_CAND 16
typedef struct {
    int n;             /* states besides the one in the main arrays */
    int overflow;      /* more distinct states arose than are kept */
    double F[ORC_MAX_CAND - 1];
    int32_t W[ORC_MAX_CAND - 1];
    uint8_t C[ORC_MAX_CAND - 1][4];
} orc_cand;

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
    orc_cand ***alt;   /* per block: NULL, or per voxel NULL / the voxel's other states */
    int64_t n_blocks, cap_blocks;
    /* per-frame visibility (one flag per hash entry) and statistics */
    uint8_t *vis;
    int64_t n_vis;
    int64_t dropped_total; /* sum over frames of the distinct blocks dropped */
    int32_t *drop_keys;    /* blocks dropped in the current frame (with repeats) */
    int64_t n_drop, cap_drop;
    int64_t updated_last;
    int64_t ambiguous_last; /* voxels of the last frame with more than one outcome */
    float z_near, z_far;
    /* swapping (section "Swapping"): per block whether it holds a device voxel
     * block and whether the host holds data not yet merged into it, the host
     * copies, the device pool and the per-frame transfer capacities */
    const int32_t *pixel_order; /* visiting order of the allocation's pixels, or NULL (row-major) */
    uint8_t *touch_e, *touch_b;  /* while counting a raycast's reads: entries / buckets read */
    int swap_on;
    uint8_t *dev, *host;
    double *hF;
    int32_t *hW;
    orc_cand ***halt;
    int64_t dev_cap, n_dev, in_cap, out_cap;
    int64_t swapped_in_last, swapped_out_last, swapped_in_total, swapped_out_total, no_block_total;
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
    for (int64_t b = 0; b < sc->n_blocks; b++) {
        if (!sc->alt[b]) continue;
        for (int i = 0; i < SDF_BLOCK3; i++) free(sc->alt[b][i]);
        free(sc->alt[b]);
    }
    free(sc->alt);
    if (sc->halt) {
        for (int64_t b = 0; b < sc->n_blocks; b++) {
            if (!sc->halt[b]) continue;
            for (int i = 0; i < SDF_BLOCK3; i++) free(sc->halt[b][i]);
            free(sc->halt[b]);
        }
    }
    free(sc->halt); free(sc->dev); free(sc->host); free(sc->hF); free(sc->hW);
    free(sc->e); free(sc->vis); free(sc->F); free(sc->W); free(sc->C); free(sc->drop_keys); free(sc);
}

/* the order in which the allocation visits pixels (a permutation of 0..W*H-1
 * for the images that follow, owned by the caller), or NULL for row-major */
void orc_set_pixel_order(orc_scene *sc, const int32_t *order) { sc->pixel_order = order; }

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
    const uint32_t bucket = orc_hash_index(x, y, z, sc->mask);
    int64_t base = (int64_t)bucket * ENTRIES_PER_BUCKET;
    if (sc->touch_b) sc->touch_b[bucket] = 1;   /* counting what a raycast reads */
    int32_t off = 0;
    for (int i = 0; i < ENTRIES_PER_BUCKET; i++) {
        const orc_entry *h = &sc->e[base + i];
        off = h->offset - 1;
        if (h->x == x && h->y == y && h->z == z && h->ptr >= 0) {
            if (sc->touch_e) sc->touch_e[base + i] = 1;
            return base + i;
        }
    }
    while (off >= 0) {
        int64_t idx = ENTRIES_PER_BUCKET * sc->n_buckets + off;
        const orc_entry *h = &sc->e[idx];
        if (h->x == x && h->y == y && h->z == z && h->ptr >= 0) {
            if (sc->touch_e) sc->touch_e[idx] = 1;
            return idx;
        }
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
        orc_cand ***alt = (orc_cand ***)realloc(sc->alt, sizeof(orc_cand **) * (size_t)nc);
        if (!alt) return -2;
        for (int64_t i = sc->cap_blocks; i < nc; i++) alt[i] = NULL;
        sc->alt = alt;
        if (sc->swap_on) {
            uint8_t *dv = (uint8_t *)realloc(sc->dev, (size_t)nc), *hs = (uint8_t *)realloc(sc->host, (size_t)nc);
            if (dv) sc->dev = dv;
            if (hs) sc->host = hs;
            double *hF = (double *)realloc(sc->hF, sizeof(double) * SDF_BLOCK3 * (size_t)nc);
            if (hF) sc->hF = hF;
            int32_t *hW = (int32_t *)realloc(sc->hW, sizeof(int32_t) * SDF_BLOCK3 * (size_t)nc);
            if (hW) sc->hW = hW;
            orc_cand ***ha = (orc_cand ***)realloc(sc->halt, sizeof(orc_cand **) * (size_t)nc);
            if (ha) sc->halt = ha;
            if (!dv || !hs || !hF || !hW || !ha) return -2;
            for (int64_t i = sc->cap_blocks; i < nc; i++) { sc->dev[i] = 0; sc->host[i] = 0; sc->halt[i] = NULL; }
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
    for (int64_t pi = 0; pi < (int64_t)W * H; pi++) {
        {
            const int64_t px = sc->pixel_order ? sc->pixel_order[pi] : pi;
            const int u = (int)(px % W), v = (int)(px / W);
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
/* Integration, section "Integration".  Two steps per voxel v = 8 k + l of a   */
/* visible block k, sitting at world point v s:                                 */
/*  1. the depth sample: the camera point p = M_d (v s) (M_d = T_cw, the       */
/*     world-to-camera pose); nothing when p_z <= 0; the pixel x = fx p_x/p_z + */
/*     cx, y = fy p_y/p_z + cy, nothing outside [1, W-2] x [1, H-2]; the image   */
/*     is read at the nearest pixel ((int)(x + 1/2), (int)(y + 1/2)); nothing    */
/*     when that depth d is invalid; the signed distance along the camera axis  */
/*     eta = d - p_z; nothing behind the band (eta < -mu); else the truncated   */
/*     SDF sample f = min(1, eta / mu);                                         */
/*  2. the running average: F <- (W F + f) / (W + 1), W <- min(W + 1, max_w)    */
/*     (the average divides by the uncapped W + 1).                             */
/* All of it in binary64 from the definitions above.                            */
/*                                                                              */
/* Decision margins.  Floating point decides integers in step 1: whether p is  */
/* in front of the camera, inside the border, which pixel is nearest, whether  */
/* eta is inside the band (and, with colour, inside mu).  A GPU evaluates these */
/* in binary32, so where the binary64 value lies within the binary32 error      */
/* bound tau of a threshold both outcomes are correct readings of the method.   */
/* The oracle then keeps every outcome: a voxel carries a small set of          */
/* candidate states (F, W, colour), the first of them the one the binary64      */
/* decisions take; a candidate follows each outcome of each later frame.  The   */
/* error bounds (u = 2^-24, unit roundoff of binary32) assume an evaluation     */
/* whose error is relative to the camera point itself (a camera-space point    */
/* exact to binary32 within the voxel's block, plus at most 3 x 7 voxel steps), */
/* and a quotient p_x / p_z formed as p_x times a reciprocal of p_z accurate to */
/* one ulp (relative error 3 u: 2 u for the reciprocal, u for the product):     */
/*   e_p   = 1.5 u max|p_a| + 24 u s            per component of p              */
/*   e_x   = fx ((e_p (1 + |X|)) / p_z + 3 u |X|) + u (fx |X| + 2 |x| + |cx|),   */
/*           X = p_x / p_z (likewise y)                                         */
/*   e_eta = e_p + 2 u (|d| + |p_z| + |eta|)                                   */
/* and tau = 2 e (a factor two of headroom).  A voxel whose candidate set would  */
/* exceed ORC_MAX_CAND states keeps the first ORC_MAX_CAND and is marked        */
/* unresolved.                                                                  */
/* ------------------------------------------------------------------------- */
#define ORC_U 0x1p-24

typedef struct {
    orc_cam c;
    const float *depth;
    const uint8_t *rgbx;   /* registered colour image, 4 bytes per pixel, or NULL */
    double mu, s;
    int max_w;
} orc_frame;

static void orc_frame_setup(orc_frame *fr, double s, double mu, int max_w, const float *depth, int W,
                            int H, const double *K, const double *T_wc)
{
    orc_cam_setup(&fr->c, W, H, K, T_wc);
    fr->depth = depth;
    fr->rgbx = NULL;
    fr->mu = mu;
    fr->s = s;
    fr->max_w = max_w;
}

/* one outcome of step 1: no update, or an update with sample f (and, with a
 * colour image, whether the voxel takes the pixel's colour) */
typedef struct {
    int upd, cs;
    double f;
    uint8_t rgb[3];
} orc_outcome;

#define ORC_MAX_OUT 16

static int orc_same_outcome(const orc_outcome *a, const orc_outcome *b)
{
    if (a->upd != b->upd) return 0;
    if (!a->upd) return 1;
    if (a->f != b->f || a->cs != b->cs) return 0;
    return !a->cs || memcmp(a->rgb, b->rgb, 3) == 0;
}

static int orc_add_outcome(orc_outcome *out, int n, const orc_outcome *o)
{
    for (int i = 0; i < n; i++)
        if (orc_same_outcome(out + i, o)) return n;
    if (n < ORC_MAX_OUT) out[n++] = *o;
    return n;
}

/* the outcomes of reading the depth at pixel (ix, iy) for a voxel at camera
 * depth pz (error bound ep); the binary64 decision first when primary */
static int orc_pixel_outcomes(const orc_frame *fr, int ix, int iy, double pz, double ep,
                              orc_outcome *out, int n)
{
    const int64_t pix = (int64_t)iy * fr->c.W + ix;
    const float d = fr->depth[pix];
    orc_outcome o;
    memset(&o, 0, sizeof o);
    if (!(d > 0.0f) || isinf(d)) return orc_add_outcome(out, n, &o);
    const double eta = (double)d - pz;
    const double tau = 2.0 * (ep + 2.0 * ORC_U * (fabs((double)d) + fabs(pz) + fabs(eta)));
    const double mu = fr->mu;
    double f = eta / mu;
    if (f > 1.0) f = 1.0;
    /* the binary64 decision first, then the other side of any threshold within tau */
    const int upd0 = !(eta < -mu);
    for (int k = 0; k < 2; k++) {
        const int upd = k ? !upd0 : upd0;
        if (k && !(fabs(eta + mu) <= tau)) break;
        if (!upd) {
            memset(&o, 0, sizeof o);
            n = orc_add_outcome(out, n, &o);
            continue;
        }
        o.upd = 1;
        o.f = f;
        if (!fr->rgbx) {
            o.cs = 0;
            n = orc_add_outcome(out, n, &o);
            continue;
        }
        memcpy(o.rgb, fr->rgbx + 4 * pix, 3);
        const int cs0 = eta <= mu;
        o.cs = cs0;
        n = orc_add_outcome(out, n, &o);
        if (fabs(eta - mu) <= tau) {
            o.cs = !cs0;
            n = orc_add_outcome(out, n, &o);
        }
    }
    return n;
}

/* step 1 for voxel v (integer voxel coordinates): every outcome within the
 * decision margins, the binary64 one first.  *unresolved is set when a case
 * the margins cannot decide remains (a point within tau of the camera plane). */
static int orc_outcomes(const orc_frame *fr, const int64_t *v, orc_outcome *out, int *unresolved)
{
    const orc_cam *c = &fr->c;
    double vs[3], p[3];
    for (int a = 0; a < 3; a++) vs[a] = (double)v[a] * fr->s;
    for (int a = 0; a < 3; a++)
        p[a] = ((c->Rcw[3 * a] * vs[0] + c->Rcw[3 * a + 1] * vs[1]) + c->Rcw[3 * a + 2] * vs[2]) + c->tcw[a];
    double pm = fabs(p[0]);
    if (fabs(p[1]) > pm) pm = fabs(p[1]);
    if (fabs(p[2]) > pm) pm = fabs(p[2]);
    const double ep = 1.5 * ORC_U * pm + 24.0 * ORC_U * fr->s;
    orc_outcome none;
    memset(&none, 0, sizeof none);
    int n = 0;
    if (!(p[2] > 0.0)) {
        if (fabs(p[2]) <= 2.0 * ep) *unresolved = 1;
        out[0] = none;
        return 1;
    }
    const int z_tie = p[2] <= 2.0 * ep;
    const double X = p[0] / p[2], Y = p[1] / p[2];
    const double x = c->fx * X + c->cx, y = c->fy * Y + c->cy;
    const double tx = 2.0 * (c->fx * ((ep * (1.0 + fabs(X))) / p[2] + 3.0 * ORC_U * fabs(X)) +
                             ORC_U * (c->fx * fabs(X) + 2.0 * fabs(x) + fabs(c->cx)));
    const double ty = 2.0 * (c->fy * ((ep * (1.0 + fabs(Y))) / p[2] + 3.0 * ORC_U * fabs(Y)) +
                             ORC_U * (c->fy * fabs(Y) + 2.0 * fabs(y) + fabs(c->cy)));
    const double xmax = (double)(c->W - 2), ymax = (double)(c->H - 2);
    const int inside = x >= 1.0 && x <= xmax && y >= 1.0 && y <= ymax;
    const int inside_possible = x >= 1.0 - tx && x <= xmax + tx && y >= 1.0 - ty && y <= ymax + ty;
    const int outside_possible = z_tie || x < 1.0 + tx || x > xmax - tx || y < 1.0 + ty || y > ymax - ty;
    if (!inside_possible) {
        out[0] = none;
        return 1;
    }
    /* nearest pixel and the neighbour across a rounding tie, per axis */
    const double hx = x + 0.5, hy = y + 0.5;
    const double ix0 = floor(hx), iy0 = floor(hy);
    int ixs[2] = {(int)ix0, (int)ix0}, iys[2] = {(int)iy0, (int)iy0}, nx = 1, ny = 1;
    if (hx - ix0 <= tx) ixs[nx++] = (int)ix0 - 1;
    else if (ix0 + 1.0 - hx <= tx) ixs[nx++] = (int)ix0 + 1;
    if (hy - iy0 <= ty) iys[ny++] = (int)iy0 - 1;
    else if (iy0 + 1.0 - hy <= ty) iys[ny++] = (int)iy0 + 1;
    if (inside) n = orc_pixel_outcomes(fr, ixs[0], iys[0], p[2], ep, out, n);
    else n = orc_add_outcome(out, n, &none);
    if (outside_possible) n = orc_add_outcome(out, n, &none);
    for (int i = 0; i < nx; i++)
        for (int j = 0; j < ny; j++) {
            if (i == 0 && j == 0 && inside) continue;
            if (ixs[i] < 0 || ixs[i] >= c->W || iys[j] < 0 || iys[j] >= c->H) continue;
            n = orc_pixel_outcomes(fr, ixs[i], iys[j], p[2], ep, out, n);
        }
    return n;
}

/* Colour (readings; the paper shows the voxel type and says a similar function
 * updates the colour): the colour image is registered with the depth image and
 * read at the same pixel; a voxel whose depth update ran takes a colour sample
 * when it lies inside the band, eta <= mu; each channel keeps the running
 * average of its samples rounded to the nearest integer (ties to even), new =
 * round((w_c c + sample) / (w_c + 1)) in exact integer arithmetic, and
 * w_c <- min(w_c + 1, min(max_w, 255)). */
static uint8_t orc_colour_mean(int c, int w, int sample)
{
    const int num = w * c + sample, den = w + 1;
    int q = num / den;
    const int r2 = 2 * (num - q * den);
    if (r2 > den || (r2 == den && (q & 1))) q++;
    return (uint8_t)q;
}

/* step 2: the running average of one candidate state */
static void orc_average(const orc_frame *fr, const orc_outcome *o, double *F, int32_t *Wt, uint8_t *C)
{
    if (!o->upd) return;
    const double w = (double)(*Wt);
    *F = (w * (*F) + o->f) / (w + 1.0);
    const int nw = *Wt + 1;
    *Wt = nw < fr->max_w ? nw : fr->max_w;
    if (C && o->cs) {
        const int wc = C[3];
        for (int ch = 0; ch < 3; ch++) C[ch] = orc_colour_mean(C[ch], wc, o->rgb[ch]);
        const int cap = fr->max_w < 255 ? fr->max_w : 255;
        C[3] = (uint8_t)(wc + 1 < cap ? wc + 1 : cap);
    }
}

/* the voxel's state(s) after one frame.  Main arrays hold the first candidate;
 * *alt (NULL when the voxel has one state) the others.  Returns 1 when the
 * first candidate was updated. */
static int orc_voxel_frame(const orc_frame *fr, const int64_t *v, double *F, int32_t *Wt, uint8_t *C,
                           orc_cand **alt, int *ambiguous)
{
    orc_outcome out[ORC_MAX_OUT];
    int unresolved = 0;
    const int n = orc_outcomes(fr, v, out, &unresolved);
    *ambiguous = n > 1 || unresolved;
    if (n == 1 && !*alt && !unresolved) {
        orc_average(fr, &out[0], F, Wt, C);
        return out[0].upd;
    }
    /* every candidate state follows every outcome; equal states merge */
    double sF[ORC_MAX_CAND];
    int32_t sW[ORC_MAX_CAND];
    uint8_t sC[ORC_MAX_CAND][4];
    int ns = 1;
    sF[0] = *F; sW[0] = *Wt;
    if (C) memcpy(sC[0], C, 4); else memset(sC[0], 0, 4);
    int over = unresolved;
    if (*alt) {
        over |= (*alt)->overflow;
        for (int i = 0; i < (*alt)->n; i++, ns++) {
            sF[ns] = (*alt)->F[i]; sW[ns] = (*alt)->W[i]; memcpy(sC[ns], (*alt)->C[i], 4);
        }
    }
    double nF[ORC_MAX_CAND];
    int32_t nW[ORC_MAX_CAND];
    uint8_t nC[ORC_MAX_CAND][4];
    int nn = 0;
    for (int i = 0; i < ns; i++)
        for (int k = 0; k < n; k++) {
            double f2 = sF[i];
            int32_t w2 = sW[i];
            uint8_t c2[4];
            memcpy(c2, sC[i], 4);
            orc_average(fr, &out[k], &f2, &w2, C ? c2 : NULL);
            int dup = 0;
            for (int j = 0; j < nn && !dup; j++)
                dup = nW[j] == w2 && fabs(nF[j] - f2) <= 1e-12 && memcmp(nC[j], c2, 4) == 0;
            if (dup) continue;
            if (nn == ORC_MAX_CAND) { over = 1; continue; }
            nF[nn] = f2; nW[nn] = w2; memcpy(nC[nn], c2, 4);
            nn++;
        }
    *F = nF[0]; *Wt = nW[0];
    if (C) memcpy(C, nC[0], 4);
    if (nn > 1 || over) {
        if (!*alt) {
            *alt = (orc_cand *)calloc(1, sizeof(orc_cand));
            if (!*alt) return out[0].upd;   /* out of memory: the voxel loses its other states */
        }
        (*alt)->n = nn - 1;
        (*alt)->overflow = over;
        for (int j = 1; j < nn; j++) {
            (*alt)->F[j - 1] = nF[j]; (*alt)->W[j - 1] = nW[j]; memcpy((*alt)->C[j - 1], nC[j], 4);
        }
    } else if (*alt) {
        free(*alt);
        *alt = NULL;
    }
    return out[0].upd;
}

/* integration over the visible blocks of the current frame */
static int64_t orc_integrate_visible(orc_scene *sc, const orc_frame *fr)
{
    int64_t n = 0;
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(sc->n_vis + 1));
    if (!list) return -1;
    for (int64_t i = 0; i < sc->n_entries; i++)
        if (sc->vis[i] && (!sc->swap_on || sc->dev[sc->e[i].ptr])) list[n++] = i;
    int64_t updated = 0, ambiguous = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : updated, ambiguous)
    for (int64_t j = 0; j < n; j++) {
        const orc_entry *h = &sc->e[list[j]];
        const int64_t b = h->ptr;
        double *F = sc->F + b * SDF_BLOCK3;
        int32_t *W = sc->W + b * SDF_BLOCK3;
        uint8_t *Cb = sc->C ? sc->C + 4 * b * SDF_BLOCK3 : NULL;
        for (int lz = 0; lz < 8; lz++)
            for (int ly = 0; ly < 8; ly++)
                for (int lx = 0; lx < 8; lx++) {
                    const int li = lx + 8 * ly + 64 * lz;
                    const int64_t v[3] = {8 * (int64_t)h->x + lx, 8 * (int64_t)h->y + ly, 8 * (int64_t)h->z + lz};
                    orc_cand *alt = sc->alt[b] ? sc->alt[b][li] : NULL;
                    const orc_cand *was = alt;
                    int amb = 0;
                    updated += orc_voxel_frame(fr, v, &F[li], &W[li], Cb ? Cb + 4 * li : NULL, &alt, &amb);
                    ambiguous += amb;
                    if (alt != was) {
                        if (!sc->alt[b]) sc->alt[b] = (orc_cand **)calloc(SDF_BLOCK3, sizeof(orc_cand *));
                        if (sc->alt[b]) sc->alt[b][li] = alt;
                        else free(alt);
                    }
                }
    }
    free(list);
    sc->updated_last = updated;
    sc->ambiguous_last = ambiguous;
    return updated;
}

/* one frame: allocation then integration.  Returns the number of updated voxels. */
static void orc_swap_blocks_for_visible(orc_scene *sc);
static int orc_swap(orc_scene *sc);

int64_t orc_integrate(orc_scene *sc, const float *depth, int W, int H, const double *K,
                      const double *T_wc)
{
    if (orc_allocate(sc, depth, W, H, K, T_wc) < 0) return -1;
    if (sc->swap_on) orc_swap_blocks_for_visible(sc);
    orc_frame fr;
    orc_frame_setup(&fr, sc->s, sc->mu, sc->max_w, depth, W, H, K, T_wc);
    const int64_t upd = orc_integrate_visible(sc, &fr);
    if (sc->swap_on && orc_swap(sc)) return -1;
    return upd;
}

/* colour voxels: storage for every block, present and future (colour (0, 0, 0),
   weight 0) */
int orc_enable_colour(orc_scene *sc)
{
    if (sc->C) return 0;
    if (sc->swap_on) return -1;
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
    orc_frame_setup(&fr, sc->s, sc->mu, sc->max_w, depth, W, H, K, T_wc);
    fr.rgbx = rgbx;
    return orc_integrate_visible(sc, &fr);
}

/* Loading a volume (the inverse of orc_export): each block key is found or
 * inserted (section "Hash Table Operations"), its voxels take the given F and
 * W (colour, when enabled, is cleared), and any other candidate states it had
 * are dropped.  The loaded blocks become the visible set, as if one frame had
 * visited them (the expected depth range projects them).  A block that finds
 * no entry is dropped and counted.  Returns the number of blocks loaded. */
int64_t orc_import(orc_scene *sc, const int32_t *coords, const double *F, const int32_t *Wt, int64_t n)
{
    if (sc->swap_on) return -1;
    sc->n_drop = 0;
    memset(sc->vis, 0, (size_t)sc->n_entries);
    int64_t loaded = 0;
    for (int64_t i = 0; i < n; i++) {
        const int64_t e = orc_insert(sc, coords[3 * i], coords[3 * i + 1], coords[3 * i + 2]);
        if (e < 0) continue;
        sc->vis[e] = 1;
        const int64_t b = sc->e[e].ptr;
        memcpy(sc->F + b * SDF_BLOCK3, F + i * SDF_BLOCK3, sizeof(double) * SDF_BLOCK3);
        memcpy(sc->W + b * SDF_BLOCK3, Wt + i * SDF_BLOCK3, sizeof(int32_t) * SDF_BLOCK3);
        if (sc->C) memset(sc->C + 4 * b * SDF_BLOCK3, 0, 4 * SDF_BLOCK3);
        if (sc->alt[b]) {
            for (int li = 0; li < SDF_BLOCK3; li++) free(sc->alt[b][li]);
            free(sc->alt[b]);
            sc->alt[b] = NULL;
        }
        loaded++;
    }
    if (sc->n_drop > 0) {
        qsort(sc->drop_keys, (size_t)sc->n_drop, sizeof(int32_t) * 3, orc_key_cmp3);
        int64_t u = 1;
        for (int64_t i = 1; i < sc->n_drop; i++)
            u += orc_key_cmp3(sc->drop_keys + 3 * i, sc->drop_keys + 3 * (i - 1)) != 0;
        sc->dropped_total += u;
    }
    int64_t nv = 0;
    for (int64_t i = 0; i < sc->n_entries; i++) nv += sc->vis[i];
    sc->n_vis = nv;
    sc->updated_last = 0;
    sc->ambiguous_last = 0;
    return loaded;
}

/* ------------------------------------------------------------------------- */
/* Swapping, section "Swapping".  The host can hold a copy of every allocated  */
/* block (the paper's host voxel block array is indexed by hash entry; here by */
/* the oracle's block index, which is one per entry), the device a pool of     */
/* dev_cap voxel blocks.  Per frame:                                            */
/*  1. allocation as always; then every visible block without a device block   */
/*     takes a fresh one (F = 1, W = 0) from the pool, in entry order; with    */
/*     the pool empty it is not integrated in this frame (counted);            */
/*  2. integration of the visible blocks that hold a device block (new data    */
/*     is fused whether or not the block's host copy has come back yet);       */
/*  3. swap in: of the blocks whose host copy is not yet merged, the first     */
/*     in_cap in key order (x, then y, then z) are merged into their device     */
/*     block, the secondary integration: F = (W_d F_d + W_h F_h)/(W_d + W_h),   */
/*     W = min(W_d + W_h, max_w) (two running averages joined by their weights; */
/*     unchanged when both weights are 0);                                     */
/*  4. swap out: of the device blocks that were not visible in this frame and  */
/*     have nothing left to merge, the first out_cap in key order go to the    */
/*     host and their device blocks back to the pool.                          */
/* Readings: the transfers are taken in key order, so the schedule does not    */
/* depend on where a block sits in memory; the transfer buffers are as large   */
/* as in_cap and out_cap blocks.  A voxel's other candidate states (decision   */
/* margins) travel with its copy and combine pairwise at the merge.           */
/* ------------------------------------------------------------------------- */
int orc_enable_swapping(orc_scene *sc, int64_t dev_cap, int64_t in_cap, int64_t out_cap)
{
    if (sc->swap_on || dev_cap < 1 || in_cap < 0 || out_cap < 0 || sc->C) return -1;
    const int64_t nc = sc->cap_blocks ? sc->cap_blocks : 1;
    sc->dev = (uint8_t *)calloc((size_t)nc, 1);
    sc->host = (uint8_t *)calloc((size_t)nc, 1);
    sc->hF = (double *)malloc(sizeof(double) * SDF_BLOCK3 * (size_t)nc);
    sc->hW = (int32_t *)malloc(sizeof(int32_t) * SDF_BLOCK3 * (size_t)nc);
    sc->halt = (orc_cand ***)calloc((size_t)nc, sizeof(orc_cand **));
    if (!sc->dev || !sc->host || !sc->hF || !sc->hW || !sc->halt) return -1;
    /* blocks allocated before: each holds a device block (taken from the pool) */
    if (sc->n_blocks > dev_cap) return -1;
    for (int64_t b = 0; b < sc->n_blocks; b++) sc->dev[b] = 1;
    sc->n_dev = sc->n_blocks;
    sc->dev_cap = dev_cap;
    sc->in_cap = in_cap;
    sc->out_cap = out_cap;
    sc->swap_on = 1;
    return 0;
}

static void orc_free_alts(orc_cand **a)
{
    if (!a) return;
    for (int i = 0; i < SDF_BLOCK3; i++) free(a[i]);
    free(a);
}

/* step 1: a device block for every visible block that has none */
static void orc_swap_blocks_for_visible(orc_scene *sc)
{
    for (int64_t i = 0; i < sc->n_entries; i++) {
        if (!sc->vis[i]) continue;
        const int64_t b = sc->e[i].ptr;
        if (sc->dev[b]) continue;
        if (sc->n_dev >= sc->dev_cap) { sc->no_block_total++; continue; }
        sc->dev[b] = 1;
        sc->n_dev++;
        for (int l = 0; l < SDF_BLOCK3; l++) { sc->F[b * SDF_BLOCK3 + l] = 1.0; sc->W[b * SDF_BLOCK3 + l] = 0; }
        orc_free_alts(sc->alt[b]);
        sc->alt[b] = NULL;
    }
}

static void orc_merge_state(int max_w, double Fd, int32_t Wd, double Fh, int32_t Wh, double *F, int32_t *W)
{
    const int32_t w = Wd + Wh;
    if (w == 0) { *F = Fd; *W = 0; return; }
    *F = ((double)Wd * Fd + (double)Wh * Fh) / (double)w;
    *W = w < max_w ? w : max_w;
}

/* every state of a voxel of block b: the device copy merged with the host copy
 * when both exist (all pairs of their candidates, the first pair first), else
 * the one copy there is.  Returns the number of states (<= ORC_MAX_CAND);
 * *over when more arose or either copy was unresolved. */
static int orc_voxel_states(const orc_scene *sc, int64_t b, int li, double *F, int32_t *W, int *over)
{
    const int64_t k = b * SDF_BLOCK3 + li;
    const orc_cand *ad = sc->alt[b] ? sc->alt[b][li] : NULL;
    const int has_host = sc->swap_on && sc->host[b];
    const int has_dev = !sc->swap_on || sc->dev[b];
    *over = 0;
    if (!has_host || !has_dev) {
        const double *mF = has_host ? sc->hF : sc->F;
        const int32_t *mW = has_host ? sc->hW : sc->W;
        const orc_cand *a = has_host ? (sc->halt[b] ? sc->halt[b][li] : NULL) : ad;
        F[0] = mF[k]; W[0] = mW[k];
        int n = 1;
        if (a) {
            *over = a->overflow;
            for (int j = 0; j < a->n; j++, n++) { F[n] = a->F[j]; W[n] = a->W[j]; }
        }
        return n;
    }
    const orc_cand *ah = sc->halt[b] ? sc->halt[b][li] : NULL;
    double dF[ORC_MAX_CAND], hF[ORC_MAX_CAND];
    int32_t dW[ORC_MAX_CAND], hW[ORC_MAX_CAND];
    int nd = 1, nh = 1;
    dF[0] = sc->F[k]; dW[0] = sc->W[k];
    hF[0] = sc->hF[k]; hW[0] = sc->hW[k];
    if (ad) { *over |= ad->overflow; for (int j = 0; j < ad->n; j++, nd++) { dF[nd] = ad->F[j]; dW[nd] = ad->W[j]; } }
    if (ah) { *over |= ah->overflow; for (int j = 0; j < ah->n; j++, nh++) { hF[nh] = ah->F[j]; hW[nh] = ah->W[j]; } }
    int n = 0;
    for (int i = 0; i < nd; i++)
        for (int j = 0; j < nh; j++) {
            double f;
            int32_t w;
            orc_merge_state(sc->max_w, dF[i], dW[i], hF[j], hW[j], &f, &w);
            int dup = 0;
            for (int q = 0; q < n && !dup; q++) dup = W[q] == w && fabs(F[q] - f) <= 1e-12;
            if (dup) continue;
            if (n == ORC_MAX_CAND) { *over = 1; continue; }
            F[n] = f; W[n] = w;
            n++;
        }
    return n;
}

static const orc_scene *orc_sort_sc;
static int orc_block_key_cmp(const void *a, const void *b)
{
    /* blocks by key (x, y, z) through the key of any entry pointing at them */
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    const orc_entry *p = &orc_sort_sc->e[x[1]], *q = &orc_sort_sc->e[y[1]];
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    if (p->y != q->y) return p->y < q->y ? -1 : 1;
    if (p->z != q->z) return p->z < q->z ? -1 : 1;
    return 0;
}

/* steps 3 and 4 (after the integration) */
static int orc_swap(orc_scene *sc)
{
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)(sc->n_blocks + 1));
    if (!cand) return -1;
    /* 3. swap in: merge pending host copies */
    int64_t n = 0;
    for (int64_t i = 0; i < sc->n_entries; i++) {
        const int64_t b = sc->e[i].ptr;
        if (b >= 0 && sc->dev[b] && sc->host[b]) { cand[2 * n] = b; cand[2 * n + 1] = i; n++; }
    }
    orc_sort_sc = sc;
    qsort(cand, (size_t)n, 2 * sizeof(int64_t), orc_block_key_cmp);
    const int64_t nin = n < sc->in_cap ? n : sc->in_cap;
    for (int64_t j = 0; j < nin; j++) {
        const int64_t b = cand[2 * j];
        orc_cand **na = NULL;
        for (int li = 0; li < SDF_BLOCK3; li++) {
            double F[ORC_MAX_CAND];
            int32_t W[ORC_MAX_CAND];
            int over = 0;
            const int ns = orc_voxel_states(sc, b, li, F, W, &over);
            sc->F[b * SDF_BLOCK3 + li] = F[0];
            sc->W[b * SDF_BLOCK3 + li] = W[0];
            if (ns > 1 || over) {
                if (!na) na = (orc_cand **)calloc(SDF_BLOCK3, sizeof(orc_cand *));
                orc_cand *c = na ? (orc_cand *)calloc(1, sizeof(orc_cand)) : NULL;
                if (c) {
                    c->n = ns - 1;
                    c->overflow = over;
                    for (int q = 1; q < ns; q++) { c->F[q - 1] = F[q]; c->W[q - 1] = W[q]; }
                    na[li] = c;
                }
            }
        }
        orc_free_alts(sc->alt[b]);
        sc->alt[b] = na;
        orc_free_alts(sc->halt[b]);
        sc->halt[b] = NULL;
        sc->host[b] = 0;
    }
    sc->swapped_in_last = nin;
    sc->swapped_in_total += nin;
    /* 4. swap out: device blocks not visible in this frame, nothing to merge */
    n = 0;
    for (int64_t i = 0; i < sc->n_entries; i++) {
        const int64_t b = sc->e[i].ptr;
        if (b >= 0 && sc->dev[b] && !sc->host[b] && !sc->vis[i]) { cand[2 * n] = b; cand[2 * n + 1] = i; n++; }
    }
    qsort(cand, (size_t)n, 2 * sizeof(int64_t), orc_block_key_cmp);
    const int64_t nout = n < sc->out_cap ? n : sc->out_cap;
    for (int64_t j = 0; j < nout; j++) {
        const int64_t b = cand[2 * j];
        memcpy(sc->hF + b * SDF_BLOCK3, sc->F + b * SDF_BLOCK3, sizeof(double) * SDF_BLOCK3);
        memcpy(sc->hW + b * SDF_BLOCK3, sc->W + b * SDF_BLOCK3, sizeof(int32_t) * SDF_BLOCK3);
        orc_free_alts(sc->halt[b]);
        sc->halt[b] = sc->alt[b];
        sc->alt[b] = NULL;
        sc->host[b] = 1;
        sc->dev[b] = 0;
        sc->n_dev--;
    }
    sc->swapped_out_last = nout;
    sc->swapped_out_total += nout;
    free(cand);
    return 0;
}

/* swapping statistics: device blocks in use, blocks whose data is on the host
 * only, blocks with a host copy still to merge, swapped in / out in the last
 * frame, totals, visible blocks left without a device block (total) */
void orc_swap_stats(const orc_scene *sc, int64_t *out)
{
    int64_t host_only = 0, pending = 0;
    for (int64_t b = 0; sc->swap_on && b < sc->n_blocks; b++) {
        host_only += sc->host[b] && !sc->dev[b];
        pending += sc->host[b] && sc->dev[b];
    }
    out[0] = sc->n_dev; out[1] = host_only; out[2] = pending;
    out[3] = sc->swapped_in_last; out[4] = sc->swapped_out_last;
    out[5] = sc->swapped_in_total; out[6] = sc->swapped_out_total; out[7] = sc->no_block_total;
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
 * voxels (last frame), voxels of the last frame whose update had more than one
 * outcome within the decision margins */
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
    out[6] = sc->ambiguous_last;
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
        const int64_t b = tmp[4 * i + 3];
        if (sc->swap_on) {   /* the block's state wherever it is (merged when both copies exist) */
            for (int li = 0; li < SDF_BLOCK3; li++) {
                double sF[ORC_MAX_CAND];
                int32_t sW[ORC_MAX_CAND];
                int over;
                orc_voxel_states(sc, b, li, sF, sW, &over);
                if (F) F[i * SDF_BLOCK3 + li] = sF[0];
                if (Wt) Wt[i * SDF_BLOCK3 + li] = sW[0];
            }
            continue;
        }
        if (F) memcpy(F + i * SDF_BLOCK3, sc->F + b * SDF_BLOCK3, sizeof(double) * SDF_BLOCK3);
        if (Wt) memcpy(Wt + i * SDF_BLOCK3, sc->W + b * SDF_BLOCK3, sizeof(int32_t) * SDF_BLOCK3);
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

/* the voxels with more than one candidate state (see "Decision margins" at the
 * integration): per state besides the first one row key[4] = (block x, y, z,
 * in-block index) with its F, W and colour (r, g, b, colour weight; zeros
 * without colour); unresolved[i] = 1 when the voxel had more states than kept
 * or a case the margins cannot decide.  NULL key counts.  Returns the rows. */
int64_t orc_export_candidates(const orc_scene *sc, int32_t *key, double *F, int32_t *Wt, uint8_t *rgbw,
                              uint8_t *unresolved, int64_t cap)
{
    int64_t n = 0;
    for (int64_t i = 0; i < sc->n_entries; i++) {
        const int32_t b = sc->e[i].ptr;
        if (b < 0) continue;
        if (sc->swap_on) {   /* states of the block wherever it is */
            if (!sc->alt[b] && !sc->halt[b]) continue;
            for (int li = 0; li < SDF_BLOCK3; li++) {
                double sF[ORC_MAX_CAND];
                int32_t sW[ORC_MAX_CAND];
                int over;
                const int ns = orc_voxel_states(sc, b, li, sF, sW, &over);
                if (ns < 2 && !over) continue;
                const int rows = ns > 1 ? ns - 1 : 1;
                for (int r = 0; r < rows; r++, n++) {
                    if (!key || n >= cap) continue;
                    key[4 * n] = sc->e[i].x; key[4 * n + 1] = sc->e[i].y; key[4 * n + 2] = sc->e[i].z;
                    key[4 * n + 3] = li;
                    F[n] = ns > 1 ? sF[r + 1] : sF[0];
                    Wt[n] = ns > 1 ? sW[r + 1] : sW[0];
                    memset(rgbw + 4 * n, 0, 4);
                    unresolved[n] = (uint8_t)over;
                }
            }
            continue;
        }
        if (!sc->alt[b]) continue;
        for (int li = 0; li < SDF_BLOCK3; li++) {
            const orc_cand *cd = sc->alt[b][li];
            if (!cd) continue;
            const int rows = cd->n > 0 ? cd->n : 1;   /* an unresolved voxel with one state: one row */
            for (int r = 0; r < rows; r++, n++) {
                if (!key || n >= cap) continue;
                key[4 * n] = sc->e[i].x; key[4 * n + 1] = sc->e[i].y; key[4 * n + 2] = sc->e[i].z;
                key[4 * n + 3] = li;
                const int has = cd->n > 0;
                F[n] = has ? cd->F[r] : sc->F[(int64_t)b * SDF_BLOCK3 + li];
                Wt[n] = has ? cd->W[r] : sc->W[(int64_t)b * SDF_BLOCK3 + li];
                if (has) memcpy(rgbw + 4 * n, cd->C[r], 4);
                else if (sc->C) memcpy(rgbw + 4 * n, sc->C + 4 * ((int64_t)b * SDF_BLOCK3 + li), 4);
                else memset(rgbw + 4 * n, 0, 4);
                unresolved[n] = (uint8_t)cd->overflow;
            }
        }
    }
    return n;
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
    orc_frame_setup(&fr, sc->s, sc->mu, sc->max_w, depth, W, H, K, T_wc);
    int64_t upd = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!active[i]) continue;
        const int64_t v[3] = {vox[3 * i], vox[3 * i + 1], vox[3 * i + 2]};
        orc_outcome out[ORC_MAX_OUT];
        int unresolved = 0;
        orc_outcomes(&fr, v, out, &unresolved);
        orc_average(&fr, &out[0], &F[i], &Wt[i], NULL);
        upd += out[0].upd;
    }
    return upd;
}

/* step 1 alone for one voxel: every outcome within the decision margins (the
 * binary64 one first), for checks of the margins.  upd[i], f[i] per outcome;
 * returns their number, negative when a case is unresolved. */
int orc_voxel_outcomes(const orc_scene *sc, const float *depth, int W, int H, const double *K,
                       const double *T_wc, const int32_t *vox, int32_t *upd, double *f)
{
    orc_frame fr;
    orc_frame_setup(&fr, sc->s, sc->mu, sc->max_w, depth, W, H, K, T_wc);
    const int64_t v[3] = {vox[0], vox[1], vox[2]};
    orc_outcome out[ORC_MAX_OUT];
    int unresolved = 0;
    const int n = orc_outcomes(&fr, v, out, &unresolved);
    for (int i = 0; i < n; i++) { upd[i] = out[i].upd; f[i] = out[i].f; }
    return unresolved ? -n : n;
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
    orc_frame_setup(&fr, dv->s, dv->mu, dv->max_w, depth, W, H, K, T_wc);
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
                int32_t k[3];
                for (int a = 0; a < 3; a++) k[a] = (int32_t)fdiv8(v[a]);
                if (bm && !bm[(k[0] - kb0[0]) + kn[0] * ((k[1] - kb0[1]) + kn[1] * (k[2] - kb0[2]))])
                    continue;
                int64_t i = ix + dv->n[0] * (iy + dv->n[1] * iz);
                /* the binary64 decisions (the first candidate of the hashed volume) */
                orc_outcome out[ORC_MAX_OUT];
                int unresolved = 0;
                orc_outcomes(&fr, v, out, &unresolved);
                orc_average(&fr, &out[0], &dv->F[i], &dv->W[i], NULL);
                int u = out[0].upd;
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
static double orc_voxel_F(const orc_scene *sc, int32_t vx, int32_t vy, int32_t vz)
{
    int32_t k[3] = {(int32_t)fdiv8(vx), (int32_t)fdiv8(vy), (int32_t)fdiv8(vz)};
    int64_t e = orc_find(sc, k[0], k[1], k[2]);
    if (e < 0 || (sc->swap_on && !sc->dev[sc->e[e].ptr])) return 1.0;
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

/* Decision margins of the march.  The search reads F at the nearest lattice
 * voxel, an integer decided by rounding; a GPU marches in binary32.  Where a
 * sample's coordinate lies within the binary32 error bound tau of a rounding
 * boundary and the neighbouring voxel reads differently (found or not, or
 * another F), both reads are correct, and the oracle follows both: the march
 * becomes a small tree of paths whose outcomes (miss, or the hit after the
 * refinement) are all correct results of the method.  Likewise at the end of
 * the range.  The bound, in voxel units, after k updates of t (each rounded to
 * binary32, relative error u = 2^-24, plus the sample position's own
 * roundings): tau = 2 (u (k + 2) T / s + u (|o| / s + |q|)), T = the range end
 * in metres, o the ray origin, q = p / s.  The first path is the one the
 * binary64 reads take. */
enum { ORC_MAX_PATHS = 256, ORC_RAY_ALT = 8 };

typedef struct {
    double t;
    int state, fine_miss, it, k;   /* k: updates of t so far */
    int forced;                    /* the next sample reads voxel fv (a branch) */
    int32_t fv[3];
    int past_end;                  /* the next end-of-range test is taken as "inside" */
} orc_mstate;

typedef struct {
    int hit;
    double t;
} orc_mout;

static int orc_read_voxel(const orc_scene *sc, const int32_t *n, double *F)
{
    const int32_t k[3] = {(int32_t)fdiv8(n[0]), (int32_t)fdiv8(n[1]), (int32_t)fdiv8(n[2])};
    int64_t e = orc_find(sc, k[0], k[1], k[2]);
    /* with swapping the raycast sees the blocks held on the device only */
    if (e < 0 || (sc->swap_on && !sc->dev[sc->e[e].ptr])) { *F = 1.0; return 0; }
    int li = (n[0] - 8 * k[0]) + 8 * (n[1] - 8 * k[1]) + 64 * (n[2] - 8 * k[2]);
    *F = sc->F[(int64_t)sc->e[e].ptr * SDF_BLOCK3 + li];
    return 1;
}

/* one path from state st until it ends: returns the outcome; pushes the other
 * branches it meets onto the stack (as long as there is room) */
static orc_mout orc_march_path(const orc_scene *sc, const orc_ray *r, orc_mstate st, orc_mstate *stack,
                               int *sp, int *flags, int *steps, int branching)
{
    const double bs = 8.0 * sc->s;
    const int fine_budget = (int)ceil(bs / sc->mu) + 1;
    const int cap = (int)((r->t_far - r->t_near) / sc->s) * 4 + 1000;
    double omax = fabs(r->o[0]);
    if (fabs(r->o[1]) > omax) omax = fabs(r->o[1]);
    if (fabs(r->o[2]) > omax) omax = fabs(r->o[2]);
    orc_mout res = {0, 0.0};
    double t = st.t;
    int state = st.state, fine_miss = st.fine_miss, it = st.it, k = st.k;
    for (; it < cap; it++) {
        const double tau_vox = 2.0 * (ORC_U * fmin((double)k + 2.0, 2.0 + 3.0 * sqrt((double)k + 1.0)) * (r->t_far / sc->s) + ORC_U * omax / sc->s);
        /* end of the range */
        const double tau_t = tau_vox * sc->s + 2.0 * ORC_U * r->t_far;
        if (!(t < r->t_far)) {
            if (st.past_end) st.past_end = 0;
            else {
                if (branching && fabs(t - r->t_far) <= tau_t && *sp < ORC_MAX_PATHS) {
                    orc_mstate b = {t, state, fine_miss, it, k, 0, {0, 0, 0}, 1};
                    stack[(*sp)++] = b;
                } else if (branching && fabs(t - r->t_far) <= tau_t) *flags |= 8;
                break;
            }
        } else if (branching && r->t_far - t <= tau_t) {
            /* the other side: the range ended here (a miss) */
            if (*sp < ORC_MAX_PATHS) {
                orc_mstate b = {r->t_far, ORC_COARSE, 0, cap, k, 0, {0, 0, 0}, 0};
                stack[(*sp)++] = b;
            } else *flags |= 8;
        }
        double p[3] = {r->o[0] + t * r->d[0], r->o[1] + t * r->d[1], r->o[2] + t * r->d[2]};
        int32_t nv[3];
        double q[3];
        int ok = 1;
        for (int a = 0; a < 3; a++) {
            q[a] = p[a] / sc->s;
            const double h = floor(q[a] + 0.5);
            if (!(h > -262000.0 && h < 262000.0)) ok = 0;
            nv[a] = ok ? (int32_t)h : 0;
        }
        double F = 1.0;
        int found = 0;
        if (st.forced) {
            memcpy(nv, st.fv, sizeof nv);
            st.forced = 0;
            found = orc_read_voxel(sc, nv, &F);
        } else if (ok) {
            found = orc_read_voxel(sc, nv, &F);
            if (branching) {
                /* neighbours across rounding boundaries within tau */
                const double qm = fabs(q[0]) > fabs(q[1]) ? (fabs(q[0]) > fabs(q[2]) ? fabs(q[0]) : fabs(q[2]))
                                                          : (fabs(q[1]) > fabs(q[2]) ? fabs(q[1]) : fabs(q[2]));
                const double tau = tau_vox + 2.0 * ORC_U * qm;
                int alt[3] = {0, 0, 0}, na = 0;
                for (int a = 0; a < 3; a++) {
                    const double fr = (q[a] + 0.5) - floor(q[a] + 0.5);
                    if (fr <= tau) alt[a] = -1;
                    else if (1.0 - fr <= tau) alt[a] = 1;
                    na += alt[a] != 0;
                }
                for (int m = 1; na && m < 8; m++) {
                    int use = 1;
                    int32_t v2[3];
                    for (int a = 0; a < 3; a++) {
                        const int bit = (m >> a) & 1;
                        if (bit && !alt[a]) use = 0;
                        v2[a] = nv[a] + (bit ? alt[a] : 0);
                    }
                    if (!use) continue;
                    double F2;
                    const int f2 = orc_read_voxel(sc, v2, &F2);
                    if (f2 == found && (!found || F2 == F)) continue;   /* reads the same */
                    if (*sp < ORC_MAX_PATHS) {
                        orc_mstate b = {t, state, fine_miss, it, k, 1, {v2[0], v2[1], v2[2]}, 0};
                        stack[(*sp)++] = b;
                    } else *flags |= 8;
                }
            }
        }
        if (found && fabs(F) < 1e-4 && state != ORC_COARSE) *flags |= 1;
        const double t_before = t;
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
        if (t != t_before) k++;
        if (state == ORC_BEHIND) break;
    }
    if (steps) *steps = it;
    if (it >= cap) *flags |= 2;
    if (state != ORC_BEHIND) return res;
    for (int j = 0; j < 2; j++) {
        double p[3] = {r->o[0] + t * r->d[0], r->o[1] + t * r->d[1], r->o[2] + t * r->d[2]};
        t += orc_read_trilinear(sc, p) * sc->mu;
    }
    res.hit = 1;
    res.t = t;
    return res;
}

/* all outcomes of one ray: out[0] the binary64 path's, then the distinct
 * others (at most cap_out); flags bit 0: a sign decision had |F_n| < 1e-4,
 * bit 1: iteration cap reached, bit 2: other outcomes exist, bit 3: more
 * branches than followed (unresolved) */
static int orc_march_all(const orc_scene *sc, const orc_ray *r, orc_mout *out, int cap_out, int *flags,
                         int *steps, int branching)
{
    orc_mstate stack[ORC_MAX_PATHS];
    int sp = 0, n = 0, paths = 0;
    *flags = 0;
    orc_mstate st0 = {r->t_near, ORC_COARSE, 0, 0, 0, 0, {0, 0, 0}, 0};
    out[n++] = orc_march_path(sc, r, st0, stack, &sp, flags, steps, branching);
    while (sp > 0) {
        orc_mstate st = stack[--sp];
        if (++paths > 4 * ORC_MAX_PATHS) { *flags |= 8; break; }
        int fl = 0;
        const orc_mout o = orc_march_path(sc, r, st, stack, &sp, &fl, NULL, branching);
        *flags |= fl & 8;
        int dup = 0;
        for (int i = 0; i < n && !dup; i++)
            dup = out[i].hit == o.hit && (!o.hit || fabs(out[i].t - o.t) <= 1e-5);
        if (dup) continue;
        if (n < cap_out) out[n++] = o;
        else *flags |= 8;
    }
    if (n > 1) *flags |= 4;
    return n;
}

/* normal at a hit: central differences of F_t at +-s along the world axes.
 * Where every voxel of the stencil holds the same F (a hit whose refinement
 * steps moved it into unobserved voxels, F = 1) the gradient is zero, and the
 * normal is undefined; binary64 rounding of the trilinear weights leaves a
 * residue of ~1e-16 there, so a gradient below 1e-12 counts as zero. */
static int orc_normal(const orc_scene *sc, const double *p, double *nrm)
{
    double g[3];
    for (int a = 0; a < 3; a++) {
        double pp[3] = {p[0], p[1], p[2]}, pm[3] = {p[0], p[1], p[2]};
        pp[a] += sc->s;
        pm[a] -= sc->s;
        g[a] = orc_read_trilinear(sc, pp) - orc_read_trilinear(sc, pm);
    }
    double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (!(gn > 1e-12)) return 0;
    for (int a = 0; a < 3; a++) nrm[a] = g[a] / gn;
    return 1;
}

/* pts/normals: H*W*4 binary64, world frame; pts w = 1 on a hit, all zero on a
 * miss; normals w = 1 when the gradient is non-zero.  zc: camera depth of the
 * hit (0 on a miss).  flags/steps per pixel may be NULL.  zr: H*W*2 expected
 * depth ranges (see orc_expected_depths) or NULL for [z_near, z_far].
 * alt: NULL, or H*W*ORC_RAY_ALT rows of 6 (hit, camera depth, normal x, y, z,
 * normal valid): the ray's other correct outcomes (decision margins above),
 * unused rows with hit = -1; with alt NULL the march follows the binary64
 * reads only. */
int orc_raycast_alt(const orc_scene *sc, int W, int H, const double *K, const double *T_wc,
                    const float *zr, double *pts, double *normals, double *zc, uint8_t *flags,
                    int32_t *steps, double *alt)
{
    orc_cam c;
    orc_cam_setup(&c, W, H, K, T_wc);
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < H; v++) {
        for (int u = 0; u < W; u++) {
            int64_t i = (int64_t)v * W + u;
            orc_ray r;
            orc_ray_setup(sc, &c, u, v, zr ? zr + 2 * i : NULL, &r);
            orc_mout out[1 + ORC_RAY_ALT];
            int fl = 0, st = 0;
            const int n = orc_march_all(sc, &r, out, alt ? 1 + ORC_RAY_ALT : 1, &fl, &st, alt != NULL);
            if (flags) flags[i] = (uint8_t)fl;
            if (steps) steps[i] = st;
            for (int a = 0; a < 4; a++) { pts[4 * i + a] = 0; normals[4 * i + a] = 0; }
            if (zc) zc[i] = 0;
            if (alt) {
                double *row = alt + 6 * ORC_RAY_ALT * i;
                for (int j = 0; j < ORC_RAY_ALT; j++) {
                    double *x = row + 6 * j;
                    x[0] = -1; x[1] = x[2] = x[3] = x[4] = x[5] = 0;
                    if (1 + j >= n) continue;
                    x[0] = out[1 + j].hit;
                    if (!out[1 + j].hit) continue;
                    const double t = out[1 + j].t;
                    double p[3] = {r.o[0] + t * r.d[0], r.o[1] + t * r.d[1], r.o[2] + t * r.d[2]};
                    x[1] = t / r.len;
                    x[5] = orc_normal(sc, p, x + 2);
                }
            }
            if (!out[0].hit) continue;
            const double t = out[0].t;
            double p[3] = {r.o[0] + t * r.d[0], r.o[1] + t * r.d[1], r.o[2] + t * r.d[2]};
            for (int a = 0; a < 3; a++) pts[4 * i + a] = p[a];
            pts[4 * i + 3] = 1.0;
            if (zc) zc[i] = t / r.len;
            if (orc_normal(sc, p, normals + 4 * i)) normals[4 * i + 3] = 1.0;
        }
    }
    return 0;
}

int orc_raycast_range(const orc_scene *sc, int W, int H, const double *K, const double *T_wc,
                      const float *zr, double *pts, double *normals, double *zc, uint8_t *flags,
                      int32_t *steps)
{
    return orc_raycast_alt(sc, W, H, K, T_wc, zr, pts, normals, zc, flags, steps, NULL);
}

int orc_raycast(const orc_scene *sc, int W, int H, const double *K, const double *T_wc,
                double *pts, double *normals, double *zc, uint8_t *flags, int32_t *steps)
{
    return orc_raycast_range(sc, W, H, K, T_wc, NULL, pts, normals, zc, flags, steps);
}

/* What one raycast reads (the algorithmic bytes of a raycast): the distinct
 * allocated blocks whose voxels the marches, refinements and normals read, and
 * the distinct buckets probed.  The same raycast as orc_raycast_range (binary64
 * reads, no branches), run on one thread.  out[0] = blocks, out[1] = buckets. */
int orc_raycast_touched(orc_scene *sc, int W, int H, const double *K, const double *T_wc, const float *zr,
                        int64_t *out)
{
    sc->touch_e = (uint8_t *)calloc((size_t)sc->n_entries, 1);
    sc->touch_b = (uint8_t *)calloc((size_t)sc->n_buckets, 1);
    if (!sc->touch_e || !sc->touch_b) {
        free(sc->touch_e); free(sc->touch_b); sc->touch_e = sc->touch_b = NULL;
        return -1;
    }
    orc_cam c;
    orc_cam_setup(&c, W, H, K, T_wc);
    for (int v = 0; v < H; v++)
        for (int u = 0; u < W; u++) {
            const int64_t i = (int64_t)v * W + u;
            orc_ray r;
            orc_ray_setup(sc, &c, u, v, zr ? zr + 2 * i : NULL, &r);
            orc_mout o;
            int fl = 0, st = 0;
            orc_march_all(sc, &r, &o, 1, &fl, &st, 0);
            if (!o.hit) continue;
            double p[3] = {r.o[0] + o.t * r.d[0], r.o[1] + o.t * r.d[1], r.o[2] + o.t * r.d[2]}, nrm[3];
            orc_normal(sc, p, nrm);
        }
    int64_t nb = 0, nk = 0;
    for (int64_t e = 0; e < sc->n_entries; e++) nb += sc->touch_e[e];
    for (int64_t b = 0; b < sc->n_buckets; b++) nk += sc->touch_b[b];
    free(sc->touch_e); free(sc->touch_b);
    sc->touch_e = sc->touch_b = NULL;
    out[0] = nb;
    out[1] = nk;
    return 0;
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

/* threads of the OpenMP loops from now on (n >= 1) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
