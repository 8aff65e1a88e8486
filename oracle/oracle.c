/*
 * oracle.c — plain, slow CPU reference of the residency-octree hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load this library.  It shares no code with the GPU
 * library: it computes the plain definitions below in FP64 (geometry,
 * sampling, classification, compositing) and exact integer arithmetic (brick
 * IDs, page tables, residency masks, requests, LRU).  It does no octree
 * traversal and no empty-space skipping: both are optimisations that must not
 * change any output.
 *
 * Paper: Herzberger et al., "Residency Octree: A Hybrid Approach for Scalable
 * Web-Based Multi-Volume Rendering" (arXiv 2309.04393).
 *
 *  - Brick hierarchy, bricks of equal voxel size, per-level extent:
 *    Sec. 3 "Brick hierarchy".
 *  - Partially mapped nodes: Sec. 3 "Fully vs. partially mapped".
 *  - Brick IDs: 24-bit spatial offset + 8-bit page-table ID: Sec. 7.
 *  - Residency masks (OR of children, leaves marked by overlapping bricks,
 *    eviction recheck): Sec. 5.3 "Updating residency information",
 *    "LRU cache eviction".
 *  - Per-sample traversal, request on miss, substitution by another resident
 *    level: Sec. 6.1 and Alg. 1; multi-channel emptiness: Sec. 6.1 (a node is
 *    skipped only when every channel is empty there).
 *  - Per-channel resolution ranges: Sec. 6.2.
 *  - Accumulation-level intermixing of channels: Sec. 2 "Multi-volume
 *    rendering".
 *
 * Readings of points the paper leaves open (coordinates, halo, level
 * schedule, tree shape, emptiness test, LOD rule, step grid, mix formula,
 * transfer-function form, LRU order) are listed in the design notes; each
 * function below states the one it uses.
 *
 * Parity status: every function is pinned by CPU tests (closed forms,
 * brute force on tiny inputs, invariants); see tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXL 16
#define OR_MAXC 16

/* ------------------------------------------------------------- geometry */

typedef struct {
    int dims[3];       /* L0 voxels */
    double spacing[3]; /* world units per L0 voxel */
    int n_channels;    /* channels held by the cache (m) */
    int bits;          /* 8 or 16 */
    int B;             /* brick edge in voxels (interior; a 1-voxel halo is added in storage) */
    int n_levels;      /* resolution levels (k) */
    int leaf[3];       /* leaf node size in L0 voxels */
    int depth;         /* subdivision levels below the root */
} or_volume;

/* Level schedule: axis a is halved from level l-1 to l iff its spacing at
 * l-1 is below twice the smallest spacing at l-1; halved dims are ceil(n/2).
 * f[l][a] is the L0 factor (a power of two). */
static void levels(const or_volume *V, int dl[][3], int f[][3]) {
    double s[3] = {V->spacing[0], V->spacing[1], V->spacing[2]};
    for (int a = 0; a < 3; ++a) { dl[0][a] = V->dims[a]; f[0][a] = 1; }
    for (int l = 1; l < V->n_levels; ++l) {
        double m = s[0] < s[1] ? (s[0] < s[2] ? s[0] : s[2]) : (s[1] < s[2] ? s[1] : s[2]);
        for (int a = 0; a < 3; ++a) {
            int h = s[a] < 2.0 * m;
            dl[l][a] = h ? (dl[l - 1][a] + 1) / 2 : dl[l - 1][a];
            f[l][a] = h ? f[l - 1][a] * 2 : f[l - 1][a];
        }
        for (int a = 0; a < 3; ++a)
            if (f[l][a] != f[l - 1][a]) s[a] *= 2.0;
    }
}

int or_level_info(const or_volume *V, int *dims_out /* [L][3] */, int *f_out /* [L][3] */,
                  int *nb_out /* [L][3] bricks per axis */) {
    int dl[OR_MAXL][3], f[OR_MAXL][3];
    if (V->n_levels < 1 || V->n_levels > OR_MAXL) return -1;
    levels(V, dl, f);
    for (int l = 0; l < V->n_levels; ++l)
        for (int a = 0; a < 3; ++a) {
            if (dims_out) dims_out[3 * l + a] = dl[l][a];
            if (f_out) f_out[3 * l + a] = f[l][a];
            if (nb_out) nb_out[3 * l + a] = (dl[l][a] + V->B - 1) / V->B;
        }
    return 0;
}

/* Dense enumeration of all bricks: channel-major, then level, then
 * (bz, by, bx) row-major.  This is the oracle's own bookkeeping; results
 * leave the oracle as brick IDs. */
typedef struct {
    int L, C, B;
    int dl[OR_MAXL][3], f[OR_MAXL][3], nb[OR_MAXL][3];
    long long off[OR_MAXC][OR_MAXL];
    long long total;
} geo_t;

static void geo(const or_volume *V, geo_t *G) {
    G->L = V->n_levels;
    G->C = V->n_channels;
    G->B = V->B;
    levels(V, G->dl, G->f);
    long long o = 0;
    for (int c = 0; c < G->C; ++c)
        for (int l = 0; l < G->L; ++l) {
            for (int a = 0; a < 3; ++a) G->nb[l][a] = (G->dl[l][a] + V->B - 1) / V->B;
            G->off[c][l] = o;
            o += (long long)G->nb[l][0] * G->nb[l][1] * G->nb[l][2];
        }
    G->total = o;
}

long long or_brick_count(const or_volume *V) {
    geo_t G;
    geo(V, &G);
    return G.total;
}

static inline long long dense(const geo_t *G, int c, int l, int bx, int by, int bz) {
    return G->off[c][l] + ((long long)bz * G->nb[l][1] + by) * G->nb[l][0] + bx;
}

/* Brick ID (Sec. 7): 8-bit page-table ID in the top byte, then z, y, x
 * offsets of 8 bits each; the page table of (channel c, level l) has ID
 * c * k + l where k is the number of levels. */
uint32_t or_brick_id(int n_levels, int c, int l, int bx, int by, int bz) {
    uint32_t pt = (uint32_t)(c * n_levels + l);
    return (pt << 24) | ((uint32_t)bz << 16) | ((uint32_t)by << 8) | (uint32_t)bx;
}

void or_brick_id_decode(int n_levels, uint32_t id, int *c, int *l, int *bx, int *by, int *bz) {
    uint32_t pt = id >> 24;
    *c = (int)(pt / (uint32_t)n_levels);
    *l = (int)(pt % (uint32_t)n_levels);
    *bz = (int)((id >> 16) & 255u);
    *by = (int)((id >> 8) & 255u);
    *bx = (int)(id & 255u);
}

/* dense index -> ID, for every brick (out[total]) */
int or_dense_ids(const or_volume *V, uint32_t *out) {
    geo_t G;
    geo(V, &G);
    for (int c = 0; c < G.C; ++c)
        for (int l = 0; l < G.L; ++l)
            for (int bz = 0; bz < G.nb[l][2]; ++bz)
                for (int by = 0; by < G.nb[l][1]; ++by)
                    for (int bx = 0; bx < G.nb[l][0]; ++bx)
                        out[dense(&G, c, l, bx, by, bz)] = or_brick_id(G.L, c, l, bx, by, bz);
    return 0;
}

/* ----------------------------------------------------------------- tree */

/* Generalised 2^k tree over a power-of-two padded L0 domain: axis a needs
 * s_a = ceil(log2(ceil(dims_a / leaf_a))) splits and takes them at the last
 * s_a subdivision levels.  Node size at level d: leaf_a << min(s_a, depth-d). */
typedef struct {
    int depth;
    int size[OR_MAXL + 8][3];
    int n[OR_MAXL + 8][3];
    long long off[OR_MAXL + 8];
    long long total;
} tree_t;

static int tree(const or_volume *V, tree_t *T) {
    T->depth = V->depth;
    if (V->depth < 0 || V->depth >= OR_MAXL + 7) return -1;
    int s[3];
    for (int a = 0; a < 3; ++a) {
        int nl = (V->dims[a] + V->leaf[a] - 1) / V->leaf[a];
        s[a] = 0;
        while ((1 << s[a]) < nl) s[a]++;
        if (s[a] > V->depth) return -1;
    }
    long long o = 0;
    for (int d = 0; d <= V->depth; ++d) {
        for (int a = 0; a < 3; ++a) {
            int k = V->depth - d < s[a] ? V->depth - d : s[a];
            T->size[d][a] = V->leaf[a] << k;
            T->n[d][a] = 1 << (s[a] - k);
        }
        T->off[d] = o;
        o += (long long)T->n[d][0] * T->n[d][1] * T->n[d][2];
    }
    T->total = o;
    return 0;
}

long long or_node_count(const or_volume *V, long long *level_off /* [depth+2] or NULL */,
                        int *level_n /* [depth+1][3] or NULL */) {
    tree_t T;
    if (tree(V, &T)) return -1;
    if (level_off) {
        for (int d = 0; d <= T.depth; ++d) level_off[d] = T.off[d];
        level_off[T.depth + 1] = T.total;
    }
    if (level_n)
        for (int d = 0; d <= T.depth; ++d)
            for (int a = 0; a < 3; ++a) level_n[3 * d + a] = T.n[d][a];
    return T.total;
}

/* Metadata for all nodes from leaf metadata (Sec. 5.3 "Updating culling
 * information"; parents bound their children): node [min, max] = [min of
 * leaf mins, max of leaf maxes] over the leaves inside the node.
 * leaf_mm[c][leaf][2] (leaf grid order), out[node][c][2]. */
int or_meta_all(const or_volume *V, const uint16_t *leaf_mm, uint16_t *out) {
    tree_t T;
    if (tree(V, &T)) return -1;
    int C = V->n_channels, D = T.depth;
    long long nleaf = (long long)T.n[D][0] * T.n[D][1] * T.n[D][2];
    for (int d = 0; d <= D; ++d) {
        int r[3];
        for (int a = 0; a < 3; ++a) r[a] = T.size[d][a] / T.size[D][a]; /* leaves per node edge */
        for (int z = 0; z < T.n[d][2]; ++z)
            for (int y = 0; y < T.n[d][1]; ++y)
                for (int x = 0; x < T.n[d][0]; ++x) {
                    long long node = T.off[d] + ((long long)z * T.n[d][1] + y) * T.n[d][0] + x;
                    for (int c = 0; c < C; ++c) {
                        int mn = 65535, mx = 0;
                        for (int lz = z * r[2]; lz < (z + 1) * r[2]; ++lz)
                            for (int ly = y * r[1]; ly < (y + 1) * r[1]; ++ly)
                                for (int lx = x * r[0]; lx < (x + 1) * r[0]; ++lx) {
                                    long long li = ((long long)lz * T.n[D][1] + ly) * T.n[D][0] + lx;
                                    const uint16_t *p = leaf_mm + ((long long)c * nleaf + li) * 2;
                                    if (p[0] < mn) mn = p[0];
                                    if (p[1] > mx) mx = p[1];
                                }
                        out[(node * C + c) * 2 + 0] = (uint16_t)mn;
                        out[(node * C + c) * 2 + 1] = (uint16_t)mx;
                    }
                }
    }
    return 0;
}

/* Residency masks from scratch (Sec. 3 partial mapping; Sec. 5.2 bitmask of
 * partially mapped levels): bit l of mask[node][c] is set iff some resident
 * brick (c, l, b) overlaps the node with positive volume.  Extents are
 * half-open integer boxes in L0 voxels: brick interior
 * [b B f_l, (b+1) B f_l), node [x size_d, (x+1) size_d).
 * res_slot[dense] >= 0 marks resident bricks.  out[node][c] (uint16). */
int or_masks(const or_volume *V, const int32_t *res_slot, uint16_t *out) {
    geo_t G;
    tree_t T;
    geo(V, &G);
    if (tree(V, &T)) return -1;
    int C = V->n_channels;
#pragma omp parallel for schedule(dynamic, 64)
    for (long long node = 0; node < T.total; ++node) {
        int d = 0;
        while (d < T.depth && node >= T.off[d + 1]) d++;
        long long li = node - T.off[d];
        int x = (int)(li % T.n[d][0]);
        int y = (int)((li / T.n[d][0]) % T.n[d][1]);
        int z = (int)(li / ((long long)T.n[d][0] * T.n[d][1]));
        long long lo[3] = {(long long)x * T.size[d][0], (long long)y * T.size[d][1],
                           (long long)z * T.size[d][2]};
        for (int c = 0; c < C; ++c) {
            uint16_t m = 0;
            for (int l = 0; l < G.L; ++l) {
                int b0[3], b1[3], ok = 1;
                for (int a = 0; a < 3; ++a) {
                    long long e = (long long)G.B * G.f[l][a];
                    long long hi = lo[a] + T.size[d][a]; /* exclusive */
                    b0[a] = (int)(lo[a] / e);
                    b1[a] = (int)((hi - 1) / e);
                    if (b1[a] > G.nb[l][a] - 1) b1[a] = G.nb[l][a] - 1;
                    if (b0[a] > b1[a]) ok = 0;
                }
                if (!ok) continue;
                int hit = 0;
                for (int bz = b0[2]; bz <= b1[2] && !hit; ++bz)
                    for (int by = b0[1]; by <= b1[1] && !hit; ++by)
                        for (int bx = b0[0]; bx <= b1[0] && !hit; ++bx)
                            if (res_slot[dense(&G, c, l, bx, by, bz)] >= 0) hit = 1;
                if (hit) m |= (uint16_t)(1u << l);
            }
            out[node * C + c] = m;
        }
    }
    return 0;
}

/* --------------------------------------------------- transfer functions */

/* Window given as raw values in 24.8 fixed point: W0 = 256*w0_raw,
 * W1 = 256*w1_raw.  A value v (raw units) maps to the table position
 * p = 255 * clamp((v - w0) / (w1 - w0), 0, 1). */

/* Emptiness of a [mn, mx] raw range for one transfer function: empty iff
 * every table entry that linear interpolation can reach for values in
 * [mn, mx] has alpha 0; the reachable entries are
 * floor(p(mn)) .. ceil(p(mx)).  Exact integer arithmetic. */
int or_tf_empty(uint32_t mn, uint32_t mx, uint32_t W0, uint32_t W1, const float *tf /*256x4*/) {
    long long den = (long long)W1 - (long long)W0;
    long long nlo = 255LL * ((long long)mn * 256 - (long long)W0);
    long long nhi = 255LL * ((long long)mx * 256 - (long long)W0);
    long long lo, hi;
    if (nlo <= 0) lo = 0;
    else lo = nlo / den; /* floor for positive operands */
    if (nhi <= 0) hi = 0;
    else hi = (nhi + den - 1) / den; /* ceil */
    if (lo > 255) lo = 255;
    if (hi > 255) hi = 255;
    for (long long e = lo; e <= hi; ++e)
        if (tf[4 * e + 3] != 0.0f) return 0;
    return 1;
}

static void tf_eval(double v, uint32_t W0, uint32_t W1, const float *tf, double out[4]) {
    double w0 = W0 / 256.0, w1 = W1 / 256.0;
    double x = (v - w0) / (w1 - w0);
    if (x < 0) x = 0;
    if (x > 1) x = 1;
    double p = 255.0 * x;
    int i0 = (int)floor(p);
    if (i0 > 255) i0 = 255;
    int i1 = i0 < 255 ? i0 + 1 : 255;
    double fr = p - i0;
    for (int k = 0; k < 4; ++k) out[k] = (double)tf[4 * i0 + k] * (1.0 - fr) + (double)tf[4 * i1 + k] * fr;
}

/* -------------------------------------------------------------- frames */

typedef struct {
    int proj; /* 0 orthographic, 1 perspective */
    double eye[3], F[3], R[3], U[3];
    double tx, ty; /* ortho: half extents (world); persp: tan of half angles */
    int W, H;
    double delta;    /* world step between samples */
    double lod_bias; /* beta */
    int nvis;
    int vis[OR_MAXC];    /* cache channel of each visible slot */
    int lod_lo[OR_MAXC]; /* per visible slot resolution range */
    int lod_hi[OR_MAXC];
    uint32_t W0[OR_MAXC], W1[OR_MAXC];
    const float *tf[OR_MAXC]; /* 256 x RGBA per visible slot */
    double term_alpha;
    double term_margin; /* |A - term_alpha| below this marks an ambiguous termination */
    int adaptive;       /* LOD-adaptive step (Sec. 6.1, the sampling distance grows with the level) */
    int homogeneous;    /* leaves homogeneous for all channels rendered from their metadata (Alg. 1 renderAndSkipNode) */
    int channel_rates;  /* with adaptive: each channel sampled at the rate of its own level (Sec. 6.1) */
    int traversal_depth; /* with adaptive: emptiness decided at the node the step size allows (Alg. 1) */
} or_frame;

/* Level data: lvl[c * L + l] points to the level's array [z][y][x]
 * (uint8 or uint16 per V->bits).  When lvl is NULL the voxels come from a
 * data source instead (the generator's region query) through a small
 * per-thread tile cache; the values are the same, only the access differs. */

typedef int (*or_fetch_fn)(void *ctx, const int f[3], int x0, int y0, int z0, int nx, int ny, int nz,
                           int nchan, const int *chans, uint16_t *out);

typedef struct {
    void *ctx;
    or_fetch_fn fetch;
} or_source;

#define TILE 16
#define TCACHE 64

typedef struct {
    int key[5]; /* c, l, tx, ty, tz; c = -1 when empty */
    uint16_t v[TILE * TILE * TILE];
} tile_t;

typedef struct {
    const or_volume *V;
    const void *const *lvl;
    const int *box; /* optional [C*L][6]: window origin and size of each level array */
    const or_source *src;
    tile_t *tiles; /* TCACHE entries, this thread's */
    const int (*dl)[3];
    const int (*f)[3];
    int L;
} sampler_t;

static inline double voxel(const sampler_t *S, int c, int l, int x, int y, int z) {
    const int *d = S->dl[l];
    if (x < 0) x = 0;
    if (y < 0) y = 0;
    if (z < 0) z = 0;
    if (x > d[0] - 1) x = d[0] - 1;
    if (y > d[1] - 1) y = d[1] - 1;
    if (z > d[2] - 1) z = d[2] - 1;
    if (S->lvl) {
        const void *a = S->lvl[c * S->L + l];
        size_t i;
        if (S->box) {
            /* the array holds only a window of the level */
            const int *w = S->box + 6 * (c * S->L + l);
            int X = x - w[0], Y = y - w[1], Z = z - w[2];
            if (X < 0 || Y < 0 || Z < 0 || X >= w[3] || Y >= w[4] || Z >= w[5]) return NAN;
            i = ((size_t)Z * w[4] + Y) * w[3] + X;
        } else {
            i = ((size_t)z * d[1] + y) * d[0] + x;
        }
        return S->V->bits == 8 ? (double)((const uint8_t *)a)[i] : (double)((const uint16_t *)a)[i];
    }
    int tx = x / TILE, ty = y / TILE, tz = z / TILE;
    unsigned h = ((unsigned)c * 73856093u) ^ ((unsigned)l * 19349663u) ^ ((unsigned)tx * 83492791u) ^
                 ((unsigned)ty * 2654435761u) ^ ((unsigned)tz * 40503u);
    tile_t *t = &S->tiles[h % TCACHE];
    if (!(t->key[0] == c && t->key[1] == l && t->key[2] == tx && t->key[3] == ty && t->key[4] == tz)) {
        int x0 = tx * TILE, y0 = ty * TILE, z0 = tz * TILE;
        int nx = d[0] - x0 < TILE ? d[0] - x0 : TILE;
        int ny = d[1] - y0 < TILE ? d[1] - y0 : TILE;
        int nz = d[2] - z0 < TILE ? d[2] - z0 : TILE;
        uint16_t buf[TILE * TILE * TILE];
        S->src->fetch(S->src->ctx, S->f[l], x0, y0, z0, nx, ny, nz, 1, &c, buf);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) t->v[(k * TILE + j) * TILE + i] = buf[(k * ny + j) * nx + i];
        t->key[0] = c; t->key[1] = l; t->key[2] = tx; t->key[3] = ty; t->key[4] = tz;
    }
    return (double)t->v[((z - tz * TILE) * TILE + (y - ty * TILE)) * TILE + (x - tx * TILE)];
}

/* Trilinear interpolation in level l of channel c at level coordinates q
 * (voxel i centred at i + 1/2; clamp-to-edge indices). */
static double trilinear(const sampler_t *S, int c, int l, const double q[3]) {
    int i0[3];
    double w[3];
    for (int k = 0; k < 3; ++k) {
        double p = q[k] - 0.5;
        double fl = floor(p);
        i0[k] = (int)fl;
        w[k] = p - fl;
    }
    double cc[2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy) {
            double v0 = voxel(S, c, l, i0[0], i0[1] + dy, i0[2] + dz);
            double v1 = voxel(S, c, l, i0[0] + 1, i0[1] + dy, i0[2] + dz);
            cc[dz][dy] = v0 * (1.0 - w[0]) + v1 * w[0];
        }
    double e0 = cc[0][0] * (1.0 - w[1]) + cc[0][1] * w[1];
    double e1 = cc[1][0] * (1.0 - w[1]) + cc[1][1] * w[1];
    return e0 * (1.0 - w[2]) + e1 * w[2];
}

static tile_t *new_tiles(void) {
    tile_t *t = (tile_t *)malloc(sizeof(tile_t) * TCACHE);
    if (t)
        for (int i = 0; i < TCACHE; ++i) t[i].key[0] = -1;
    return t;
}

/* Ray of pixel (i, j), row 0 at the top: a = (2i+1-W)/W, b = (H-2j-1)/H.
 * Ortho: origin eye + a tx R + b ty U, direction F.  Perspective: origin
 * eye, direction normalize(F + a tx R + b ty U).  Returned in L0 voxel
 * units: o/spacing, d/spacing (t stays the world distance along the ray). */
static void pixel_ray(const or_volume *V, const or_frame *Fr, int i, int j, double o[3], double d[3]) {
    double a = (double)(2 * i + 1 - Fr->W) / (double)Fr->W;
    double b = (double)(Fr->H - 2 * j - 1) / (double)Fr->H;
    double ow[3], dw[3];
    if (Fr->proj == 0) {
        for (int k = 0; k < 3; ++k) {
            ow[k] = Fr->eye[k] + a * Fr->tx * Fr->R[k] + b * Fr->ty * Fr->U[k];
            dw[k] = Fr->F[k];
        }
    } else {
        double n = 0;
        for (int k = 0; k < 3; ++k) {
            ow[k] = Fr->eye[k];
            dw[k] = Fr->F[k] + a * Fr->tx * Fr->R[k] + b * Fr->ty * Fr->U[k];
            n += dw[k] * dw[k];
        }
        n = sqrt(n);
        for (int k = 0; k < 3; ++k) dw[k] /= n;
    }
    for (int k = 0; k < 3; ++k) {
        o[k] = ow[k] / V->spacing[k];
        d[k] = dw[k] / V->spacing[k];
    }
}

/* Parameter interval [t0, t1] where o + t d lies in the box [0, dims]. */
static int box_interval(const or_volume *V, const double o[3], const double d[3], double *t0, double *t1) {
    double a = -INFINITY, b = INFINITY;
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0) {
            if (o[k] < 0.0 || o[k] >= V->dims[k]) return 0;
            continue;
        }
        double u = (0.0 - o[k]) / d[k], v = (V->dims[k] - o[k]) / d[k];
        if (u > v) { double s = u; u = v; v = s; }
        if (u > a) a = u;
        if (v < b) b = v;
    }
    if (a > b) return 0;
    *t0 = a;
    *t1 = b;
    return 1;
}

/* Desired level (Sec. 6.1, chooseResolutionLevel; Sec. 6.2 per-channel
 * range): n(t) = #{l >= 1 : t >= D_l}, D_l = s_l / (beta theta_pix), with s_l
 * the level's x voxel size in world units and theta_pix = 2 ty / H (radians
 * per pixel, perspective).  Orthographic views use the constant pixel size
 * 2 ty / H: n = #{l >= 1 : beta * pixel >= s_l}.  Then clamped per channel. */

typedef struct {
    long long samples;        /* ray samples inside the volume */
    long long channel_samples;/* (sample, visible channel) pairs sampled from a brick */
    long long missing;        /* (sample, channel) pairs whose desired brick is missing */
    long long amb_samples;    /* samples within the ambiguity margin of a decision */
    long long amb_pixels;
} or_stats;

#define AMB_POS 1e-9

static int cmp_ll(const void *a, const void *b) {
    const long long x = *(const long long *)a, y = *(const long long *)b;
    return x < y ? -1 : x > y;
}

/* O1: one frame.  Inputs: volume, level arrays, resident slots per dense
 * brick (-1 = not resident), leaf metadata leaf_mm[c][leaf][2], frame.
 * Outputs (any may be NULL):
 *   rgba[H][W][4]      premultiplied colour and opacity
 *   counts[dense]      requests: one per (sample, channel) whose desired
 *                      brick is not resident, in a leaf that is not empty
 *                      for that channel (Alg. 1 reportBrickRequest)
 *   used[slot]         1 if some sample read from the slot
 *   aov[H][W][L]       samples per level actually used
 *   amb_pix[H][W]      1 if the pixel has a sample within the ambiguity
 *                      margin, or a second early-termination decision within
 *                      it
 *   amb_counts[dense]  requests of samples after an ambiguous termination
 *   amb_used[slot]     slots read by samples after an ambiguous termination
 *   reqb[H][W]         bricks the pixel requires (Sec. 8, bricks required to
 *                      be resident per pixel): the number of distinct desired
 *                      bricks (c, l*, b*) of its samples that need data (a
 *                      channel not empty in the sample's leaf, the leaf not
 *                      rendered from its values), up to its termination
 *   alt_rgba[H][W][4]  with alt_pix[H][W] = 1: the pixel's other valid
 *                      value, had its one early-termination decision within
 *                      the margin gone the other way (stopped there, or
 *                      composited on to the next stop)
 * Every pixel's ray samples t_k = k delta, k = 0, 1, ...; samples outside
 * [0, dims) are void.  Early termination when A >= term_alpha.  With
 * Fr->adaptive only the samples on the grid of their level band are taken
 * (see the step range below). */
int or_render(const or_volume *V, const void *const *lvl, const int *lvl_box, const or_source *src,
              const int32_t *res_slot, const uint16_t *leaf_mm, const or_frame *Fr, int row0,
              int row1, double *rgba, uint32_t *counts, uint8_t *used, uint32_t *aov,
              uint8_t *amb_pix, uint32_t *amb_counts, uint8_t *amb_used, double *alt_rgba,
              uint8_t *alt_pix, uint32_t *reqb, or_stats *stats, int n_threads) {
    geo_t G;
    tree_t T;
    geo(V, &G);
    if (tree(V, &T)) return -1;
    if (Fr->nvis < 0 || Fr->nvis > OR_MAXC) return -1;
    const int L = G.L, Dp = T.depth;
    const long long nleaf = (long long)T.n[Dp][0] * T.n[Dp][1] * T.n[Dp][2];
    double Dl[OR_MAXL];
    int n_ortho = 0;
    double pix = 2.0 * Fr->ty / Fr->H;
    for (int l = 1; l < L; ++l) {
        double s_l = G.f[l][0] * V->spacing[0];
        Dl[l] = s_l / (Fr->lod_bias * pix);
        if (Fr->proj == 0 && Fr->lod_bias * pix >= s_l) n_ortho++;
    }
    /* LOD-adaptive step: the sampling distance follows the finest desired
     * level over the visible channels, min_c clamp(l*, lo_c, hi_c) =
     * clamp(l*, min_c lo_c, min_c hi_c); a sample k is taken only when k is
     * a multiple of that level's x factor r, and its mixed opacity is
     * corrected to 1 - (1 - alpha)^r (the premultiplied colour scaled with
     * it), so a coarse band keeps the opacity per unit length. */
    int step_lo = OR_MAXL, step_hi = OR_MAXL;
    for (int jv = 0; jv < Fr->nvis; ++jv) {
        if (Fr->lod_lo[jv] < step_lo) step_lo = Fr->lod_lo[jv];
        if (Fr->lod_hi[jv] < step_hi) step_hi = Fr->lod_hi[jv];
    }
    /* Traversal depth from the step (Alg. 1 chooseTraversalDepth: the tree is
     * traversed no deeper than a node the step cannot jump over): with the
     * option, a sample taken with step factor r decides emptiness and
     * homogeneity on the deepest node whose smallest world extent is at
     * least r delta (the leaf when the leaf is large enough), reading that
     * node's metadata: min and max over the leaves inside it. */
    uint16_t *node_mm = NULL;
    int ddep[OR_MAXL];
    for (int l = 0; l < OR_MAXL; ++l) ddep[l] = Dp;
    if (Fr->adaptive && Fr->traversal_depth) {
        node_mm = (uint16_t *)malloc((size_t)T.total * V->n_channels * 2 * sizeof(uint16_t));
        if (!node_mm || or_meta_all(V, leaf_mm, node_mm)) {
            free(node_mm);
            return -1;
        }
        for (int l = 0; l < L; ++l) {
            const double dist = G.f[l][0] * Fr->delta;
            int d = Dp;
            for (;;) {
                double ext = INFINITY;
                for (int a = 0; a < 3; ++a) ext = fmin(ext, T.size[d][a] * V->spacing[a]);
                if (ext >= dist || d == 0) break;
                --d;
            }
            ddep[l] = d;
        }
    }
    long long st_s = 0, st_cs = 0, st_m = 0, st_as = 0, st_ap = 0;
    if (!lvl && !(src && src->fetch)) {
        free(node_mm);
        return -1;
    }
    if (row0 < 0) row0 = 0;
    if (row1 <= 0 || row1 > Fr->H) row1 = Fr->H;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel reduction(+ : st_s, st_cs, st_m, st_as, st_ap)
    {
    sampler_t SM = {V, lvl, lvl_box, src, lvl ? NULL : new_tiles(), (const int(*)[3])G.dl,
                    (const int(*)[3])G.f, L};
    long long *rkeys = NULL; /* desired bricks of the current pixel (with repeats) */
    size_t nrk = 0, caprk = 0;
#pragma omp for schedule(dynamic, 1)
    for (int j = row0; j < row1; ++j) {
        for (int i = 0; i < Fr->W; ++i) {
            long long pidx = (long long)j * Fr->W + i;
            double o[3], d[3], t0, t1;
            double Cc[3] = {0, 0, 0}, A = 0.0;
            /* tol: an early-termination decision was within the margin, so a
             * reduced-precision renderer may have stopped (or not) there:
             * every later sample's requests and reads are tolerated.
             * shadow: this oracle has stopped compositing (A >= term) but
             * keeps walking the ray to collect those tolerated sets.
             * Both outcomes of that one decision are valid images of the
             * pixel: the one not taken is kept as the alternate (Ca, Aa); when
             * this oracle stopped there, the alternate goes on compositing
             * (altrun) until its own termination. */
            double Ca[3] = {0, 0, 0}, Aa = 0.0;
            int pamb = 0, shadow = 0, tol = 0, alt = 0, altrun = 0;
            nrk = 0;
            pixel_ray(V, Fr, i, j, o, d);
            if (box_interval(V, o, d, &t0, &t1)) {
                long long k0 = (long long)floor(t0 / Fr->delta) - 1;
                long long k1 = (long long)ceil(t1 / Fr->delta) + 1;
                if (k0 < 0) k0 = 0;
                for (long long k = k0; k <= k1; ++k) {
                    double t = (double)k * Fr->delta;
                    double u[3];
                    int inside = 1, samb = 0;
                    for (int a = 0; a < 3; ++a) {
                        u[a] = o[a] + t * d[a];
                        if (!(u[a] >= 0.0 && u[a] < (double)V->dims[a])) inside = 0;
                        if (fabs(u[a] - nearbyint(u[a])) < AMB_POS) samb = 1;
                    }
                    if (!inside) {
                        if (samb && !tol) pamb = 1; /* box decision is close */
                        continue;
                    }
                    int iu[3] = {(int)floor(u[0]), (int)floor(u[1]), (int)floor(u[2])};
                    int lc[3];
                    for (int a = 0; a < 3; ++a) lc[a] = iu[a] / V->leaf[a];
                    long long leaf = ((long long)lc[2] * T.n[Dp][1] + lc[1]) * T.n[Dp][0] + lc[0];
                    int nlev, lamb = 0;
                    if (Fr->proj == 0) nlev = n_ortho;
                    else {
                        nlev = 0;
                        for (int l = 1; l < L; ++l) {
                            if (t >= Dl[l]) nlev++;
                            if (fabs(t - Dl[l]) <= 1e-9 * Dl[l]) lamb = 1;
                        }
                    }
                    int rstep = 1, dn = Dp;
                    if (Fr->adaptive) {
                        int ls = nlev;
                        if (ls < step_lo) ls = step_lo;
                        if (ls > step_hi) ls = step_hi;
                        if (ls > L - 1) ls = L - 1;
                        rstep = G.f[ls][0];
                        dn = ddep[ls];
                        if (k % rstep != 0) {
                            /* not on this band's grid; a level decision close to
                             * its threshold may take it on another renderer */
                            if (lamb && !tol) { pamb = 1; st_as++; }
                            continue;
                        }
                    }
                    samb |= lamb;
                    if (samb && !tol) { pamb = 1; st_as++; }
                    if (!shadow) st_s++;
                    /* Render-and-skip leaf (Alg. 1 isHomogeneous / renderAndSkipNode;
                     * Sec. 6.1: only a node homogeneous for all channels is rendered
                     * from its value): with the option on, when every visible channel
                     * is empty in the leaf or has one value there (metadata
                     * min == max), and at least one has a value, each such channel's
                     * value stands for the sample; nothing is read, requested or
                     * stamped, whatever is resident.  Otherwise every non-empty
                     * channel, homogeneous or not, samples its brick. */
                    /* the decision node's metadata of channel c: the leaf's, or with a
                     * traversal depth above the leaves that node's */
                    long long dnode = leaf;
                    if (dn < Dp)
                        dnode = T.off[dn] + ((long long)(iu[2] / T.size[dn][2]) * T.n[dn][1] + iu[1] / T.size[dn][1]) *
                                                T.n[dn][0] +
                                iu[0] / T.size[dn][0];
#define DMM(c) (dn < Dp ? node_mm + (dnode * V->n_channels + (c)) * 2 : leaf_mm + ((long long)(c) * nleaf + leaf) * 2)
                    int rskip = 0;
                    if (Fr->homogeneous) {
                        int anyv = 0;
                        rskip = 1;
                        for (int jv = 0; jv < Fr->nvis && rskip; ++jv) {
                            const uint16_t *mm = DMM(Fr->vis[jv]);
                            if (or_tf_empty(mm[0], mm[1], Fr->W0[jv], Fr->W1[jv], Fr->tf[jv])) continue;
                            if (mm[0] == mm[1]) anyv = 1;
                            else rskip = 0;
                        }
                        rskip = rskip && anyv;
                    }
                    /* Per-channel sampling rates (Sec. 6.1: a channel may need only every
                     * second step; the channel needing the highest rate sets the step):
                     * with the option, channel c takes part in sample k only when k is a
                     * multiple of r_c, the x factor of its own clamped desired level, and
                     * then stands for r_c base steps: transparency (1 - alpha_c)^r_c,
                     * colour weight r_c alpha_c.  The sample's opacity is then
                     * 1 - prod of those transparencies, with no further correction
                     * (with every r_c = r this is the adaptive step's correction). */
                    const int rates = Fr->adaptive && Fr->channel_rates;
                    double prod = 1.0, sa = 0.0, srgb[3] = {0, 0, 0};
                    for (int jv = 0; jv < Fr->nvis; ++jv) {
                        int c = Fr->vis[jv];
                        const uint16_t *mm = DMM(c);
                        if (or_tf_empty(mm[0], mm[1], Fr->W0[jv], Fr->W1[jv], Fr->tf[jv])) continue;
                        int rc = 1;
                        if (rates) {
                            int lc = nlev;
                            if (lc < Fr->lod_lo[jv]) lc = Fr->lod_lo[jv];
                            if (lc > Fr->lod_hi[jv]) lc = Fr->lod_hi[jv];
                            if (lc > L - 1) lc = L - 1;
                            rc = G.f[lc][0];
                            if (k % rc != 0) continue; /* not this channel's sample */
                        }
                        if (rskip) {
                            if (shadow && !altrun) continue;
                            double rgbaH[4];
                            tf_eval((double)mm[0], Fr->W0[jv], Fr->W1[jv], Fr->tf[jv], rgbaH);
                            prod *= rates ? pow(1.0 - rgbaH[3], (double)rc) : (1.0 - rgbaH[3]);
                            sa += rc * rgbaH[3];
                            for (int k2 = 0; k2 < 3; ++k2) srgb[k2] += rc * rgbaH[3] * rgbaH[k2];
                            continue;
                        }
                        int ls = nlev;
                        if (ls < Fr->lod_lo[jv]) ls = Fr->lod_lo[jv];
                        if (ls > Fr->lod_hi[jv]) ls = Fr->lod_hi[jv];
                        /* desired brick */
                        int bs[3];
                        for (int a = 0; a < 3; ++a) bs[a] = iu[a] / (G.B * G.f[ls][a]);
                        long long want = dense(&G, c, ls, bs[0], bs[1], bs[2]);
                        if (reqb && !shadow) {
                            if (nrk == caprk) {
                                caprk = caprk ? 2 * caprk : 1024;
                                rkeys = (long long *)realloc(rkeys, caprk * sizeof(long long));
                            }
                            rkeys[nrk++] = want;
                        }
                        if (res_slot[want] < 0) {
                            if (tol) {
                                if (amb_counts) {
#pragma omp atomic
                                    amb_counts[want]++;
                                }
                            } else {
                                if (counts) {
#pragma omp atomic
                                    counts[want]++;
                                }
                                st_m++;
                            }
                        }
                        /* substitution: finest resident level >= ls */
                        int lu = -1;
                        long long slot = -1;
                        for (int l = ls; l < L; ++l) {
                            int bb[3];
                            for (int a = 0; a < 3; ++a) bb[a] = iu[a] / (G.B * G.f[l][a]);
                            long long di = dense(&G, c, l, bb[0], bb[1], bb[2]);
                            if (res_slot[di] >= 0) { lu = l; slot = res_slot[di]; break; }
                        }
                        if (lu < 0) continue;
                        if (tol) {
                            if (amb_used) __atomic_store_n(&amb_used[slot], 1, __ATOMIC_RELAXED);
                            if (shadow && !altrun) continue;
                        } else {
                            if (used) __atomic_store_n(&used[slot], 1, __ATOMIC_RELAXED);
                            if (aov) aov[pidx * L + lu]++;
                            st_cs++;
                        }
                        double q[3];
                        for (int a = 0; a < 3; ++a) q[a] = u[a] / G.f[lu][a];
                        double v = trilinear(&SM, c, lu, q);
                        double rgbaC[4];
                        tf_eval(v, Fr->W0[jv], Fr->W1[jv], Fr->tf[jv], rgbaC);
                        double ac = rgbaC[3];
                        prod *= rates ? pow(1.0 - ac, (double)rc) : (1.0 - ac);
                        sa += rc * ac;
                        for (int k2 = 0; k2 < 3; ++k2) srgb[k2] += rc * ac * rgbaC[k2];
                    }
                    if (shadow && !altrun) continue;
                    /* mix: alpha_s = 1 - prod(1 - alpha_c);
                     * C_s = alpha_s * sum(alpha_c rgb_c) / sum(alpha_c) */
                    double as = 1.0 - prod;
                    if (rstep > 1 && !rates) as = 1.0 - pow(prod, (double)rstep);
                    double Cs[3] = {0, 0, 0};
                    if (sa > 0.0)
                        for (int k2 = 0; k2 < 3; ++k2) Cs[k2] = as * srgb[k2] / sa;
                    if (shadow) {
                        /* the alternate outcome: composited on to its own stop */
                        for (int k2 = 0; k2 < 3; ++k2) Ca[k2] += (1.0 - Aa) * Cs[k2];
                        Aa += (1.0 - Aa) * as;
                        if (fabs(Aa - Fr->term_alpha) < Fr->term_margin) pamb = 1; /* a second close call */
                        if (Aa >= Fr->term_alpha) altrun = 0;
                        continue;
                    }
                    for (int k2 = 0; k2 < 3; ++k2) Cc[k2] += (1.0 - A) * Cs[k2];
                    A += (1.0 - A) * as;
                    if (fabs(A - Fr->term_alpha) < Fr->term_margin) {
                        /* a reduced-precision renderer may decide either way here */
                        if (!tol) {
                            tol = 1;
                            alt = 1;
                            for (int k2 = 0; k2 < 3; ++k2) Ca[k2] = Cc[k2];
                            Aa = A;
                            altrun = A >= Fr->term_alpha; /* it stops here: the alternate goes on */
                        } else {
                            pamb = 1; /* a second close call: more than two outcomes */
                        }
                    }
                    if (A >= Fr->term_alpha) {
                        if (!tol) break;
                        shadow = 1;
                    }
                }
            }
            if (rgba) {
                rgba[pidx * 4 + 0] = Cc[0];
                rgba[pidx * 4 + 1] = Cc[1];
                rgba[pidx * 4 + 2] = Cc[2];
                rgba[pidx * 4 + 3] = A;
            }
            if (amb_pix) amb_pix[pidx] = (uint8_t)pamb;
            if (reqb) {
                qsort(rkeys, nrk, sizeof(long long), cmp_ll);
                uint32_t nd = 0;
                for (size_t q = 0; q < nrk; ++q)
                    if (q == 0 || rkeys[q] != rkeys[q - 1]) nd++;
                reqb[pidx] = nd;
            }
            if (alt_pix) alt_pix[pidx] = (uint8_t)(alt && !pamb);
            if (alt_rgba) {
                alt_rgba[pidx * 4 + 0] = Ca[0];
                alt_rgba[pidx * 4 + 1] = Ca[1];
                alt_rgba[pidx * 4 + 2] = Ca[2];
                alt_rgba[pidx * 4 + 3] = Aa;
            }
            if (pamb) st_ap++;
        }
    }
    free(SM.tiles);
    free(rkeys);
    }
#undef DMM
    free(node_mm);
    if (stats) {
        stats->samples = st_s;
        stats->channel_samples = st_cs;
        stats->missing = st_m;
        stats->amb_samples = st_as;
        stats->amb_pixels = st_ap;
    }
    return 0;
}

/* O4: brute-force marcher over the full level-lambda arrays: same rays,
 * samples, transfer functions, mix and compositing; no bricks, no tree, no
 * emptiness test, no residency. */
int or_brute(const or_volume *V, const void *const *lvl, int lambda, const or_frame *Fr,
             double *rgba) {
    geo_t G;
    geo(V, &G);
    if (lambda < 0 || lambda >= G.L || !lvl) return -1;
    sampler_t SM = {V, lvl, NULL, NULL, NULL, (const int(*)[3])G.dl, (const int(*)[3])G.f, G.L};
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < Fr->H; ++j)
        for (int i = 0; i < Fr->W; ++i) {
            double o[3], d[3], t0, t1, Cc[3] = {0, 0, 0}, A = 0.0;
            pixel_ray(V, Fr, i, j, o, d);
            if (box_interval(V, o, d, &t0, &t1)) {
                long long k0 = (long long)floor(t0 / Fr->delta) - 1;
                long long k1 = (long long)ceil(t1 / Fr->delta) + 1;
                if (k0 < 0) k0 = 0;
                for (long long k = k0; k <= k1; ++k) {
                    double t = (double)k * Fr->delta, u[3];
                    int inside = 1;
                    for (int a = 0; a < 3; ++a) {
                        u[a] = o[a] + t * d[a];
                        if (!(u[a] >= 0.0 && u[a] < (double)V->dims[a])) inside = 0;
                    }
                    if (!inside) continue;
                    double prod = 1.0, sa = 0.0, srgb[3] = {0, 0, 0};
                    for (int jv = 0; jv < Fr->nvis; ++jv) {
                        int c = Fr->vis[jv];
                        double q[3];
                        for (int a = 0; a < 3; ++a) q[a] = u[a] / G.f[lambda][a];
                        double v = trilinear(&SM, c, lambda, q);
                        double r[4];
                        tf_eval(v, Fr->W0[jv], Fr->W1[jv], Fr->tf[jv], r);
                        prod *= (1.0 - r[3]);
                        sa += r[3];
                        for (int k2 = 0; k2 < 3; ++k2) srgb[k2] += r[3] * r[k2];
                    }
                    double as = 1.0 - prod, Cs[3] = {0, 0, 0};
                    if (sa > 0.0)
                        for (int k2 = 0; k2 < 3; ++k2) Cs[k2] = as * srgb[k2] / sa;
                    for (int k2 = 0; k2 < 3; ++k2) Cc[k2] += (1.0 - A) * Cs[k2];
                    A += (1.0 - A) * as;
                    if (A >= Fr->term_alpha) break;
                }
            }
            long long p = (long long)j * Fr->W + i;
            rgba[p * 4 + 0] = Cc[0];
            rgba[p * 4 + 1] = Cc[1];
            rgba[p * 4 + 2] = Cc[2];
            rgba[p * 4 + 3] = A;
        }
    return 0;
}

/* ------------------------------------------------------- cache / LRU */

/* Cache state: slot_brick[S] (dense brick or -1 when free), stamp[S]
 * (frame of last use or upload), seq[S] (upload order), *seq_next. */

/* Plain request-driven policy: requested bricks ordered by (count
 * descending, ID ascending), already-resident ones dropped, at most U.
 * counts[dense]; ids[dense] gives each brick's ID.  Returns n and fills
 * out_dense[<=U]. */
int or_plain_policy(long long total, const uint32_t *counts, const uint32_t *ids,
                    const int32_t *res_slot, int U, long long *out_dense) {
    /* selection by repeated scans keeps this obviously correct; U is small */
    int n = 0;
    uint8_t *taken = (uint8_t *)calloc((size_t)total, 1);
    if (!taken) return -3;
    while (n < U) {
        long long best = -1;
        for (long long i = 0; i < total; ++i) {
            if (!counts[i] || taken[i] || res_slot[i] >= 0) continue;
            if (best < 0 || counts[i] > counts[best] || (counts[i] == counts[best] && ids[i] < ids[best]))
                best = i;
        }
        if (best < 0) break;
        taken[best] = 1;
        out_dense[n++] = best;
    }
    free(taken);
    return n;
}

/* O3: one upload batch in frame f (Sec. 5.3 "LRU cache eviction"):
 *  1. uploads up[0..n) in the caller's order.  An ID resident at the start
 *     of the batch is flagged 2 and its slot is touched (stamp = f), as a use
 *     would; an ID repeated earlier in the batch is flagged 2 as well;
 *  2. eligible slots: free slots in ascending index, then occupied slots in
 *     ascending (stamp, seq), excluding stamp == f (used this frame);
 *  3. the i-th remaining upload takes the i-th eligible slot (flag 1); the
 *     ones left without a slot are flagged 0;
 *  4. an occupied slot's brick is evicted first; the inserted slot gets
 *     stamp = f and seq = the running upload counter.
 * res_slot[dense] and the slot arrays are updated in place.
 * evicted[n] receives the evicted dense brick per upload (-1 if none);
 * slot_out[n] the slot given to each upload (-1 if none). */
int or_stream(long long total, int S, int32_t *res_slot, int64_t *slot_brick, uint32_t *stamp,
              uint32_t *seq, uint32_t *seq_next, uint32_t f, int n, const long long *up,
              uint8_t *flags, int64_t *evicted, int32_t *slot_out) {
    for (int i = 0; i < n; ++i)
        if (up[i] < 0 || up[i] >= total) return -1;
    /* step 1: flags for resident and repeated IDs, touch resident slots */
    for (int i = 0; i < n; ++i) {
        evicted[i] = -1;
        slot_out[i] = -1;
        flags[i] = 0;
        int dup = 0;
        for (int k = 0; k < i && !dup; ++k)
            if (up[k] == up[i]) dup = 1;
        if (dup) { flags[i] = 2; continue; }
        if (res_slot[up[i]] >= 0) {
            flags[i] = 2;
            stamp[res_slot[up[i]]] = f;
        }
    }
    /* step 2: eligible slot order */
    int32_t *el = (int32_t *)malloc(sizeof(int32_t) * (S > 0 ? S : 1));
    if (!el) return -3;
    int ne = 0;
    for (int s = 0; s < S; ++s)
        if (slot_brick[s] < 0) el[ne++] = s;
    int nfree = ne;
    for (int s = 0; s < S; ++s)
        if (slot_brick[s] >= 0 && stamp[s] != f) el[ne++] = s;
    /* insertion sort of the occupied part by (stamp, seq): plain and exact */
    for (int a = nfree + 1; a < ne; ++a) {
        int32_t x = el[a];
        int b = a - 1;
        while (b >= nfree && (stamp[el[b]] > stamp[x] || (stamp[el[b]] == stamp[x] && seq[el[b]] > seq[x]))) {
            el[b + 1] = el[b];
            b--;
        }
        el[b + 1] = x;
    }
    /* steps 3-4 */
    int next = 0;
    for (int i = 0; i < n; ++i) {
        if (flags[i] == 2) continue;
        if (next >= ne) { flags[i] = 0; continue; }
        int s = el[next++];
        if (slot_brick[s] >= 0) {
            evicted[i] = slot_brick[s];
            res_slot[slot_brick[s]] = -1;
        }
        slot_brick[s] = up[i];
        res_slot[up[i]] = s;
        stamp[s] = f;
        seq[s] = (*seq_next)++;
        flags[i] = 1;
        slot_out[i] = s;
    }
    free(el);
    return 0;
}
