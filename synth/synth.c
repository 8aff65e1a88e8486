/*
 * synth.c — seeded synthetic volume generator (the "data server").
 *
 * This module produces input data only: voxel values of a bricked
 * multi-resolution multi-channel volume hierarchy and conservative
 * per-region metadata, the two things the paper's server provides
 * (Sec. 4 System Overview: a server holding the bricked hierarchy, which may
 * also answer metadata queries for regions of the volume).  It holds none of
 * the rendering method's arithmetic: no page tables, trees, sampling,
 * transfer functions or compositing.  Both the CPU oracle and the GPU path
 * consume its output bytes.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), keyed by
 * (seed, purpose, index) so that every brick / region can be produced on
 * demand and independently.
 *
 * Two volume families:
 *  - blobs: sum of isotropic Gaussian blobs plus uniform noise, full arrays
 *    (small volumes); coarser levels are made by the caller with
 *    synth_downsample (2x box filter, round half up).
 *  - cells: Poisson-placed ellipsoidal "cells" with lognormal per-channel
 *    intensity, optional low-frequency tissue mask and per-channel gain;
 *    any level, any box, on demand.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t sm_next(uint64_t *s) {
    *s += SM_GAMMA;
    return sm_mix(*s);
}

/* Stream key for (seed, purpose, index): three chained mixes. */
uint64_t synth_key(uint64_t seed, uint64_t purpose, uint64_t index) {
    uint64_t z = sm_mix(seed + SM_GAMMA);
    z = sm_mix(z ^ (purpose * 0xD1B54A32D192ED03ULL + SM_GAMMA));
    z = sm_mix(z ^ (index * 0xAEF17502108EF2D9ULL + SM_GAMMA));
    return z;
}

static inline double u01(uint64_t *s) { return (double)(sm_next(s) >> 11) * 0x1.0p-53; }

static double normal01(uint64_t *s) {
    double u1 = u01(s), u2 = u01(s);
    if (u1 < 0x1.0p-60) u1 = 0x1.0p-60;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static int poisson(uint64_t *s, double lambda) {
    /* Knuth's multiplicative method; lambda here is at most a few hundred. */
    double L = exp(-lambda), p = 1.0;
    int k = 0;
    do { k++; p *= u01(s); } while (p > L);
    return k - 1;
}

/* Purposes. */
enum { P_BLOB = 1, P_NOISE = 2, P_CELLS = 3, P_TISSUE = 4, P_GAIN = 5 };

static inline double clamp01(double x) { return x < 0 ? 0 : (x > 1 ? 1 : x); }

/* ------------------------------------------------------------------ blobs */

/* Fill out[nz][ny][nx] (uint8 if bits==8 else uint16) with
 * f(x) = sum_b A_b exp(-|x - mu_b|^2 / (2 sigma_b^2)) + U[0, noise),
 * clamped to [0,1] and rounded half up to the integer range.
 * Blob centers mu ~ U[0, n)^3 in voxel units; voxel i is centered at i+0.5. */
int synth_blobs(int nx, int ny, int nz, int n_blobs, double smin, double smax,
                double amin, double amax, double noise, uint64_t seed, int bits,
                void *out) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || n_blobs < 0 || (bits != 8 && bits != 16)) return -1;
    double *bp = (double *)malloc(sizeof(double) * 5 * (n_blobs > 0 ? n_blobs : 1));
    if (!bp) return -3;
    uint64_t s = synth_key(seed, P_BLOB, 0);
    for (int b = 0; b < n_blobs; ++b) {
        bp[5 * b + 0] = nx * u01(&s);
        bp[5 * b + 1] = ny * u01(&s);
        bp[5 * b + 2] = nz * u01(&s);
        bp[5 * b + 3] = smin + (smax - smin) * u01(&s);
        bp[5 * b + 4] = amin + (amax - amin) * u01(&s);
    }
    const double maxv = bits == 8 ? 255.0 : 65535.0;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            uint64_t ns = synth_key(seed, P_NOISE, (uint64_t)z * (uint64_t)ny + (uint64_t)y);
            for (int x = 0; x < nx; ++x) {
                double px = x + 0.5, py = y + 0.5, pz = z + 0.5, f = 0.0;
                for (int b = 0; b < n_blobs; ++b) {
                    double dx = px - bp[5 * b], dy = py - bp[5 * b + 1], dz = pz - bp[5 * b + 2];
                    double sg = bp[5 * b + 3];
                    f += bp[5 * b + 4] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * sg * sg));
                }
                f += noise * u01(&ns);
                double v = floor(clamp01(f) * maxv + 0.5);
                size_t i = ((size_t)z * ny + y) * nx + x;
                if (bits == 8) ((uint8_t *)out)[i] = (uint8_t)v;
                else ((uint16_t *)out)[i] = (uint16_t)v;
            }
        }
    }
    free(bp);
    return 0;
}

/* 2x box filter on the axes flagged in h[3]: each output voxel is the mean
 * of the existing children (1, 2, 4 or 8 of them at ragged borders),
 * rounded half up: floor((sum + n/2) / n). Output dims ceil(n/2) on halved
 * axes, unchanged elsewhere. */
int synth_downsample(const void *src, int bits, int sx, int sy, int sz, int hx, int hy,
                     int hz, void *dst) {
    if (bits != 8 && bits != 16) return -1;
    int dx = hx ? (sx + 1) / 2 : sx, dy = hy ? (sy + 1) / 2 : sy, dz = hz ? (sz + 1) / 2 : sz;
    int fx = hx ? 2 : 1, fy = hy ? 2 : 1, fz = hz ? 2 : 1;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < dz; ++z)
        for (int y = 0; y < dy; ++y)
            for (int x = 0; x < dx; ++x) {
                uint64_t sum = 0, n = 0;
                for (int cz = 0; cz < fz; ++cz)
                    for (int cy = 0; cy < fy; ++cy)
                        for (int cx = 0; cx < fx; ++cx) {
                            int X = x * fx + cx, Y = y * fy + cy, Z = z * fz + cz;
                            if (X >= sx || Y >= sy || Z >= sz) continue;
                            size_t i = ((size_t)Z * sy + Y) * sx + X;
                            sum += bits == 8 ? ((const uint8_t *)src)[i] : ((const uint16_t *)src)[i];
                            n++;
                        }
                uint64_t v = (sum + n / 2) / n;
                size_t o = ((size_t)z * dy + y) * dx + x;
                if (bits == 8) ((uint8_t *)dst)[o] = (uint8_t)v;
                else ((uint16_t *)dst)[o] = (uint16_t)v;
            }
    return 0;
}

/* ------------------------------------------------------------------ cells */

#define MAXCH 16

typedef struct {
    double c[3], r[3], sg[3];
    float inten[MAXCH];
} cell_t;

typedef struct {
    int dims[3];
    int nch;
    double density, rmin, rmax, mu, sigma;
    uint64_t seed;
    int region;            /* edge of the Poisson regions, L0 voxels */
    int nreg[3];           /* regions per axis */
    int tissue;            /* 1: multiply intensities by tissue mask and gain */
    double tissue_feature; /* lattice spacing of the tissue value noise */
    double gain_feature;
} cells_ctx;

static inline double smoothstep(double e0, double e1, double x) {
    double t = clamp01((x - e0) / (e1 - e0));
    return t * t * (3.0 - 2.0 * t);
}

/* 2-D value noise in [0,1): random lattice values, smoothstep-weighted
 * bilinear interpolation. */
static double value_noise(uint64_t seed, uint64_t purpose, double x, double y, double feat) {
    double gx = x / feat, gy = y / feat;
    double fx = floor(gx), fy = floor(gy);
    int64_t ix = (int64_t)fx, iy = (int64_t)fy;
    double tx = gx - fx, ty = gy - fy;
    tx = tx * tx * (3 - 2 * tx);
    ty = ty * ty * (3 - 2 * ty);
    double v[4];
    for (int k = 0; k < 4; ++k) {
        uint64_t idx = ((uint64_t)(ix + (k & 1) + 1024) << 32) | (uint64_t)(iy + (k >> 1) + 1024);
        uint64_t s = synth_key(seed, purpose, idx);
        v[k] = u01(&s);
    }
    double a = v[0] + (v[1] - v[0]) * tx, b = v[2] + (v[3] - v[2]) * tx;
    return a + (b - a) * ty;
}

void *synth_cells_create(int nx, int ny, int nz, int nch, double density, double rmin,
                         double rmax, double mu, double sigma, uint64_t seed, int tissue,
                         double tissue_feature, double gain_feature, int region) {
    if (nch <= 0 || nch > MAXCH || nx <= 0 || ny <= 0 || nz <= 0 || region <= 0) return NULL;
    cells_ctx *c = (cells_ctx *)calloc(1, sizeof(cells_ctx));
    if (!c) return NULL;
    c->dims[0] = nx; c->dims[1] = ny; c->dims[2] = nz;
    c->nch = nch; c->density = density; c->rmin = rmin; c->rmax = rmax;
    c->mu = mu; c->sigma = sigma; c->seed = seed; c->region = region;
    for (int a = 0; a < 3; ++a) c->nreg[a] = (c->dims[a] + region - 1) / region;
    c->tissue = tissue; c->tissue_feature = tissue_feature; c->gain_feature = gain_feature;
    return c;
}

void synth_cells_destroy(void *ctx) { free(ctx); }

/* Tissue factor at (x, y): smoothstep(0.45, 0.55, noise), exactly 0 on
 * roughly half of the slide. */
double synth_tissue(void *ctx, double x, double y) {
    cells_ctx *C = (cells_ctx *)ctx;
    return smoothstep(0.45, 0.55, value_noise(C->seed, P_TISSUE, x, y, C->tissue_feature));
}

/* Generate the cells of one region into out (capacity cap); returns count.
 * Region index r = (rz * nreg_y + ry) * nreg_x + rx. */
static int region_cells(const cells_ctx *C, int rx, int ry, int rz, cell_t *out, int cap) {
    uint64_t r = ((uint64_t)rz * C->nreg[1] + ry) * C->nreg[0] + rx;
    uint64_t s = synth_key(C->seed, P_CELLS, r);
    double R = C->region;
    int n = poisson(&s, C->density * R * R * R);
    int k = 0;
    for (int i = 0; i < n; ++i) {
        cell_t cl;
        cl.c[0] = rx * R + R * u01(&s);
        cl.c[1] = ry * R + R * u01(&s);
        cl.c[2] = rz * R + R * u01(&s);
        for (int a = 0; a < 3; ++a) {
            cl.r[a] = C->rmin + (C->rmax - C->rmin) * u01(&s);
            cl.sg[a] = cl.r[a] / 2.5;
        }
        double tmod = 1.0;
        if (C->tissue) tmod = synth_tissue((void *)C, cl.c[0], cl.c[1]);
        for (int ch = 0; ch < C->nch; ++ch) {
            double I = exp(C->mu + C->sigma * normal01(&s));
            if (I > 65535.0) I = 65535.0;
            double g = 1.0;
            if (C->tissue)
                g = 0.3 + 0.7 * value_noise(C->seed, P_GAIN + 16 * (uint64_t)ch, cl.c[0], cl.c[1],
                                            C->gain_feature);
            cl.inten[ch] = (float)(I * tmod * g);
        }
        if (tmod <= 0.0) continue; /* no tissue here: the cell is invisible */
        if (k < cap) out[k] = cl;
        k++;
    }
    return k;
}

/* Collect all cells whose bounding box [c-r, c+r] may meet the L0 box
 * [lo, hi) (pass hi - lo > 0). Returns a malloc'ed array and its count. */
static cell_t *collect_cells(const cells_ctx *C, const double lo[3], const double hi[3], int *count) {
    int r0[3], r1[3];
    for (int a = 0; a < 3; ++a) {
        double l = lo[a] - C->rmax, h = hi[a] + C->rmax;
        r0[a] = (int)floor(l / C->region);
        r1[a] = (int)floor(h / C->region);
        if (r0[a] < 0) r0[a] = 0;
        if (r1[a] > C->nreg[a] - 1) r1[a] = C->nreg[a] - 1;
    }
    int cap = 256, n = 0;
    cell_t *arr = (cell_t *)malloc(sizeof(cell_t) * cap);
    cell_t *tmp = (cell_t *)malloc(sizeof(cell_t) * 1024);
    for (int rz = r0[2]; rz <= r1[2]; ++rz)
        for (int ry = r0[1]; ry <= r1[1]; ++ry)
            for (int rx = r0[0]; rx <= r1[0]; ++rx) {
                int k = region_cells(C, rx, ry, rz, tmp, 1024);
                if (k > 1024) k = 1024;
                for (int i = 0; i < k; ++i) {
                    const cell_t *cl = &tmp[i];
                    int meets = 1;
                    for (int a = 0; a < 3; ++a)
                        if (!(cl->c[a] - cl->r[a] < hi[a] && lo[a] < cl->c[a] + cl->r[a])) meets = 0;
                    if (!meets) continue;
                    if (n == cap) {
                        cap *= 2;
                        arr = (cell_t *)realloc(arr, sizeof(cell_t) * cap);
                    }
                    arr[n++] = *cl;
                }
            }
    free(tmp);
    *count = n;
    return arr;
}

/* Integral of exp(-0.5 ((x-c)/s)^2) over [a, b], divided by (b - a). */
static inline double gauss_box_mean(double a, double b, double c, double s) {
    const double k = 0.7071067811865476; /* 1/sqrt(2) */
    return s * 1.2533141373155003 * (erf((b - c) * k / s) - erf((a - c) * k / s)) / (b - a);
}

/* Voxel values of level `level` (per-axis L0 factors f[3]) for the level
 * voxel box [x0, x0+nx) x ... for the channels chans[0..nchan), written as
 * out[ci][z][y][x] uint16.  Level 0: point value at the voxel center,
 * I * exp(-0.5 sum (d/sigma)^2) inside the ellipsoid sum (d/r)^2 < 1, else 0.
 * Level > 0: per cell, product over axes of the box mean of the (untruncated)
 * Gaussian over the voxel's L0 footprint, for cells whose bounding box meets
 * the footprint.  Sums are rounded half up and clamped to 65535.
 * Voxels are not clamped to the level's dims: callers ask for valid boxes. */
int synth_cells_region(void *ctx, const int f[3], int x0, int y0, int z0, int nx, int ny, int nz,
                       int nchan, const int *chans, uint16_t *out) {
    cells_ctx *C = (cells_ctx *)ctx;
    if (!C || nx <= 0 || ny <= 0 || nz <= 0 || nchan <= 0) return -1;
    for (int i = 0; i < nchan; ++i)
        if (chans[i] < 0 || chans[i] >= C->nch) return -1;
    int lvl0 = (f[0] == 1 && f[1] == 1 && f[2] == 1);
    double lo[3] = {(double)x0 * f[0], (double)y0 * f[1], (double)z0 * f[2]};
    double hi[3] = {(double)(x0 + nx) * f[0], (double)(y0 + ny) * f[1], (double)(z0 + nz) * f[2]};
    int nc = 0;
    cell_t *cells = collect_cells(C, lo, hi, &nc);
    size_t nvox = (size_t)nx * ny * nz;
    double *acc = (double *)calloc(nvox * nchan, sizeof(double));
    if (!acc) { free(cells); return -3; }
    int n[3] = {nx, ny, nz}, o[3] = {x0, y0, z0};
    for (int k = 0; k < nc; ++k) {
        const cell_t *cl = &cells[k];
        int i0[3], i1[3];
        for (int a = 0; a < 3; ++a) {
            /* level voxels whose L0 footprint [i f, (i+1) f) meets (c-r, c+r) */
            i0[a] = (int)floor((cl->c[a] - cl->r[a]) / f[a]);
            i1[a] = (int)floor((cl->c[a] + cl->r[a]) / f[a]);
            if (i0[a] < o[a]) i0[a] = o[a];
            if (i1[a] > o[a] + n[a] - 1) i1[a] = o[a] + n[a] - 1;
        }
        if (i0[0] > i1[0] || i0[1] > i1[1] || i0[2] > i1[2]) continue;
        double wx[64], wy[64], wz[64];
        double *w[3] = {wx, wy, wz};
        int tooBig = 0;
        for (int a = 0; a < 3; ++a) {
            if (i1[a] - i0[a] + 1 > 64) { tooBig = 1; break; }
            for (int i = i0[a]; i <= i1[a]; ++i) {
                if (lvl0) {
                    double d = (i + 0.5 - cl->c[a]) / cl->sg[a];
                    w[a][i - i0[a]] = d * d;
                } else {
                    w[a][i - i0[a]] = gauss_box_mean((double)i * f[a], (double)(i + 1) * f[a],
                                                     cl->c[a], cl->sg[a]);
                }
            }
        }
        if (tooBig) continue; /* unreachable: r <= rmax < 32 */
        for (int z = i0[2]; z <= i1[2]; ++z)
            for (int y = i0[1]; y <= i1[1]; ++y)
                for (int x = i0[0]; x <= i1[0]; ++x) {
                    double g;
                    if (lvl0) {
                        double ex = (x + 0.5 - cl->c[0]) / cl->r[0];
                        double ey = (y + 0.5 - cl->c[1]) / cl->r[1];
                        double ez = (z + 0.5 - cl->c[2]) / cl->r[2];
                        if (ex * ex + ey * ey + ez * ez >= 1.0) continue;
                        g = exp(-0.5 * (wx[x - i0[0]] + wy[y - i0[1]] + wz[z - i0[2]]));
                    } else {
                        g = wx[x - i0[0]] * wy[y - i0[1]] * wz[z - i0[2]];
                    }
                    size_t vi = ((size_t)(z - z0) * ny + (y - y0)) * nx + (x - x0);
                    for (int ci = 0; ci < nchan; ++ci)
                        acc[(size_t)ci * nvox + vi] += cl->inten[chans[ci]] * g;
                }
    }
    for (size_t i = 0; i < nvox * nchan; ++i) {
        double v = floor(acc[i] + 0.5);
        out[i] = (uint16_t)(v > 65535.0 ? 65535.0 : v);
    }
    free(acc);
    free(cells);
    return 0;
}

/* Bricks with a 1-voxel halo for a list of brick coordinates at one level:
 * out[i][ci] is a (B+2)^3 uint16 block holding level voxels
 * [b*B - 1, b*B + B] per axis at indices clamped to [0, ldims-1]
 * (clamp-replicate at the level's borders). ldims are the level's dims. */
int synth_cells_bricks(void *ctx, const int f[3], const int ldims[3], int B, int nb,
                       const int *bcoords, int nchan, const int *chans, uint16_t *out) {
    cells_ctx *C = (cells_ctx *)ctx;
    if (!C || B <= 0 || nb < 0) return -1;
    const int E = B + 2;
    const size_t bvox = (size_t)E * E * E;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nb; ++i) {
        int lo[3], hi[3], n[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = bcoords[3 * i + a] * B - 1;
            hi[a] = bcoords[3 * i + a] * B + B; /* inclusive */
            if (lo[a] < 0) lo[a] = 0;
            if (hi[a] > ldims[a] - 1) hi[a] = ldims[a] - 1;
            n[a] = hi[a] - lo[a] + 1;
        }
        if (n[0] <= 0 || n[1] <= 0 || n[2] <= 0) { err = -1; continue; }
        uint16_t *reg = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)n[0] * n[1] * n[2] * nchan);
        if (!reg) { err = -3; continue; }
        if (synth_cells_region(ctx, f, lo[0], lo[1], lo[2], n[0], n[1], n[2], nchan, chans, reg)) {
            err = -1;
            free(reg);
            continue;
        }
        size_t rvox = (size_t)n[0] * n[1] * n[2];
        for (int ci = 0; ci < nchan; ++ci) {
            uint16_t *dst = out + ((size_t)i * nchan + ci) * bvox;
            for (int hz = 0; hz < E; ++hz) {
                int z = bcoords[3 * i + 2] * B - 1 + hz;
                z = z < 0 ? 0 : (z > ldims[2] - 1 ? ldims[2] - 1 : z);
                for (int hy = 0; hy < E; ++hy) {
                    int y = bcoords[3 * i + 1] * B - 1 + hy;
                    y = y < 0 ? 0 : (y > ldims[1] - 1 ? ldims[1] - 1 : y);
                    for (int hx = 0; hx < E; ++hx) {
                        int x = bcoords[3 * i] * B - 1 + hx;
                        x = x < 0 ? 0 : (x > ldims[0] - 1 ? ldims[0] - 1 : x);
                        dst[((size_t)hz * E + hy) * E + hx] =
                            reg[ci * rvox + ((size_t)(z - lo[2]) * n[1] + (y - lo[1])) * n[0] + (x - lo[0])];
                    }
                }
            }
        }
        free(reg);
    }
    return err;
}

/* Conservative per-leaf maxima of the L0 values of all channels:
 * out[c][leaf] = min(65535, ceil(sum of I_c over cells whose bounding box
 * meets the leaf box dilated by one voxel on every side)), leaves of size
 * leaf[3] on a grid nleaf[3] (linear index (z*ny + y)*nx + x).  Any L0 voxel
 * whose center lies within one voxel of the leaf box is bounded by this
 * sum, since every cell profile is at most its intensity. */
int synth_cells_leaf_max(void *ctx, const int leaf[3], const int nleaf[3], uint16_t *out) {
    cells_ctx *C = (cells_ctx *)ctx;
    if (!C) return -1;
    size_t nl = (size_t)nleaf[0] * nleaf[1] * nleaf[2];
    float *acc = (float *)calloc(nl * C->nch, sizeof(float));
    if (!acc) return -3;
    /* Walk regions slab by slab in y to keep the per-thread work balanced;
     * each thread owns disjoint output rows only through atomics-free
     * accumulation into a private buffer merged at the end would cost too
     * much memory at large sizes, so accumulate serially per region row. */
    for (int rz = 0; rz < C->nreg[2]; ++rz)
        for (int ry = 0; ry < C->nreg[1]; ++ry) {
            int nrx = C->nreg[0];
            /* cells of this row of regions */
            for (int rx = 0; rx < nrx; ++rx) {
                static cell_t tmp[1024];
                int k = region_cells(C, rx, ry, rz, tmp, 1024);
                if (k > 1024) k = 1024;
                for (int i = 0; i < k; ++i) {
                    const cell_t *cl = &tmp[i];
                    int l0[3], l1[3], ok = 1;
                    for (int a = 0; a < 3; ++a) {
                        /* leaf [j*L, (j+1)*L) dilated to [j*L - 1, (j+1)*L + 1)
                         * meets (c - r, c + r) */
                        double lo = cl->c[a] - cl->r[a] - 1.0, hi = cl->c[a] + cl->r[a] + 1.0;
                        l0[a] = (int)floor(lo / leaf[a]);
                        l1[a] = (int)floor(hi / leaf[a]);
                        if (l0[a] < 0) l0[a] = 0;
                        if (l1[a] > nleaf[a] - 1) l1[a] = nleaf[a] - 1;
                        if (l0[a] > l1[a]) ok = 0;
                    }
                    if (!ok) continue;
                    for (int z = l0[2]; z <= l1[2]; ++z)
                        for (int y = l0[1]; y <= l1[1]; ++y)
                            for (int x = l0[0]; x <= l1[0]; ++x) {
                                size_t li = ((size_t)z * nleaf[1] + y) * nleaf[0] + x;
                                for (int ch = 0; ch < C->nch; ++ch) acc[(size_t)ch * nl + li] += cl->inten[ch];
                            }
                }
            }
        }
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)(nl * C->nch); ++i) {
        /* float sums: add a relative safety margin before the ceiling */
        double v = ceil((double)acc[i] * (1.0 + 1e-5) + (acc[i] > 0 ? 1.0 : 0.0));
        out[i] = (uint16_t)(v > 65535.0 ? 65535.0 : v);
    }
    free(acc);
    return 0;
}

/* Number of cells (after the tissue cut) in the whole volume, for reporting. */
long long synth_cells_count(void *ctx) {
    cells_ctx *C = (cells_ctx *)ctx;
    long long n = 0;
    static cell_t tmp[1024];
    for (int rz = 0; rz < C->nreg[2]; ++rz)
        for (int ry = 0; ry < C->nreg[1]; ++ry)
            for (int rx = 0; rx < C->nreg[0]; ++rx) n += region_cells(C, rx, ry, rz, tmp, 1024);
    return n;
}
