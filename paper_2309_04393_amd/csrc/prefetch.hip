// Predictor rows, history, labels and candidates for the brick-request
// predictor (an addition to the paper's method: it decides which extra
// bricks a policy streams, never how a frame is rendered).
//
// Rows: one per (cache channel c, L0 brick position p); row = c * P + p with
// p = (pz * nby + py) * nbx + px over the L0 brick grid.
// History: one byte per brick; bits 0-3 = requested in frames f, f-1, f-2,
// f-3; bits 4-7 = read in those frames.
// Features (24, FP16), for the row's brick centre q (world units) and the
// frame's camera, t = distance from the eye (orthographic: along forward):
//   0 log2(brick edge in pixels at t) / 8      1 log2(t / D_1) / 8
//   2 desired level at q / 8                   3 q inside the view frustum (0/1)
//   4, 5 projected x, y (clamped to [-2, 2]) / 2
//   6 brick z / bricks in z                    7 fraction of the brick's leaves
//                                                not empty for c under its TF
//   8..11 requested bits of the L0 brick       12..15 read bits of the L0 brick
//   16..23 residency of the bricks covering p at levels 0..7
// Labels for rows whose features were taken 4 frames earlier: level l is 1
// iff the level-l brick covering p was requested or read in the last 4
// frames; mask = 1 for l < number of levels.
#include <math.h>
#include <string.h>

#include "common.h"

namespace ro {

struct PfArgs {
    int32_t m, L, Blog, nbx, nby, nbz;
    uint32_t per_channel;
    uint32_t loff[kMaxL];
    uint32_t nbxl[kMaxL], nbyl[kMaxL];
    uint32_t lsh[kMaxL];  // packed level factor shifts
    double sp[3];
    double eye[3], F[3], R[3], U[3], tx, ty, pix;
    double D[kMaxL];  // desired-level distance thresholds (l >= 1)
    int32_t proj;
    int32_t nvis;
    int32_t vis[kMaxC];
    uint32_t W0[kMaxC], W1[kMaxC];
    // tree
    int32_t depth, leaf_log[3];
    uint32_t leaf_off, nlx_log, nly_log;
    const uint32_t *meta;
    const uint32_t *pt;
    const uint8_t *hist;
    const float4 *tf;  // [nvis][256]
};

__device__ __forceinline__ uint32_t fld(uint32_t p, int a) { return (p >> (8 * a)) & 255u; }

// A leaf range [mn, mx] is empty for a table iff every entry reachable by
// interpolation from values in the range has alpha 0 (exact integers).
__device__ inline bool pf_empty(uint32_t mm, uint32_t W0, uint32_t W1, const float4 *tf) {
    const long long mn = mm & 0xFFFF, mx = mm >> 16;
    const long long den = (long long)W1 - (long long)W0;
    const long long nlo = 255LL * (mn * 256 - (long long)W0), nhi = 255LL * (mx * 256 - (long long)W0);
    long long lo = nlo <= 0 ? 0 : nlo / den, hi = nhi <= 0 ? 0 : (nhi + den - 1) / den;
    lo = lo > 255 ? 255 : lo;
    hi = hi > 255 ? 255 : hi;
    for (long long e = lo; e <= hi; ++e)
        if (tf[e].w != 0.0f) return false;
    return true;
}

__global__ void __launch_bounds__(256) k_pf_features(const PfArgs A, _Float16 *__restrict__ x) {
    const uint32_t P = (uint32_t)A.nbx * A.nby * A.nbz;
    const uint32_t row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= P * (uint32_t)A.m) return;
    const int c = (int)(row / P);
    const uint32_t p = row - (uint32_t)c * P;
    const int px = (int)(p % A.nbx), py = (int)((p / A.nbx) % A.nby), pz = (int)(p / ((uint32_t)A.nbx * A.nby));
    const double B = (double)(1 << A.Blog);
    double q[3] = {(px + 0.5) * B * A.sp[0], (py + 0.5) * B * A.sp[1], (pz + 0.5) * B * A.sp[2]};
    double v[3] = {q[0] - A.eye[0], q[1] - A.eye[1], q[2] - A.eye[2]};
    const double zf = v[0] * A.F[0] + v[1] * A.F[1] + v[2] * A.F[2];
    const double xr = v[0] * A.R[0] + v[1] * A.R[1] + v[2] * A.R[2];
    const double yu = v[0] * A.U[0] + v[1] * A.U[1] + v[2] * A.U[2];
    double t, sx, sy;
    if (A.proj == RO_PROJ_ORTHO) {
        t = fmax(zf, 1e-6);
        sx = xr / A.tx;
        sy = yu / A.ty;
    } else {
        t = fmax(sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]), 1e-6);
        const double zz = fmax(zf, 1e-6);
        sx = xr / (zz * A.tx);
        sy = yu / (zz * A.ty);
    }
    const double foot = A.proj == RO_PROJ_ORTHO ? A.pix : t * A.pix;
    float f[24];
    f[0] = (float)fmin(fmax(log2(B * A.sp[0] / foot), -8.0), 8.0) / 8.0f;
    f[1] = A.L > 1 ? (float)fmin(fmax(log2(t / A.D[1]), -8.0), 8.0) / 8.0f : 0.0f;
    int lod = 0;
    for (int l = 1; l < A.L; ++l)
        if (A.proj == RO_PROJ_ORTHO ? A.pix >= (double)(1 << fld(A.lsh[l], 0)) * A.sp[0] : t >= A.D[l]) ++lod;
    f[2] = (float)lod / 8.0f;
    const bool inview = zf > 0.0 && fabs(sx) <= 1.0 && fabs(sy) <= 1.0;
    f[3] = inview ? 1.0f : 0.0f;
    f[4] = (float)fmin(fmax(sx, -2.0), 2.0) / 2.0f;
    f[5] = (float)fmin(fmax(sy, -2.0), 2.0) / 2.0f;
    f[6] = (float)(pz + 0.5) / (float)A.nbz;
    // leaves of this brick that are not empty for c (visible channels only)
    int j = -1;
    for (int k = 0; k < A.nvis; ++k)
        if (A.vis[k] == c) j = k;
    float frac = 0.0f;
    if (j >= 0) {
        const int lx = A.Blog - A.leaf_log[0], ly = A.Blog - A.leaf_log[1], lz = A.Blog - A.leaf_log[2];
        int tot = 0, ne = 0;
        for (int az = 0; az < (1 << lz); ++az)
            for (int ay = 0; ay < (1 << ly); ++ay)
                for (int ax = 0; ax < (1 << lx); ++ax) {
                    const uint32_t gx = ((uint32_t)px << lx) + ax, gy = ((uint32_t)py << ly) + ay,
                                   gz = ((uint32_t)pz << lz) + az;
                    const uint32_t leaf = A.leaf_off + (((gz << A.nly_log) + gy) << A.nlx_log) + gx;
                    ++tot;
                    if (!pf_empty(A.meta[(size_t)leaf * A.m + c], A.W0[j], A.W1[j], A.tf + j * 256)) ++ne;
                }
        frac = (float)ne / (float)tot;
    }
    f[7] = frac;
    const uint32_t b0 = (uint32_t)c * A.per_channel + A.loff[0] + p;
    const uint8_t h = A.hist[b0];
    for (int k = 0; k < 4; ++k) {
        f[8 + k] = (float)((h >> k) & 1u);
        f[12 + k] = (float)((h >> (4 + k)) & 1u);
    }
    for (int l = 0; l < 8; ++l) {
        float r = 0.0f;
        if (l < A.L) {
            const uint32_t bx = (uint32_t)px >> fld(A.lsh[l], 0), by = (uint32_t)py >> fld(A.lsh[l], 1),
                           bz = (uint32_t)pz >> fld(A.lsh[l], 2);
            const uint32_t b = (uint32_t)c * A.per_channel + A.loff[l] + (bz * A.nbyl[l] + by) * A.nbxl[l] + bx;
            r = A.pt[b] != kInvalid ? 1.0f : 0.0f;
        }
        f[16 + l] = r;
    }
    _Float16 *o = x + (size_t)row * 32;
    for (int k = 0; k < 24; ++k) o[k] = (_Float16)f[k];
    for (int k = 24; k < 32; ++k) o[k] = (_Float16)0.0f;
}

// History: shift, then record this frame's requests (counter > 0) and reads
// (resident and stamped with the frame).
__global__ void k_pf_record(uint8_t *__restrict__ hist, const uint32_t *__restrict__ cnt,
                            const uint32_t *__restrict__ pt, const uint32_t *__restrict__ stamp, uint64_t n,
                            uint32_t frame) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const uint32_t s = pt[b];
    const uint32_t req = cnt[b] != 0, use = s != kInvalid && stamp[s] == frame;
    hist[b] = (uint8_t)(((hist[b] << 1) & 0xEEu) | req | (use << 4));
}

__global__ void k_pf_labels(const PfArgs A, uint8_t *__restrict__ y, uint8_t *__restrict__ mask) {
    const uint32_t P = (uint32_t)A.nbx * A.nby * A.nbz;
    const uint32_t row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= P * (uint32_t)A.m) return;
    const int c = (int)(row / P);
    const uint32_t p = row - (uint32_t)c * P;
    const uint32_t px = p % A.nbx, py = (p / A.nbx) % A.nby, pz = p / ((uint32_t)A.nbx * A.nby);
    for (int l = 0; l < 16; ++l) {
        uint8_t yy = 0, mm = 0;
        if (l < A.L && l < 9) {
            const uint32_t bx = px >> fld(A.lsh[l], 0), by = py >> fld(A.lsh[l], 1), bz = pz >> fld(A.lsh[l], 2);
            const uint32_t b = (uint32_t)c * A.per_channel + A.loff[l] + (bz * A.nbyl[l] + by) * A.nbxl[l] + bx;
            yy = A.hist[b] != 0;
            mm = 1;
        }
        y[(size_t)row * 16 + l] = yy;
        mask[(size_t)row * 16 + l] = mm;
    }
}

// Candidate bricks: not resident, predicted with probability above the
// threshold; each brick keeps the best probability over its rows (float bits
// of a positive number order like unsigned integers).
__global__ void k_pf_candidates(const PfArgs A, const float *__restrict__ z, float thr,
                                uint32_t *__restrict__ score) {
    const uint32_t P = (uint32_t)A.nbx * A.nby * A.nbz;
    const uint32_t row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= P * (uint32_t)A.m) return;
    const int c = (int)(row / P);
    const uint32_t p = row - (uint32_t)c * P;
    const uint32_t px = p % A.nbx, py = (p / A.nbx) % A.nby, pz = p / ((uint32_t)A.nbx * A.nby);
    for (int l = 0; l < A.L && l < 9; ++l) {
        const float pr = 1.0f / (1.0f + expf(-z[(size_t)row * 16 + l]));
        if (!(pr > thr)) continue;
        const uint32_t bx = px >> fld(A.lsh[l], 0), by = py >> fld(A.lsh[l], 1), bz = pz >> fld(A.lsh[l], 2);
        const uint32_t b = (uint32_t)c * A.per_channel + A.loff[l] + (bz * A.nbyl[l] + by) * A.nbxl[l] + bx;
        if (A.pt[b] != kInvalid) continue;
        atomicMax(&score[b], __float_as_uint(pr));
    }
}

}  // namespace ro

using namespace ro;

struct ro_prefetch {
    ro_octree *tree;
    uint8_t *hist;
    uint32_t *score;
    uint32_t rows;
};

extern "C" ro_status ro_pf_query(const ro_octree *t, uint32_t *rows, size_t *hist_bytes, size_t *score_bytes) {
    RO_CHECK(t && rows && hist_bytes && score_bytes, RO_E_ARG, "null argument");
    const VolGeo &g = t->cache->vol->g;
    RO_CHECK(t->t.leaf_log[0] <= g.Blog && t->t.leaf_log[1] <= g.Blog && t->t.leaf_log[2] <= g.Blog, RO_E_ARG,
             "bad tree");
    *rows = (uint32_t)(g.nb[0][0] * g.nb[0][1] * g.nb[0][2]) * (uint32_t)g.m;
    *hist_bytes = g.total;
    *score_bytes = 4 * g.total;
    return RO_OK;
}

extern "C" ro_status ro_pf_create(ro_octree *t, uint8_t *hist_dev, uint32_t *score_dev, void *stream,
                                  ro_prefetch **out) {
    RO_CHECK(t && hist_dev && score_dev && out, RO_E_ARG, "null argument");
    const VolGeo &g = t->cache->vol->g;
    RO_CHECK(g.L <= kMaxL, RO_E_ARG, "too many levels");
    ro_prefetch *p = new (std::nothrow) ro_prefetch;
    RO_CHECK(p, RO_E_NOMEM, "out of host memory");
    p->tree = t;
    p->hist = hist_dev;
    p->score = score_dev;
    p->rows = (uint32_t)(g.nb[0][0] * g.nb[0][1] * g.nb[0][2]) * (uint32_t)g.m;
    hipStream_t s = (hipStream_t)stream;
    ro_status st;
    if ((st = launch_fill_u8(hist_dev, g.total, 0, s)) || (st = launch_fill_u32(score_dev, g.total, 0, s))) {
        delete p;
        return st;
    }
    *out = p;
    return RO_OK;
}

extern "C" void ro_pf_destroy(ro_prefetch *p) { delete p; }

static ro_status pf_args(const ro_prefetch *pf, const ro_frame_desc *fd, PfArgs &A) {
    const ro_octree *t = pf->tree;
    const VolGeo &g = t->cache->vol->g;
    memset(&A, 0, sizeof(A));
    A.m = g.m;
    A.L = g.L;
    A.Blog = g.Blog;
    A.nbx = g.nb[0][0];
    A.nby = g.nb[0][1];
    A.nbz = g.nb[0][2];
    A.per_channel = g.per_channel;
    for (int l = 0; l < g.L; ++l) {
        A.loff[l] = g.loff[l];
        A.nbxl[l] = (uint32_t)g.nb[l][0];
        A.nbyl[l] = (uint32_t)g.nb[l][1];
        A.lsh[l] = (uint32_t)g.lshift[l][0] | ((uint32_t)g.lshift[l][1] << 8) | ((uint32_t)g.lshift[l][2] << 16);
    }
    for (int k = 0; k < 3; ++k) A.sp[k] = g.spacing[k];
    A.depth = t->t.depth;
    for (int k = 0; k < 3; ++k) A.leaf_log[k] = t->t.leaf_log[k];
    A.leaf_off = t->t.noff[t->t.depth];
    A.nlx_log = (uint32_t)t->t.nlog[t->t.depth][0];
    A.nly_log = (uint32_t)t->t.nlog[t->t.depth][1];
    A.meta = t->b.node_meta;
    A.pt = t->cache->b.page_table;
    A.hist = pf->hist;
    if (fd) {
        RO_CHECK(fd->n_vis >= 1 && fd->n_vis <= g.m && fd->tf_dev && fd->height > 0 && fd->ty > 0 && fd->lod_bias > 0,
                 RO_E_ARG, "bad frame");
        for (int k = 0; k < 3; ++k) {
            A.eye[k] = fd->eye[k];
            A.F[k] = fd->forward[k];
            A.R[k] = fd->right[k];
            A.U[k] = fd->up[k];
        }
        A.tx = fd->tx;
        A.ty = fd->ty;
        A.proj = fd->projection;
        A.pix = 2.0 * fd->ty / fd->height;
        for (int l = 1; l < g.L; ++l) A.D[l] = (double)(1 << g.lshift[l][0]) * g.spacing[0] / (fd->lod_bias * A.pix);
        A.pix *= fd->lod_bias;
        A.nvis = fd->n_vis;
        for (int j = 0; j < fd->n_vis; ++j) {
            A.vis[j] = fd->vis[j];
            A.W0[j] = fd->win_lo[j];
            A.W1[j] = fd->win_hi[j];
            RO_CHECK(fd->win_lo[j] < fd->win_hi[j], RO_E_ARG, "bad window");
        }
        A.tf = (const float4 *)fd->tf_dev;
    }
    return RO_OK;
}

extern "C" ro_status ro_pf_record(ro_prefetch *pf, uint32_t frame, void *stream) {
    RO_CHECK(pf, RO_E_ARG, "null argument");
    const ro_cache *c = pf->tree->cache;
    const uint64_t n = c->vol->g.total;
    hipLaunchKernelGGL(k_pf_record, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, pf->hist,
                       c->b.counters, c->b.page_table, c->b.stamps, n, frame);
    RO_HIP(hipGetLastError());
    return RO_OK;
}

extern "C" ro_status ro_pf_features(ro_prefetch *pf, const ro_frame_desc *fd, uint16_t *x_dev, void *stream) {
    RO_CHECK(pf && fd && x_dev, RO_E_ARG, "null argument");
    PfArgs A;
    ro_status st = pf_args(pf, fd, A);
    if (st) return st;
    hipLaunchKernelGGL(k_pf_features, dim3((pf->rows + 255) / 256), dim3(256), 0, (hipStream_t)stream, A,
                       (_Float16 *)x_dev);
    RO_HIP(hipGetLastError());
    return RO_OK;
}

extern "C" ro_status ro_pf_labels(ro_prefetch *pf, uint8_t *y_dev, uint8_t *mask_dev, void *stream) {
    RO_CHECK(pf && y_dev && mask_dev, RO_E_ARG, "null argument");
    PfArgs A;
    ro_status st = pf_args(pf, nullptr, A);
    if (st) return st;
    hipLaunchKernelGGL(k_pf_labels, dim3((pf->rows + 255) / 256), dim3(256), 0, (hipStream_t)stream, A, y_dev, mask_dev);
    RO_HIP(hipGetLastError());
    return RO_OK;
}

extern "C" ro_status ro_pf_candidates(ro_prefetch *pf, const float *z_dev, float threshold, uint32_t cap,
                                      uint32_t *ids_host, float *prob_host, uint32_t *n_out, void *stream) {
    RO_CHECK(pf && z_dev && n_out && (cap == 0 || (ids_host && prob_host)), RO_E_ARG, "null argument");
    RO_CHECK(threshold >= 0.0f && threshold < 1.0f, RO_E_ARG, "threshold not in [0, 1)");
    PfArgs A;
    ro_status st = pf_args(pf, nullptr, A);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_pf_candidates, dim3((pf->rows + 255) / 256), dim3(256), 0, s, A, z_dev, threshold, pf->score);
    RO_HIP(hipGetLastError());
    // compact the per-brick scores (ascending ID, cleared afterwards)
    std::vector<uint32_t> ids(cap), val(cap);
    uint32_t nu = 0;
    uint64_t tot = 0;
    st = compact_dense(pf->tree->cache, pf->score, cap, ids.data(), val.data(), &nu, &tot, s);
    if (st) return st;
    const uint32_t k = nu < cap ? nu : cap;
    for (uint32_t i = 0; i < k; ++i) {
        ids_host[i] = ids[i];
        float f;
        memcpy(&f, &val[i], 4);
        prob_host[i] = f;
    }
    *n_out = nu;
    return RO_OK;
}
