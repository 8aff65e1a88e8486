// Internal definitions of the residency-octree library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "resoct.h"

namespace ro {

constexpr uint32_t kInvalid = 0xFFFFFFFFu;
constexpr int kMaxC = RO_MAX_CHANNELS;
constexpr int kMaxL = RO_MAX_LEVELS;
constexpr int kMaxD = RO_MAX_DEPTH;
constexpr int kMaxRuns = 128;  // zero-alpha runs of a 256-entry table
constexpr uint32_t kLevelUnknown = 255;  // leaf metadata level of unknown leaves

// Geometry of the bricked hierarchy (host and device copies are identical
// plain structs passed by value).
struct VolGeo {
    int32_t dims[3];
    double spacing[3];
    int32_t m;        // channels
    int32_t bpv;      // bytes per voxel
    int32_t B, Blog;  // brick edge and log2
    int32_t E;        // B + 2
    int32_t L;        // levels
    int32_t ldims[kMaxL][3];
    int32_t lshift[kMaxL][3];  // log2 of the per-axis L0 factor
    int32_t nb[kMaxL][3];      // bricks per axis
    uint32_t loff[kMaxL + 1];  // brick offset of each level inside a channel
    uint32_t per_channel;      // bricks per channel
    uint64_t total;            // bricks over all channels
    uint32_t slot_stride;      // bytes per slot
};

struct TreeGeo {
    int32_t depth;
    int32_t leaf_log[3];
    int32_t nshift[kMaxD + 1][3];  // log2 node edge (L0 voxels) per level
    int32_t nlog[kMaxD + 1][3];    // log2 nodes per axis per level
    uint32_t noff[kMaxD + 2];      // node offset of each level
    uint64_t n_nodes, n_leaves;
};

// Dense brick index (channel-major, then level, then z, y, x).
__host__ __device__ inline uint32_t dense_index(const VolGeo &g, int c, int l, int bx, int by,
                                                int bz) {
    return (uint32_t)c * g.per_channel + g.loff[l] +
           ((uint32_t)bz * (uint32_t)g.nb[l][1] + (uint32_t)by) * (uint32_t)g.nb[l][0] + (uint32_t)bx;
}

__host__ __device__ inline uint32_t dense_to_id(const VolGeo &g, uint32_t d) {
    uint32_t c = d / g.per_channel;
    uint32_t r = d - c * g.per_channel;
    int l = 0;
    while (l + 1 < g.L && g.loff[l + 1] <= r) ++l;
    uint32_t lin = r - g.loff[l];
    uint32_t nx = (uint32_t)g.nb[l][0], ny = (uint32_t)g.nb[l][1];
    uint32_t bx = lin % nx, by = (lin / nx) % ny, bz = lin / (nx * ny);
    return ((c * (uint32_t)g.L + (uint32_t)l) << 24) | (bz << 16) | (by << 8) | bx;
}

__host__ __device__ inline uint32_t node_index(const TreeGeo &t, int d, uint32_t x, uint32_t y,
                                               uint32_t z) {
    return t.noff[d] + (((z << t.nlog[d][1]) + y) << t.nlog[d][0]) + x;
}

// Error handling.
void set_error(const char *fmt, ...);
ro_status hip_fail(hipError_t e, const char *what);

#define RO_HIP(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ro::hip_fail(e_, #call);     \
    } while (0)

#define RO_CHECK(cond, code, ...)            \
    do {                                     \
        if (!(cond)) {                       \
            ro::set_error(__VA_ARGS__);      \
            return (code);                   \
        }                                    \
    } while (0)

}  // namespace ro

// Handles.
struct ro_volume {
    ro_volume_desc desc;
    ro::VolGeo g;
};

// Scratch layout of a cache (byte offsets into bufs.scratch).
struct CacheScratch {
    size_t keys;       // n_slots uint64 LRU keys
    size_t hist;       // 256 uint32 radix histogram
    size_t sel;        // select state (see stream.hip)
    size_t cand;       // max_batch uint64 candidate keys
    size_t victims;    // max_batch uint32
    size_t evicted;    // max_batch uint32
    size_t uploads;    // max_batch uint32 dense indices
    size_t srcidx;     // max_batch uint32 staged index
    size_t touch;      // max_batch uint32 slots to touch
    size_t compact;    // request compaction work space (compact_scratch_bytes of every brick)
    size_t outpairs;   // usage readback output and LRU candidate slots
    size_t total;      // bytes
};

struct ro_cache {
    ro_volume *vol;
    ro_cache_desc desc;
    ro_cache_buffers b;
    CacheScratch sc;
    std::vector<uint32_t> pt_host;     // brick -> slot mirror
    std::vector<uint32_t> slot_host;   // slot -> brick mirror
    std::vector<uint32_t> dirty;       // bricks inserted / evicted since the last residency update
    std::vector<uint32_t> chmap;       // cache channel -> source channel (Sec. 5.2)
    uint32_t seq_next;
};

struct ro_octree {
    ro_cache *cache;
    ro_octree_desc desc;
    ro_octree_buffers b;
    ro::TreeGeo t;
    size_t scratch_bytes;
};

namespace ro {
// Kernel launchers (each returns RO_OK or an error).
ro_status launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
ro_status launch_fill_u16(uint16_t *p, uint64_t n, uint16_t v, hipStream_t s);
ro_status launch_fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s);

ro_status stream_bricks_device(ro_cache *c, uint32_t frame, uint32_t n_new, uint32_t n_touch,
                               const void *staged, hipStream_t s, uint32_t *k_eff_host,
                               uint32_t *victims_host, uint32_t *evicted_host);
ro_status read_requests_device(ro_cache *c, uint32_t cap, uint32_t *ids, uint32_t *counts,
                               uint32_t *n_unique, uint64_t *total, hipStream_t s);
size_t compact_scratch_bytes(uint64_t n, uint32_t lim);
ro_status compact_dense_ws(const VolGeo &g, uint32_t *arr, uint8_t *ws, uint32_t lim, uint32_t cap, uint32_t *ids,
                           uint32_t *counts, uint32_t *n_unique, uint64_t *total, hipStream_t s);
ro_status read_requests_noalloc_device(ro_cache *c, uint32_t cap, uint32_t *ids, uint32_t *counts,
                                       uint32_t *n_unique, uint64_t *total, hipStream_t s);
ro_status compact_dense(ro_cache *c, uint32_t *arr, uint32_t cap, uint32_t *ids, uint32_t *vals,
                        uint32_t *n_unique, uint64_t *total, hipStream_t s);
ro_status cache_evict_channel(ro_cache *c, uint32_t ch, hipStream_t s);
ro_status read_usage_device(ro_cache *c, uint32_t frame, uint32_t cap, uint32_t *slots,
                            uint32_t *n_out, hipStream_t s);

ro_status octree_set_meta(ro_octree *t, uint32_t channel, const uint16_t *leaf_mm, hipStream_t s);
ro_status octree_update(ro_octree *t, const std::vector<uint32_t> &dirty, hipStream_t s);
ro_status octree_rebuild(ro_octree *t, hipStream_t s);
ro_status octree_meta_from_bricks(ro_octree *t, const std::vector<uint32_t> &dense, hipStream_t s);

ro_status render_device(ro_octree *t, const ro_frame_desc *fd, float *rgba, hipStream_t s);
ro_status validate_frame(const ro_octree *t, const ro_frame_desc *fd, const float *rgba);
}  // namespace ro
