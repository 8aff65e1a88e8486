// Residency-octree maintenance (Sec. 5.2, Sec. 5.3): metadata reduction,
// incremental residency update with early-stopping OR propagation, and
// from-scratch rebuild.
#include <algorithm>

#include "common.h"

namespace ro {

// Leaf metadata of one channel -> node_meta of the leaf level.
// Leaf metadata of channel c: from the caller's [n_leaves][2] array (level
// 0), or, with leaf_mm null, unknown ([0, unknown_max], level unknown).
__global__ void k_meta_leaf(const uint16_t *__restrict__ leaf_mm, uint32_t *__restrict__ meta,
                            uint8_t *__restrict__ level, uint64_t n_leaves, uint32_t leaf_off, int m, int c,
                            uint32_t unknown_max) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_leaves) return;
    const uint32_t mn = leaf_mm ? leaf_mm[2 * i] : 0u, mx = leaf_mm ? leaf_mm[2 * i + 1] : unknown_max;
    meta[((uint64_t)leaf_off + i) * m + c] = mn | (mx << 16);
    level[i * m + c] = leaf_mm ? 0 : (uint8_t)kLevelUnknown;
}

// Child index range of a level-d node: children per axis are 1 or 2.
__device__ inline void child_range(const TreeGeo &t, int d, uint32_t x, uint32_t y, uint32_t z, uint32_t c0[3],
                                   uint32_t cn[3]) {
    const uint32_t p[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int r = t.nlog[d + 1][a] - t.nlog[d][a];
        c0[a] = p[a] << r;
        cn[a] = 1u << r;
    }
}

// Parents of level d: min of mins, max of maxes for one channel.
__global__ void k_meta_reduce(TreeGeo t, int d, uint32_t *__restrict__ meta, int m, int c) {
    const uint64_t n = 1ull << (t.nlog[d][0] + t.nlog[d][1] + t.nlog[d][2]);
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t x = (uint32_t)(i & ((1u << t.nlog[d][0]) - 1));
    const uint32_t y = (uint32_t)((i >> t.nlog[d][0]) & ((1u << t.nlog[d][1]) - 1));
    const uint32_t z = (uint32_t)(i >> (t.nlog[d][0] + t.nlog[d][1]));
    uint32_t c0[3], cn[3];
    child_range(t, d, x, y, z, c0, cn);
    uint32_t mn = 0xFFFFu, mx = 0;
    for (uint32_t cz = 0; cz < cn[2]; ++cz)
        for (uint32_t cy = 0; cy < cn[1]; ++cy)
            for (uint32_t cx = 0; cx < cn[0]; ++cx) {
                const uint32_t v = meta[(uint64_t)node_index(t, d + 1, c0[0] + cx, c0[1] + cy, c0[2] + cz) * m + c];
                mn = min(mn, v & 0xFFFFu);
                mx = max(mx, v >> 16);
            }
    meta[((uint64_t)t.noff[d] + i) * m + c] = mn | (mx << 16);
}

static inline unsigned nblocks(uint64_t n) { return (unsigned)((n + 255) / 256); }

// Parents of level d for every channel in `chans` (bit c = channel c).
__global__ void k_meta_reduce_chans(TreeGeo t, int d, uint32_t *__restrict__ meta, int m, uint32_t chans) {
    const uint64_t n = 1ull << (t.nlog[d][0] + t.nlog[d][1] + t.nlog[d][2]);
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t x = (uint32_t)(i & ((1u << t.nlog[d][0]) - 1));
    const uint32_t y = (uint32_t)((i >> t.nlog[d][0]) & ((1u << t.nlog[d][1]) - 1));
    const uint32_t z = (uint32_t)(i >> (t.nlog[d][0] + t.nlog[d][1]));
    uint32_t c0[3], cn[3];
    child_range(t, d, x, y, z, c0, cn);
    for (int c = 0; c < m; ++c) {
        if (!((chans >> c) & 1u)) continue;
        uint32_t mn = 0xFFFFu, mx = 0;
        for (uint32_t cz = 0; cz < cn[2]; ++cz)
            for (uint32_t cy = 0; cy < cn[1]; ++cy)
                for (uint32_t cx = 0; cx < cn[0]; ++cx) {
                    const uint32_t v =
                        meta[(uint64_t)node_index(t, d + 1, c0[0] + cx, c0[1] + cy, c0[2] + cz) * m + c];
                    mn = min(mn, v & 0xFFFFu);
                    mx = max(mx, v >> 16);
                }
        meta[((uint64_t)t.noff[d] + i) * m + c] = mn | (mx << 16);
    }
}

// Work item of the metadata-from-bricks pass: the leaves inside one
// resident brick (leaf grid coordinates, clipped to the grid).
struct MetaItem {
    uint32_t c, l, slot, b[3], x0, y0, z0, nx, ny, nz, start;  // start = prefix of leaf counts
};

// One wave per leaf: [min, max] over the voxels of the brick's level that
// overlap the leaf box dilated by one voxel of that level, clamped to the
// level's grid (at level 0: the L0 voxels within one voxel of the leaf).
// The dilated box stays inside the slot: the leaf lies inside the brick and
// the slot holds a one-voxel halo.  A box that misses the grid gives [0, 0].
__global__ __launch_bounds__(256) void k_meta_from_bricks(VolGeo g, TreeGeo t, const MetaItem *__restrict__ items,
                                                          uint32_t n_items, uint32_t w0, uint32_t n_work,
                                                          const uint8_t *__restrict__ slots,
                                                          uint32_t *__restrict__ meta,
                                                          uint8_t *__restrict__ level) {
    const uint32_t w = w0 + blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= n_work) return;  // whole waves leave together
    uint32_t lo = 0, hi = n_items - 1;
    while (lo < hi) {  // last item with start <= w
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (items[mid].start <= w) lo = mid;
        else hi = mid - 1;
    }
    const MetaItem it = items[lo];
    const uint32_t r = w - it.start;
    const uint32_t leaf[3] = {it.x0 + r % it.nx, it.y0 + (r / it.nx) % it.ny, it.z0 + r / (it.nx * it.ny)};
    const int l = (int)it.l;
    // metadata from finer data stay (the whole wave leaves together)
    const uint64_t li = ((((uint64_t)leaf[2] << t.nlog[t.depth][1]) + leaf[1]) << t.nlog[t.depth][0]) + leaf[0];
    uint8_t *lev = level + li * (uint64_t)g.m + it.c;
    if (*lev < (uint8_t)l) return;
    int vlo[3], vn[3];
    bool empty = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t x0 = (int64_t)leaf[a] << t.leaf_log[a];
        const int64_t x1 = x0 + (1ll << t.leaf_log[a]);
        const int sh = g.lshift[l][a];
        const int64_t a0 = (x0 >> sh) > 0 ? (x0 >> sh) - 1 : 0;
        const int64_t e = ((x1 - 1) >> sh) + 1, top = (int64_t)g.ldims[l][a] - 1;
        const int64_t a1 = e < top ? e : top;
        if (a0 > a1) empty = true;
        // slot coordinate of level voxel v: v - b * B + 1
        vlo[a] = (int)(a0 - ((int64_t)it.b[a] << g.Blog) + 1);
        vn[a] = (int)(a1 - a0 + 1);
    }
    uint32_t mn = 0xFFFFu, mx = 0;
    if (!empty) {
        const uint8_t *base = slots + (size_t)it.slot * g.slot_stride;
        const uint32_t E = (uint32_t)g.E;
        const int n = vn[0] * vn[1] * vn[2];
        for (int i = lane; i < n; i += 64) {
            const int x = vlo[0] + i % vn[0], y = vlo[1] + (i / vn[0]) % vn[1], z = vlo[2] + i / (vn[0] * vn[1]);
            const size_t o = ((size_t)z * E + (size_t)y) * E + (size_t)x;
            const uint32_t v = g.bpv == 1 ? (uint32_t)base[o] : (uint32_t)((const uint16_t *)base)[o];
            mn = min(mn, v);
            mx = max(mx, v);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            mn = min(mn, (uint32_t)__shfl_xor((int)mn, off));
            mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
        }
    } else {
        mn = 0;
    }
    if (lane == 0) {
        meta[(uint64_t)node_index(t, t.depth, leaf[0], leaf[1], leaf[2]) * g.m + it.c] = mn | (mx << 16);
        *lev = (uint8_t)l;
    }
}

ro_status octree_set_meta(ro_octree *tr, uint32_t c, const uint16_t *leaf_mm, hipStream_t s) {
    const TreeGeo &t = tr->t;
    const VolGeo &g = tr->cache->vol->g;
    const int m = g.m;
    const uint32_t unknown_max = g.bpv == 1 ? 255u : 65535u;
    hipLaunchKernelGGL(k_meta_leaf, dim3(nblocks(t.n_leaves)), dim3(256), 0, s, leaf_mm, tr->b.node_meta,
                       tr->b.leaf_level, t.n_leaves, t.noff[t.depth], m, (int)c, unknown_max);
    RO_HIP(hipGetLastError());
    for (int d = t.depth - 1; d >= 0; --d) {
        const uint64_t n = 1ull << (t.nlog[d][0] + t.nlog[d][1] + t.nlog[d][2]);
        hipLaunchKernelGGL(k_meta_reduce, dim3(nblocks(n)), dim3(256), 0, s, t, d, tr->b.node_meta, m, (int)c);
        RO_HIP(hipGetLastError());
    }
    return RO_OK;
}

// Residency mask of channel c at a leaf: bit l is set iff the level-l brick
// containing the leaf exists and is resident (each leaf lies in exactly one
// brick per level, so partial and full mapping coincide at leaves).
__device__ inline uint16_t leaf_mask(const VolGeo &g, const TreeGeo &t, const uint32_t *__restrict__ pt, int c,
                                     uint32_t lx, uint32_t ly, uint32_t lz) {
    uint16_t m = 0;
    const uint32_t x = lx << t.leaf_log[0], y = ly << t.leaf_log[1], z = lz << t.leaf_log[2];
    for (int l = 0; l < g.L; ++l) {
        const uint32_t bx = x >> (g.Blog + g.lshift[l][0]);
        const uint32_t by = y >> (g.Blog + g.lshift[l][1]);
        const uint32_t bz = z >> (g.Blog + g.lshift[l][2]);
        if (bx >= (uint32_t)g.nb[l][0] || by >= (uint32_t)g.nb[l][1] || bz >= (uint32_t)g.nb[l][2]) continue;
        if (pt[dense_index(g, c, l, bx, by, bz)] != kInvalid) m |= (uint16_t)(1u << l);
    }
    return m;
}

__device__ inline uint32_t parent_of(const TreeGeo &t, int d, uint32_t x, uint32_t y, uint32_t z) {
    return node_index(t, d - 1, x >> (t.nlog[d][0] - t.nlog[d - 1][0]), y >> (t.nlog[d][1] - t.nlog[d - 1][1]),
                      z >> (t.nlog[d][2] - t.nlog[d - 1][2]));
}

// Work item: the leaves overlapping one inserted or evicted brick.
struct LeafItem {
    uint32_t c, x0, y0, z0, nx, ny, nz, start;  // start = prefix of leaf counts
};

__global__ void k_res_leaf(VolGeo g, TreeGeo t, const LeafItem *__restrict__ items, uint32_t n_items,
                           uint32_t n_work, const uint32_t *__restrict__ pt, uint16_t *__restrict__ mask,
                           uint8_t *__restrict__ flags) {
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_work) return;
    uint32_t lo = 0, hi = n_items - 1;
    while (lo < hi) {  // last item with start <= w
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (items[mid].start <= w) lo = mid;
        else hi = mid - 1;
    }
    const LeafItem it = items[lo];
    const uint32_t r = w - it.start;
    const uint32_t x = it.x0 + r % it.nx, y = it.y0 + (r / it.nx) % it.ny, z = it.z0 + r / (it.nx * it.ny);
    const uint16_t nm = leaf_mask(g, t, pt, (int)it.c, x, y, z);
    const uint32_t node = node_index(t, t.depth, x, y, z);
    uint16_t *p = mask + (uint64_t)node * g.m + it.c;
    if (*p != nm) {
        *p = nm;
        if (t.depth > 0) flags[parent_of(t, t.depth, x, y, z)] = 1;
    }
}

// One level of the upward propagation: flagged nodes get the OR of their
// children per channel; a change flags the parent.
__global__ void k_res_prop(TreeGeo t, int d, int m, uint16_t *__restrict__ mask, uint8_t *__restrict__ flags,
                           int all) {
    const uint64_t n = 1ull << (t.nlog[d][0] + t.nlog[d][1] + t.nlog[d][2]);
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t node = t.noff[d] + (uint32_t)i;
    if (!all) {
        if (!flags[node]) return;
        flags[node] = 0;
    }
    const uint32_t x = (uint32_t)(i & ((1u << t.nlog[d][0]) - 1));
    const uint32_t y = (uint32_t)((i >> t.nlog[d][0]) & ((1u << t.nlog[d][1]) - 1));
    const uint32_t z = (uint32_t)(i >> (t.nlog[d][0] + t.nlog[d][1]));
    uint32_t c0[3], cn[3];
    child_range(t, d, x, y, z, c0, cn);
    bool changed = false;
    for (int c = 0; c < m; ++c) {
        uint16_t o = 0;
        for (uint32_t cz = 0; cz < cn[2]; ++cz)
            for (uint32_t cy = 0; cy < cn[1]; ++cy)
                for (uint32_t cx = 0; cx < cn[0]; ++cx)
                    o |= mask[(uint64_t)node_index(t, d + 1, c0[0] + cx, c0[1] + cy, c0[2] + cz) * m + c];
        uint16_t *p = mask + (uint64_t)node * m + c;
        if (*p != o) {
            *p = o;
            changed = true;
        }
    }
    if (changed && d > 0 && !all) flags[parent_of(t, d, x, y, z)] = 1;
}

__global__ void k_res_leaf_all(VolGeo g, TreeGeo t, const uint32_t *__restrict__ pt, uint16_t *__restrict__ mask) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= t.n_leaves) return;
    const int D = t.depth;
    const uint32_t x = (uint32_t)(i & ((1u << t.nlog[D][0]) - 1));
    const uint32_t y = (uint32_t)((i >> t.nlog[D][0]) & ((1u << t.nlog[D][1]) - 1));
    const uint32_t z = (uint32_t)(i >> (t.nlog[D][0] + t.nlog[D][1]));
    const uint32_t node = t.noff[D] + (uint32_t)i;
    for (int c = 0; c < g.m; ++c) mask[(uint64_t)node * g.m + c] = leaf_mask(g, t, pt, c, x, y, z);
}

ro_status octree_update(ro_octree *tr, const std::vector<uint32_t> &dirty, hipStream_t s) {
    if (dirty.empty()) return RO_OK;
    const VolGeo &g = tr->cache->vol->g;
    const TreeGeo &t = tr->t;
    const int D = t.depth;
    const size_t cap = (tr->scratch_bytes - 256) / sizeof(LeafItem);
    std::vector<LeafItem> items;
    items.reserve(std::min(cap, dirty.size()));
    uint64_t work = 0;
    auto launch = [&]() -> ro_status {
        if (items.empty()) return RO_OK;
        RO_HIP(hipMemcpyAsync(tr->b.scratch, items.data(), items.size() * sizeof(LeafItem), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_res_leaf, dim3(nblocks(work)), dim3(256), 0, s, g, t, (const LeafItem *)tr->b.scratch,
                           (uint32_t)items.size(), (uint32_t)work, tr->cache->b.page_table, tr->b.node_mask,
                           tr->b.node_flags);
        RO_HIP(hipGetLastError());
        // the host buffer must outlive the copy: wait before reuse
        RO_HIP(hipStreamSynchronize(s));
        items.clear();
        work = 0;
        return RO_OK;
    };
    for (uint32_t dn : dirty) {
        const uint32_t c = dn / g.per_channel;
        const uint32_t r = dn - c * g.per_channel;
        int l = 0;
        while (l + 1 < g.L && g.loff[l + 1] <= r) ++l;
        const uint32_t lin = r - g.loff[l];
        const uint32_t b[3] = {lin % (uint32_t)g.nb[l][0], (lin / (uint32_t)g.nb[l][0]) % (uint32_t)g.nb[l][1],
                               lin / ((uint32_t)g.nb[l][0] * (uint32_t)g.nb[l][1])};
        LeafItem it;
        it.c = c;
        uint32_t lo[3], n[3];
        for (int a = 0; a < 3; ++a) {
            const int sh = g.Blog + g.lshift[l][a] - t.leaf_log[a];  // >= 0: leaf divides B
            const uint64_t nl = 1ull << t.nlog[D][a];
            const uint64_t l0 = (uint64_t)b[a] << sh, l1 = std::min<uint64_t>(((uint64_t)b[a] + 1) << sh, nl);
            lo[a] = (uint32_t)l0;
            n[a] = l1 > l0 ? (uint32_t)(l1 - l0) : 0;
        }
        const uint64_t cnt = (uint64_t)n[0] * n[1] * n[2];
        if (cnt == 0) continue;
        if (items.size() == cap || work + cnt > 0x7FFFFFFFull) {
            ro_status st = launch();
            if (st) return st;
        }
        it.x0 = lo[0];
        it.y0 = lo[1];
        it.z0 = lo[2];
        it.nx = n[0];
        it.ny = n[1];
        it.nz = n[2];
        it.start = (uint32_t)work;
        items.push_back(it);
        work += cnt;
    }
    ro_status st = launch();
    if (st) return st;
    const int m = g.m;
    for (int d = D - 1; d >= 0; --d) {
        const uint64_t n = 1ull << (t.nlog[d][0] + t.nlog[d][1] + t.nlog[d][2]);
        hipLaunchKernelGGL(k_res_prop, dim3(nblocks(n)), dim3(256), 0, s, t, d, m, tr->b.node_mask, tr->b.node_flags, 0);
        RO_HIP(hipGetLastError());
    }
    return RO_OK;
}

ro_status octree_rebuild(ro_octree *tr, hipStream_t s) {
    const VolGeo &g = tr->cache->vol->g;
    const TreeGeo &t = tr->t;
    hipLaunchKernelGGL(k_res_leaf_all, dim3(nblocks(t.n_leaves)), dim3(256), 0, s, g, t, tr->cache->b.page_table,
                       tr->b.node_mask);
    RO_HIP(hipGetLastError());
    for (int d = t.depth - 1; d >= 0; --d) {
        const uint64_t n = 1ull << (t.nlog[d][0] + t.nlog[d][1] + t.nlog[d][2]);
        hipLaunchKernelGGL(k_res_prop, dim3(nblocks(n)), dim3(256), 0, s, t, d, g.m, tr->b.node_mask,
                           tr->b.node_flags, 1);
        RO_HIP(hipGetLastError());
    }
    return launch_fill_u8(tr->b.node_flags, t.n_nodes, 0, s);
}


// Leaf metadata of the leaves inside resident bricks, computed from the
// bricks' voxels (Sec. 5.3, metadata on the client when the server has
// none).  `dense` holds validated resident dense indices sorted by level,
// coarsest first, so that where bricks of several levels cover one leaf the
// finest level's pass runs last and its values stay; a leaf whose metadata
// came from finer data (its level entry) keeps them.
ro_status octree_meta_from_bricks(ro_octree *tr, const std::vector<uint32_t> &dense, hipStream_t s) {
    if (dense.empty()) return RO_OK;
    const VolGeo &g = tr->cache->vol->g;
    const TreeGeo &t = tr->t;
    const int D = t.depth;
    const size_t cap = (tr->scratch_bytes - 256) / sizeof(MetaItem);
    std::vector<MetaItem> items;
    uint64_t work = 0;
    uint32_t chans = 0;
    int cur_level = -1;
    auto launch = [&]() -> ro_status {
        if (items.empty()) return RO_OK;
        RO_HIP(hipMemcpyAsync(tr->b.scratch, items.data(), items.size() * sizeof(MetaItem), hipMemcpyHostToDevice, s));
        // at most 2^22 blocks of four waves per launch
        constexpr uint64_t kChunk = 1ull << 24;
        for (uint64_t w0 = 0; w0 < work; w0 += kChunk) {
            const uint64_t nw = std::min(kChunk, work - w0);
            hipLaunchKernelGGL(k_meta_from_bricks, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, s, g, t,
                               (const MetaItem *)tr->b.scratch, (uint32_t)items.size(), (uint32_t)w0,
                               (uint32_t)work, (const uint8_t *)tr->cache->b.slots, tr->b.node_meta,
                               tr->b.leaf_level);
            RO_HIP(hipGetLastError());
        }
        // the host buffer must outlive the copy: wait before reuse
        RO_HIP(hipStreamSynchronize(s));
        items.clear();
        work = 0;
        return RO_OK;
    };
    for (uint32_t dn : dense) {
        const uint32_t c = dn / g.per_channel;
        const uint32_t r = dn - c * g.per_channel;
        int l = 0;
        while (l + 1 < g.L && g.loff[l + 1] <= r) ++l;
        // one level per launch: the launches of coarser levels finish first
        if (l != cur_level) {
            ro_status st = launch();
            if (st) return st;
            cur_level = l;
        }
        const uint32_t lin = r - g.loff[l];
        const uint32_t b[3] = {lin % (uint32_t)g.nb[l][0], (lin / (uint32_t)g.nb[l][0]) % (uint32_t)g.nb[l][1],
                               lin / ((uint32_t)g.nb[l][0] * (uint32_t)g.nb[l][1])};
        MetaItem it;
        it.c = c;
        it.l = (uint32_t)l;
        it.slot = tr->cache->pt_host[dn];
        uint32_t lo[3], n[3];
        for (int a = 0; a < 3; ++a) {
            it.b[a] = b[a];
            const int sh = g.Blog + g.lshift[l][a] - t.leaf_log[a];  // >= 0: leaf divides B
            const uint64_t nl = 1ull << t.nlog[D][a];
            const uint64_t l0 = (uint64_t)b[a] << sh, l1 = std::min<uint64_t>(((uint64_t)b[a] + 1) << sh, nl);
            lo[a] = (uint32_t)std::min<uint64_t>(l0, nl);
            n[a] = l1 > l0 ? (uint32_t)(l1 - l0) : 0;
        }
        const uint64_t cnt = (uint64_t)n[0] * n[1] * n[2];
        if (cnt == 0) continue;
        if (items.size() == cap || work + cnt > 0x7FFFFFFFull) {
            ro_status st = launch();
            if (st) return st;
        }
        it.x0 = lo[0];
        it.y0 = lo[1];
        it.z0 = lo[2];
        it.nx = n[0];
        it.ny = n[1];
        it.nz = n[2];
        it.start = (uint32_t)work;
        items.push_back(it);
        work += cnt;
        chans |= 1u << c;
    }
    ro_status st = launch();
    if (st) return st;
    for (int d = D - 1; d >= 0; --d) {
        const uint64_t n = 1ull << (t.nlog[d][0] + t.nlog[d][1] + t.nlog[d][2]);
        hipLaunchKernelGGL(k_meta_reduce_chans, dim3(nblocks(n)), dim3(256), 0, s, t, d, tr->b.node_meta, g.m, chans);
        RO_HIP(hipGetLastError());
    }
    return RO_OK;
}

}  // namespace ro
