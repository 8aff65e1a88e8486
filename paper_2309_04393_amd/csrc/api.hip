// Host side of the C ABI: validation, geometry, handle bookkeeping.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "common.h"

namespace ro {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

ro_status hip_fail(hipError_t e, const char *what) {
    set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return RO_E_DEVICE;
}

static bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
static int ilog2(int64_t x) {
    int r = 0;
    while ((1ll << r) < x) ++r;
    return r;
}
static bool aligned(const void *p) { return ((uintptr_t)p & 255u) == 0; }

// Level schedule: halve axis a from level l-1 to l iff its spacing at l-1 is
// below twice the smallest spacing at l-1; halved dims are ceil(n/2).
static void derive_levels(const ro_volume_desc &d, VolGeo &g) {
    double s[3] = {d.spacing[0], d.spacing[1], d.spacing[2]};
    for (int a = 0; a < 3; ++a) {
        g.ldims[0][a] = d.dims[a];
        g.lshift[0][a] = 0;
    }
    for (int l = 1; l < d.n_levels; ++l) {
        double mn = std::min(s[0], std::min(s[1], s[2]));
        bool h[3];
        for (int a = 0; a < 3; ++a) h[a] = s[a] < 2.0 * mn;
        for (int a = 0; a < 3; ++a) {
            g.ldims[l][a] = h[a] ? (g.ldims[l - 1][a] + 1) / 2 : g.ldims[l - 1][a];
            g.lshift[l][a] = g.lshift[l - 1][a] + (h[a] ? 1 : 0);
            if (h[a]) s[a] *= 2.0;
        }
    }
}

}  // namespace ro

using namespace ro;

extern "C" const char *ro_last_error(void) { return g_err; }

extern "C" ro_status ro_volume_create(const ro_volume_desc *d, ro_volume **out) {
    RO_CHECK(d && out, RO_E_ARG, "null argument");
    for (int a = 0; a < 3; ++a) {
        RO_CHECK(d->dims[a] >= 1, RO_E_ARG, "dims[%d] = %d must be >= 1", a, d->dims[a]);
        RO_CHECK(d->spacing[a] > 0.0, RO_E_ARG, "spacing[%d] must be > 0", a);
    }
    RO_CHECK(d->n_channels >= 1 && d->n_channels <= kMaxC, RO_E_ARG, "n_channels %d not in 1..%d",
             d->n_channels, kMaxC);
    RO_CHECK(d->bytes_per_voxel == 1 || d->bytes_per_voxel == 2, RO_E_ARG,
             "bytes_per_voxel must be 1 or 2");
    RO_CHECK(is_pow2(d->brick) && d->brick >= 4 && d->brick <= 128, RO_E_ARG,
             "brick %d must be a power of two in [4, 128]", d->brick);
    RO_CHECK(d->n_levels >= 1 && d->n_levels <= kMaxL, RO_E_ARG, "n_levels %d not in 1..%d",
             d->n_levels, kMaxL);
    RO_CHECK(d->n_channels * d->n_levels <= 256, RO_E_CAPACITY,
             "channels x levels = %d exceeds the 8-bit page-table ID", d->n_channels * d->n_levels);
    VolGeo g;
    memset(&g, 0, sizeof(g));
    derive_levels(*d, g);
    uint64_t per = 0;
    for (int l = 0; l < d->n_levels; ++l) {
        for (int a = 0; a < 3; ++a) {
            g.nb[l][a] = (g.ldims[l][a] + d->brick - 1) / d->brick;
            RO_CHECK(g.nb[l][a] <= 256, RO_E_CAPACITY,
                     "level %d has %d bricks on axis %d; brick IDs hold 256", l, g.nb[l][a], a);
        }
        g.loff[l] = (uint32_t)per;
        per += (uint64_t)g.nb[l][0] * g.nb[l][1] * g.nb[l][2];
    }
    g.loff[d->n_levels] = (uint32_t)per;
    RO_CHECK(per * d->n_channels < 0xFFFFFFFFull, RO_E_CAPACITY, "too many bricks");
    for (int a = 0; a < 3; ++a) {
        g.dims[a] = d->dims[a];
        g.spacing[a] = d->spacing[a];
    }
    g.m = d->n_channels;
    g.bpv = d->bytes_per_voxel;
    g.B = d->brick;
    g.Blog = ilog2(d->brick);
    g.E = d->brick + 2;
    g.L = d->n_levels;
    g.per_channel = (uint32_t)per;
    g.total = per * (uint64_t)d->n_channels;
    uint64_t sb = (uint64_t)g.E * g.E * g.E * g.bpv;
    g.slot_stride = (uint32_t)((sb + 255) / 256 * 256);
    ro_volume *v = new (std::nothrow) ro_volume;
    RO_CHECK(v, RO_E_NOMEM, "out of host memory");
    v->desc = *d;
    v->g = g;
    *out = v;
    return RO_OK;
}

extern "C" void ro_volume_destroy(ro_volume *v) { delete v; }

extern "C" ro_status ro_volume_levels(const ro_volume *v, int32_t *dims_out, int32_t *factor_out,
                                      int32_t *bricks_out) {
    RO_CHECK(v, RO_E_ARG, "null volume");
    for (int l = 0; l < v->g.L; ++l)
        for (int a = 0; a < 3; ++a) {
            if (dims_out) dims_out[3 * l + a] = v->g.ldims[l][a];
            if (factor_out) factor_out[3 * l + a] = 1 << v->g.lshift[l][a];
            if (bricks_out) bricks_out[3 * l + a] = v->g.nb[l][a];
        }
    return RO_OK;
}

extern "C" ro_status ro_volume_brick_count(const ro_volume *v, uint64_t *count) {
    RO_CHECK(v && count, RO_E_ARG, "null argument");
    *count = v->g.total;
    return RO_OK;
}

extern "C" ro_status ro_brick_id_encode(const ro_volume *v, uint32_t c, uint32_t l,
                                        const uint32_t b[3], uint32_t *id) {
    RO_CHECK(v && b && id, RO_E_ARG, "null argument");
    RO_CHECK(c < (uint32_t)v->g.m && l < (uint32_t)v->g.L, RO_E_ARG, "channel or level out of range");
    for (int a = 0; a < 3; ++a)
        RO_CHECK(b[a] < (uint32_t)v->g.nb[l][a], RO_E_ARG, "brick coordinate out of range");
    *id = ((c * (uint32_t)v->g.L + l) << 24) | (b[2] << 16) | (b[1] << 8) | b[0];
    return RO_OK;
}

// Brick ID -> (c, l, b) with range checks; returns false if out of range.
static bool decode_id(const VolGeo &g, uint32_t id, uint32_t *c, uint32_t *l, uint32_t b[3]) {
    uint32_t pt = id >> 24;
    *c = pt / (uint32_t)g.L;
    *l = pt % (uint32_t)g.L;
    b[0] = id & 255u;
    b[1] = (id >> 8) & 255u;
    b[2] = (id >> 16) & 255u;
    if (*c >= (uint32_t)g.m) return false;
    for (int a = 0; a < 3; ++a)
        if (b[a] >= (uint32_t)g.nb[*l][a]) return false;
    return true;
}

extern "C" ro_status ro_brick_id_decode(const ro_volume *v, uint32_t id, uint32_t *c, uint32_t *l,
                                        uint32_t b[3]) {
    RO_CHECK(v && c && l && b, RO_E_ARG, "null argument");
    uint32_t cc, ll, bb[3];
    RO_CHECK(decode_id(v->g, id, &cc, &ll, bb), RO_E_ARG, "brick ID 0x%08x out of range", id);
    *c = cc;
    *l = ll;
    b[0] = bb[0];
    b[1] = bb[1];
    b[2] = bb[2];
    return RO_OK;
}

// ------------------------------------------------------------------ cache

static CacheScratch cache_scratch_layout(const VolGeo &g, const ro_cache_desc &d) {
    CacheScratch s;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    s.keys = take(sizeof(uint64_t) * d.n_slots);
    s.hist = take(sizeof(uint32_t) * 256);
    s.sel = take(64);
    s.cand = take(sizeof(uint64_t) * d.max_batch);
    s.victims = take(sizeof(uint32_t) * d.max_batch);
    s.evicted = take(sizeof(uint32_t) * d.max_batch);
    s.uploads = take(sizeof(uint32_t) * d.max_batch);
    s.srcidx = take(sizeof(uint32_t) * d.max_batch);
    s.touch = take(sizeof(uint32_t) * d.max_batch);
    s.compact = take(compact_scratch_bytes(g.total, (uint32_t)g.total));
    size_t n_slots_or_total = std::max<uint64_t>(g.total, d.n_slots);
    s.outpairs = take(sizeof(uint32_t) * 2 * n_slots_or_total);
    s.total = o;
    return s;
}

static ro_status check_cache_desc(const ro_volume *v, const ro_cache_desc *d) {
    RO_CHECK(v && d, RO_E_ARG, "null argument");
    RO_CHECK(d->n_slots >= 1 && d->n_slots < 0x7FFFFFFFu, RO_E_ARG, "n_slots must be >= 1");
    RO_CHECK(d->max_batch >= 1 && d->max_batch <= 8192, RO_E_ARG, "max_batch not in 1..8192");
    return RO_OK;
}

extern "C" ro_status ro_cache_query(const ro_volume *v, const ro_cache_desc *d, ro_cache_sizes *o) {
    ro_status st = check_cache_desc(v, d);
    if (st) return st;
    RO_CHECK(o, RO_E_ARG, "null output");
    const VolGeo &g = v->g;
    o->slot_stride = g.slot_stride;
    o->slots = (size_t)g.slot_stride * d->n_slots;
    o->page_table = sizeof(uint32_t) * g.total;
    o->counters = sizeof(uint32_t) * g.total;
    o->slot_brick = sizeof(uint32_t) * d->n_slots;
    o->stamps = sizeof(uint32_t) * d->n_slots;
    o->seqs = sizeof(uint32_t) * d->n_slots;
    o->scratch = cache_scratch_layout(g, *d).total;
    return RO_OK;
}

extern "C" ro_status ro_cache_create(const ro_volume *v, const ro_cache_desc *d,
                                     const ro_cache_buffers *b, void *stream, ro_cache **out) {
    ro_status st = check_cache_desc(v, d);
    if (st) return st;
    RO_CHECK(b && out, RO_E_ARG, "null argument");
    RO_CHECK(b->slots && b->page_table && b->counters && b->slot_brick && b->stamps && b->seqs &&
                 b->scratch,
             RO_E_ARG, "null device buffer");
    RO_CHECK(aligned(b->slots) && aligned(b->page_table) && aligned(b->counters) &&
                 aligned(b->slot_brick) && aligned(b->stamps) && aligned(b->seqs) &&
                 aligned(b->scratch),
             RO_E_ARG, "device buffers must be 256-byte aligned");
    ro_cache *c = new (std::nothrow) ro_cache;
    RO_CHECK(c, RO_E_NOMEM, "out of host memory");
    try {
        c->pt_host.assign(v->g.total, kInvalid);
        c->slot_host.assign(d->n_slots, kInvalid);
        c->chmap.resize(v->g.m);
        for (int j = 0; j < v->g.m; ++j) c->chmap[j] = (uint32_t)j;
    } catch (...) {
        delete c;
        RO_CHECK(false, RO_E_NOMEM, "out of host memory");
    }
    c->vol = const_cast<ro_volume *>(v);
    c->desc = *d;
    c->b = *b;
    c->sc = cache_scratch_layout(v->g, *d);
    c->seq_next = 0;
    hipStream_t s = (hipStream_t)stream;
    ro_status r;
    if ((r = launch_fill_u32(b->page_table, v->g.total, kInvalid, s)) ||
        (r = launch_fill_u32(b->counters, v->g.total, 0, s)) ||
        (r = launch_fill_u32(b->slot_brick, d->n_slots, kInvalid, s)) ||
        (r = launch_fill_u32(b->stamps, d->n_slots, 0, s)) ||
        (r = launch_fill_u32(b->seqs, d->n_slots, 0, s))) {
        delete c;
        return r;
    }
    *out = c;
    return RO_OK;
}

extern "C" void ro_cache_destroy(ro_cache *c) { delete c; }

extern "C" ro_status ro_cache_evict_channel(ro_cache *c, uint32_t channel, void *stream) {
    RO_CHECK(c, RO_E_ARG, "null cache");
    RO_CHECK(channel < (uint32_t)c->vol->g.m, RO_E_ARG, "channel %u out of range", channel);
    return cache_evict_channel(c, channel, (hipStream_t)stream);
}

extern "C" ro_status ro_cache_page_table_host(const ro_cache *c, uint32_t *out, uint64_t count) {
    RO_CHECK(c && out, RO_E_ARG, "null argument");
    RO_CHECK(count == c->pt_host.size(), RO_E_ARG, "count must equal the brick count");
    memcpy(out, c->pt_host.data(), sizeof(uint32_t) * count);
    return RO_OK;
}

// Checkpoint blob: header, then the page-table mirror, slot mirror, dirty
// list and channel map.
struct StateHeader {
    uint64_t magic, total, slots, dirty;
    uint32_t seq_next, channels;
};
static const uint64_t kStateMagic = 0x32455441545352ull;  // "RSTATE2"

extern "C" ro_status ro_cache_state_size(const ro_cache *c, size_t *bytes) {
    RO_CHECK(c && bytes, RO_E_ARG, "null argument");
    *bytes = sizeof(StateHeader) + 4 * (c->pt_host.size() + c->slot_host.size() + c->dirty.size() + c->chmap.size());
    return RO_OK;
}

extern "C" ro_status ro_cache_set_channel_map(ro_cache *c, uint32_t cache_channel, uint32_t source_channel) {
    RO_CHECK(c, RO_E_ARG, "null cache");
    RO_CHECK(cache_channel < c->chmap.size(), RO_E_ARG, "cache channel %u out of range", cache_channel);
    c->chmap[cache_channel] = source_channel;
    return RO_OK;
}

extern "C" ro_status ro_cache_get_channel_map(const ro_cache *c, uint32_t *map) {
    RO_CHECK(c && map, RO_E_ARG, "null argument");
    memcpy(map, c->chmap.data(), 4 * c->chmap.size());
    return RO_OK;
}

extern "C" ro_status ro_cache_source_bricks(const ro_cache *c, uint32_t n, const uint32_t *ids, uint32_t *out) {
    RO_CHECK(c && (n == 0 || (ids && out)), RO_E_ARG, "null argument");
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t cc, ll, bb[3];
        RO_CHECK(decode_id(c->vol->g, ids[i], &cc, &ll, bb), RO_E_ARG, "brick ID 0x%08x out of range", ids[i]);
    }
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t cc, ll, bb[3];
        decode_id(c->vol->g, ids[i], &cc, &ll, bb);
        uint32_t *o = out + 5 * (size_t)i;
        o[0] = c->chmap[cc];
        o[1] = ll;
        o[2] = bb[0];
        o[3] = bb[1];
        o[4] = bb[2];
    }
    return RO_OK;
}

extern "C" ro_status ro_cache_save_state(const ro_cache *c, void *host, size_t cap) {
    size_t need = 0;
    ro_status st = ro_cache_state_size(c, &need);
    if (st) return st;
    RO_CHECK(host && cap >= need, RO_E_ARG, "buffer of %zu bytes needed", need);
    StateHeader hd = {kStateMagic, c->pt_host.size(), c->slot_host.size(), c->dirty.size(), c->seq_next,
                      (uint32_t)c->chmap.size()};
    uint8_t *p = (uint8_t *)host;
    memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    memcpy(p, c->pt_host.data(), 4 * c->pt_host.size());
    p += 4 * c->pt_host.size();
    memcpy(p, c->slot_host.data(), 4 * c->slot_host.size());
    p += 4 * c->slot_host.size();
    if (!c->dirty.empty()) memcpy(p, c->dirty.data(), 4 * c->dirty.size());
    p += 4 * c->dirty.size();
    memcpy(p, c->chmap.data(), 4 * c->chmap.size());
    return RO_OK;
}

extern "C" ro_status ro_cache_load_state(ro_cache *c, const void *host, size_t size) {
    RO_CHECK(c && host && size >= sizeof(StateHeader), RO_E_ARG, "bad state blob");
    StateHeader hd;
    memcpy(&hd, host, sizeof(hd));
    RO_CHECK(hd.magic == kStateMagic && hd.total == c->pt_host.size() && hd.slots == c->slot_host.size() &&
                 hd.channels == c->chmap.size() && size == sizeof(hd) + 4 * (hd.total + hd.slots + hd.dirty + hd.channels),
             RO_E_ARG, "state blob does not match this cache");
    const uint8_t *p = (const uint8_t *)host + sizeof(hd);
    try {
        std::vector<uint32_t> dirty(hd.dirty);
        if (hd.dirty) memcpy(dirty.data(), p + 4 * (hd.total + hd.slots), 4 * hd.dirty);
        c->dirty.swap(dirty);
    } catch (...) {
        RO_CHECK(false, RO_E_NOMEM, "out of host memory");
    }
    memcpy(c->pt_host.data(), p, 4 * hd.total);
    memcpy(c->slot_host.data(), p + 4 * hd.total, 4 * hd.slots);
    memcpy(c->chmap.data(), p + 4 * (hd.total + hd.slots + hd.dirty), 4 * (size_t)hd.channels);
    c->seq_next = hd.seq_next;
    return RO_OK;
}

extern "C" ro_status ro_stream_bricks(ro_cache *c, uint32_t frame, uint32_t n,
                                      const uint32_t *ids, const void *staged, uint8_t *flags,
                                      void *stream) {
    RO_CHECK(c, RO_E_ARG, "null cache");
    RO_CHECK(n <= c->desc.max_batch, RO_E_ARG, "n = %u exceeds max_batch %u", n, c->desc.max_batch);
    RO_CHECK(frame != kInvalid, RO_E_ARG, "frame 0xFFFFFFFF is reserved");
    if (n == 0) return RO_OK;
    RO_CHECK(ids && staged && flags, RO_E_ARG, "null argument");
    RO_CHECK(aligned(staged), RO_E_ARG, "staged bricks must be 256-byte aligned");
    const VolGeo &g = c->vol->g;
    std::vector<uint32_t> dn(n);
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t cc, ll, bb[3];
        RO_CHECK(decode_id(g, ids[i], &cc, &ll, bb), RO_E_ARG, "brick ID 0x%08x out of range",
                 ids[i]);
        dn[i] = dense_index(g, (int)cc, (int)ll, (int)bb[0], (int)bb[1], (int)bb[2]);
    }
    // Host bookkeeping: flags for resident / repeated IDs, upload list.
    std::vector<uint32_t> up, src, touch;
    std::vector<uint8_t> f(n, 0);
    std::vector<uint32_t> sorted_seen;
    sorted_seen.reserve(n);
    for (uint32_t i = 0; i < n; ++i) {
        auto it = std::lower_bound(sorted_seen.begin(), sorted_seen.end(), dn[i]);
        bool dup = it != sorted_seen.end() && *it == dn[i];
        if (!dup) sorted_seen.insert(it, dn[i]);
        if (dup) {
            f[i] = 2;
        } else if (c->pt_host[dn[i]] != kInvalid) {
            f[i] = 2;
            touch.push_back(c->pt_host[dn[i]]);
        } else {
            up.push_back(dn[i]);
            src.push_back(i);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    uint8_t *sc = (uint8_t *)c->b.scratch;
    if (!touch.empty())
        RO_HIP(hipMemcpyAsync(sc + c->sc.touch, touch.data(), 4 * touch.size(), hipMemcpyHostToDevice, s));
    if (!up.empty()) {
        RO_HIP(hipMemcpyAsync(sc + c->sc.uploads, up.data(), 4 * up.size(), hipMemcpyHostToDevice, s));
        RO_HIP(hipMemcpyAsync(sc + c->sc.srcidx, src.data(), 4 * src.size(), hipMemcpyHostToDevice, s));
    }
    uint32_t k_eff = 0;
    std::vector<uint32_t> victims(up.size() + 1), evicted(up.size() + 1);
    ro_status st = stream_bricks_device(c, frame, (uint32_t)up.size(), (uint32_t)touch.size(), staged,
                                        s, &k_eff, victims.data(), evicted.data());
    if (st) return st;
    // Mirror the device's decisions.
    for (uint32_t i = 0; i < (uint32_t)up.size(); ++i) {
        if (i < k_eff) {
            uint32_t slot = victims[i];
            uint32_t old = c->slot_host[slot];
            if (old != kInvalid) {
                c->pt_host[old] = kInvalid;
                c->dirty.push_back(old);
            }
            c->slot_host[slot] = up[i];
            c->pt_host[up[i]] = slot;
            c->dirty.push_back(up[i]);
            f[src[i]] = 1;
        } else {
            f[src[i]] = 0;
        }
    }
    c->seq_next += k_eff;
    memcpy(flags, f.data(), n);
    return RO_OK;
}

extern "C" ro_status ro_read_requests(ro_cache *c, uint32_t cap, uint32_t *ids, uint32_t *counts,
                                      uint32_t *n_unique, uint64_t *total, void *stream) {
    RO_CHECK(c && n_unique && total, RO_E_ARG, "null argument");
    RO_CHECK(cap == 0 || (ids && counts), RO_E_ARG, "null output arrays");
    return read_requests_device(c, cap, ids, counts, n_unique, total, (hipStream_t)stream);
}

extern "C" ro_status ro_read_requests_noalloc(ro_cache *c, uint32_t cap, uint32_t *ids, uint32_t *counts,
                                              uint32_t *n_unique, uint64_t *total, void *stream) {
    RO_CHECK(c && n_unique && total, RO_E_ARG, "null argument");
    RO_CHECK(cap == 0 || (ids && counts), RO_E_ARG, "null output arrays");
    return read_requests_noalloc_device(c, cap, ids, counts, n_unique, total, (hipStream_t)stream);
}

extern "C" ro_status ro_read_usage(ro_cache *c, uint32_t frame, uint32_t cap, uint32_t *slots,
                                   uint32_t *n_out, void *stream) {
    RO_CHECK(c && n_out, RO_E_ARG, "null argument");
    RO_CHECK(cap == 0 || slots, RO_E_ARG, "null output array");
    return read_usage_device(c, frame, cap, slots, n_out, (hipStream_t)stream);
}

// ----------------------------------------------------------------- octree

static ro_status tree_geometry(const ro_volume *v, const ro_octree_desc *d, TreeGeo &t) {
    RO_CHECK(v && d, RO_E_ARG, "null argument");
    RO_CHECK(d->depth >= 0 && d->depth <= kMaxD, RO_E_ARG, "depth %d not in 0..%d", d->depth, kMaxD);
    memset(&t, 0, sizeof(t));
    t.depth = d->depth;
    int s[3];
    for (int a = 0; a < 3; ++a) {
        RO_CHECK(is_pow2(d->leaf[a]) && d->leaf[a] <= v->g.B, RO_E_ARG,
                 "leaf[%d] = %d must be a power of two dividing the brick edge", a, d->leaf[a]);
        t.leaf_log[a] = ilog2(d->leaf[a]);
        int64_t nl = ((int64_t)v->g.dims[a] + d->leaf[a] - 1) / d->leaf[a];
        s[a] = ilog2(nl);
        RO_CHECK(s[a] <= d->depth, RO_E_ARG, "depth %d too small: axis %d needs %d splits", d->depth,
                 a, s[a]);
    }
    uint64_t o = 0;
    for (int l = 0; l <= d->depth; ++l) {
        for (int a = 0; a < 3; ++a) {
            int k = std::min(d->depth - l, s[a]);
            t.nshift[l][a] = t.leaf_log[a] + k;
            t.nlog[l][a] = s[a] - k;
        }
        t.noff[l] = (uint32_t)o;
        o += 1ull << (t.nlog[l][0] + t.nlog[l][1] + t.nlog[l][2]);
        RO_CHECK(o < 0xFFFFFFFFull, RO_E_CAPACITY, "too many tree nodes");
    }
    t.noff[d->depth + 1] = (uint32_t)o;
    t.n_nodes = o;
    t.n_leaves = 1ull << (t.nlog[d->depth][0] + t.nlog[d->depth][1] + t.nlog[d->depth][2]);
    RO_CHECK(d->start_level >= 0 && d->start_level <= d->depth, RO_E_ARG,
             "start_level %d not in 0..depth", d->start_level);
    return RO_OK;
}

extern "C" ro_status ro_octree_query(const ro_volume *v, const ro_octree_desc *d,
                                     ro_octree_sizes *o) {
    TreeGeo t;
    ro_status st = tree_geometry(v, d, t);
    if (st) return st;
    RO_CHECK(o, RO_E_ARG, "null output");
    o->n_nodes = t.n_nodes;
    o->n_leaves = t.n_leaves;
    for (int a = 0; a < 3; ++a) o->leaf_grid[a] = 1 << t.nlog[d->depth][a];
    o->node_meta = sizeof(uint32_t) * t.n_nodes * v->g.m;
    o->node_mask = sizeof(uint16_t) * t.n_nodes * v->g.m;
    o->node_flags = t.n_nodes;
    o->scratch = 16 * 65536 + 256;  // leaf-update work items
    o->leaf_level = t.n_leaves * v->g.m;
    return RO_OK;
}

extern "C" ro_status ro_octree_create(ro_cache *c, const ro_octree_desc *d,
                                      const ro_octree_buffers *b, void *stream, ro_octree **out) {
    RO_CHECK(c && b && out, RO_E_ARG, "null argument");
    TreeGeo t;
    ro_status st = tree_geometry(c->vol, d, t);
    if (st) return st;
    RO_CHECK(b->node_meta && b->node_mask && b->node_flags && b->scratch && b->leaf_level, RO_E_ARG,
             "null device buffer");
    RO_CHECK(aligned(b->node_meta) && aligned(b->node_mask) && aligned(b->node_flags) &&
                 aligned(b->scratch) && aligned(b->leaf_level),
             RO_E_ARG, "device buffers must be 256-byte aligned");
    ro_octree *o = new (std::nothrow) ro_octree;
    RO_CHECK(o, RO_E_NOMEM, "out of host memory");
    o->cache = c;
    o->desc = *d;
    o->b = *b;
    o->t = t;
    o->scratch_bytes = 16 * 65536 + 256;
    hipStream_t s = (hipStream_t)stream;
    uint64_t nm = t.n_nodes * (uint64_t)c->vol->g.m;
    ro_status r;
    if ((r = launch_fill_u32(b->node_meta, nm, 0, s)) || (r = launch_fill_u16(b->node_mask, nm, 0, s)) ||
        (r = launch_fill_u8(b->node_flags, t.n_nodes, 0, s)) ||
        (r = launch_fill_u8(b->leaf_level, t.n_leaves * (uint64_t)c->vol->g.m, kLevelUnknown, s))) {
        delete o;
        return r;
    }
    *out = o;
    return RO_OK;
}

// ------------------------------------------------------------- checkpoint

// Snapshot blob: header, the cache's host state (as ro_cache_save_state
// writes it), then the device arrays in a fixed order.
struct SnapHeader {
    uint64_t magic;
    uint64_t total, slots, nodes, slot_stride;
    uint32_t m, flags;
    uint64_t host_bytes;
};
static const uint64_t kSnapMagic = 0x3150414e53524full;  // "ORSNAP1"

struct SnapPart {
    void *dev;
    size_t bytes;
};

static int snap_parts(const ro_octree *t, uint32_t flags, SnapPart *p) {
    const ro_cache *c = t->cache;
    const uint64_t total = c->vol->g.total, S = c->desc.n_slots, nn = t->t.n_nodes, m = (uint64_t)c->vol->g.m;
    int n = 0;
    p[n++] = {c->b.page_table, 4 * total};
    p[n++] = {c->b.counters, 4 * total};
    p[n++] = {c->b.slot_brick, 4 * S};
    p[n++] = {c->b.stamps, 4 * S};
    p[n++] = {c->b.seqs, 4 * S};
    p[n++] = {t->b.node_meta, 4 * nn * m};
    p[n++] = {t->b.node_mask, 2 * nn * m};
    p[n++] = {t->b.node_flags, nn};
    p[n++] = {t->b.leaf_level, (size_t)t->t.n_leaves * m};
    if (flags & RO_SNAPSHOT_SLOTS) p[n++] = {c->b.slots, (size_t)c->vol->g.slot_stride * S};
    return n;
}

extern "C" ro_status ro_snapshot_size(const ro_octree *t, uint32_t flags, size_t *bytes) {
    RO_CHECK(t && bytes, RO_E_ARG, "null argument");
    RO_CHECK(!(flags & ~RO_SNAPSHOT_SLOTS), RO_E_ARG, "unknown snapshot flags 0x%x", flags);
    size_t host = 0;
    ro_status st = ro_cache_state_size(t->cache, &host);
    if (st) return st;
    SnapPart p[10];
    const int n = snap_parts(t, flags, p);
    size_t b = sizeof(SnapHeader) + host;
    for (int i = 0; i < n; ++i) b += p[i].bytes;
    *bytes = b;
    return RO_OK;
}

extern "C" ro_status ro_snapshot(const ro_octree *t, uint32_t flags, void *host_blob, size_t cap, size_t *used,
                                 void *stream) {
    size_t need = 0;
    ro_status st = ro_snapshot_size(t, flags, &need);
    if (st) return st;
    RO_CHECK(host_blob && used, RO_E_ARG, "null argument");
    RO_CHECK(cap >= need, RO_E_CAPACITY, "snapshot needs %zu bytes, the buffer holds %zu", need, cap);
    const ro_cache *c = t->cache;
    SnapHeader hd;
    memset(&hd, 0, sizeof(hd));
    hd.magic = kSnapMagic;
    hd.total = c->vol->g.total;
    hd.slots = c->desc.n_slots;
    hd.nodes = t->t.n_nodes;
    hd.slot_stride = c->vol->g.slot_stride;
    hd.m = (uint32_t)c->vol->g.m;
    hd.flags = flags;
    st = ro_cache_state_size(c, &hd.host_bytes);
    if (st) return st;
    uint8_t *o = (uint8_t *)host_blob;
    memcpy(o, &hd, sizeof(hd));
    o += sizeof(hd);
    st = ro_cache_save_state(c, o, hd.host_bytes);
    if (st) return st;
    o += hd.host_bytes;
    hipStream_t s = (hipStream_t)stream;
    SnapPart p[10];
    const int n = snap_parts(t, flags, p);
    for (int i = 0; i < n; ++i) {
        RO_HIP(hipMemcpyAsync(o, p[i].dev, p[i].bytes, hipMemcpyDeviceToHost, s));
        o += p[i].bytes;
    }
    RO_HIP(hipStreamSynchronize(s));
    *used = need;
    return RO_OK;
}

extern "C" ro_status ro_restore(ro_octree *t, const void *host_blob, size_t size, void *stream) {
    RO_CHECK(t && host_blob, RO_E_ARG, "null argument");
    RO_CHECK(size >= sizeof(SnapHeader), RO_E_ARG, "snapshot blob too small");
    SnapHeader hd;
    memcpy(&hd, host_blob, sizeof(hd));
    ro_cache *c = t->cache;
    RO_CHECK(hd.magic == kSnapMagic, RO_E_ARG, "not a snapshot blob");
    RO_CHECK(hd.total == c->vol->g.total && hd.slots == c->desc.n_slots && hd.nodes == t->t.n_nodes &&
                 hd.slot_stride == c->vol->g.slot_stride && hd.m == (uint32_t)c->vol->g.m,
             RO_E_ARG, "snapshot was taken from an octree or cache of another shape");
    RO_CHECK(!(hd.flags & ~RO_SNAPSHOT_SLOTS), RO_E_ARG, "unknown snapshot flags 0x%x", hd.flags);
    SnapPart p[10];
    const int n = snap_parts(t, hd.flags, p);
    size_t dev_bytes = 0;
    for (int k = 0; k < n; ++k) dev_bytes += p[k].bytes;
    RO_CHECK(hd.host_bytes >= sizeof(StateHeader) && size == sizeof(hd) + hd.host_bytes + dev_bytes, RO_E_ARG,
             "snapshot blob size %zu does not match its header", size);
    const uint8_t *i = (const uint8_t *)host_blob + sizeof(hd);
    // the host state is checked before anything changes
    StateHeader sh;
    memcpy(&sh, i, sizeof(sh));
    RO_CHECK(sh.magic == kStateMagic && sh.total == c->pt_host.size() && sh.slots == c->slot_host.size() &&
                 sh.channels == c->chmap.size() &&
                 hd.host_bytes == sizeof(sh) + 4 * (sh.total + sh.slots + sh.dirty + sh.channels),
             RO_E_ARG, "snapshot blob's cache state does not match this cache");
    // device arrays, then the host mirrors
    hipStream_t s = (hipStream_t)stream;
    const uint8_t *d = i + hd.host_bytes;
    for (int k = 0; k < n; ++k) {
        RO_HIP(hipMemcpyAsync(p[k].dev, d, p[k].bytes, hipMemcpyHostToDevice, s));
        d += p[k].bytes;
    }
    RO_HIP(hipStreamSynchronize(s));
    return ro_cache_load_state(c, i, hd.host_bytes);
}

extern "C" void ro_octree_destroy(ro_octree *t) { delete t; }

extern "C" ro_status ro_octree_set_leaf_metadata(ro_octree *t, uint32_t channel,
                                                 const uint16_t *leaf_mm, void *stream) {
    RO_CHECK(t && leaf_mm, RO_E_ARG, "null argument");
    RO_CHECK(channel < (uint32_t)t->cache->vol->g.m, RO_E_ARG, "channel %u out of range", channel);
    return octree_set_meta(t, channel, leaf_mm, (hipStream_t)stream);
}

extern "C" ro_status ro_octree_set_leaf_unknown(ro_octree *t, uint32_t channel, void *stream) {
    RO_CHECK(t, RO_E_ARG, "null argument");
    RO_CHECK(channel < (uint32_t)t->cache->vol->g.m, RO_E_ARG, "channel %u out of range", channel);
    return octree_set_meta(t, channel, nullptr, (hipStream_t)stream);
}

extern "C" ro_status ro_octree_leaf_metadata_from_bricks(ro_octree *t, uint32_t n, const uint32_t *ids,
                                                        void *stream) {
    RO_CHECK(t && (ids || n == 0), RO_E_ARG, "null argument");
    const VolGeo &g = t->cache->vol->g;
    // (coarsest level first, dense index) so that finer levels are written last
    std::vector<std::pair<int, uint32_t>> order;
    order.reserve(n);
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t c, l, b[3];
        RO_CHECK(decode_id(g, ids[i], &c, &l, b), RO_E_ARG, "brick ID 0x%08x out of range", ids[i]);
        const uint32_t dn = dense_index(g, (int)c, (int)l, (int)b[0], (int)b[1], (int)b[2]);
        RO_CHECK(t->cache->pt_host[dn] != kInvalid, RO_E_STATE, "brick 0x%08x is not resident", ids[i]);
        order.emplace_back(g.L - 1 - (int)l, dn);
    }
    std::sort(order.begin(), order.end());
    order.erase(std::unique(order.begin(), order.end()), order.end());
    std::vector<uint32_t> dense(order.size());
    for (size_t i = 0; i < order.size(); ++i) dense[i] = order[i].second;
    return octree_meta_from_bricks(t, dense, (hipStream_t)stream);
}

extern "C" ro_status ro_update_residency(ro_octree *t, void *stream) {
    RO_CHECK(t, RO_E_ARG, "null octree");
    std::vector<uint32_t> d;
    d.swap(t->cache->dirty);
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    ro_status st = octree_update(t, d, (hipStream_t)stream);
    if (st) {
        t->cache->dirty.swap(d);  // keep the work for a retry
        return st;
    }
    return RO_OK;
}

extern "C" ro_status ro_rebuild_residency(ro_octree *t, void *stream) {
    RO_CHECK(t, RO_E_ARG, "null octree");
    ro_status st = octree_rebuild(t, (hipStream_t)stream);
    if (st) return st;
    t->cache->dirty.clear();
    return RO_OK;
}

namespace ro {
// Frame validation shared by ro_render and the serving launch.
ro_status validate_frame(const ro_octree *t, const ro_frame_desc *fd, const float *rgba) {
    RO_CHECK(t && fd && rgba, RO_E_ARG, "null argument");
    const VolGeo &g = t->cache->vol->g;
    RO_CHECK(aligned(rgba), RO_E_ARG, "rgba must be 256-byte aligned");
    RO_CHECK(fd->projection == RO_PROJ_ORTHO || fd->projection == RO_PROJ_PERSP, RO_E_ARG,
             "bad projection");
    RO_CHECK(fd->width >= 1 && fd->height >= 1 && fd->width <= 16384 && fd->height <= 16384, RO_E_ARG,
             "bad image size");
    RO_CHECK(fd->step > 0.0 && fd->lod_bias > 0.0 && fd->tx > 0.0 && fd->ty > 0.0, RO_E_ARG,
             "step, lod_bias, tx and ty must be > 0");
    RO_CHECK(fd->n_vis >= 1 && fd->n_vis <= g.m, RO_E_ARG, "n_vis %d not in 1..%d", fd->n_vis, g.m);
    RO_CHECK(fd->tf_dev, RO_E_ARG, "null transfer-function table");
    RO_CHECK(fd->term_alpha > 0.0f && fd->term_alpha <= 1.0f, RO_E_ARG, "term_alpha not in (0, 1]");
    RO_CHECK(fd->frame != kInvalid, RO_E_ARG, "frame 0xFFFFFFFF is reserved");
    RO_CHECK(fd->start_level >= -1 && fd->start_level <= t->t.depth, RO_E_ARG, "bad start_level");
    RO_CHECK(!(fd->flags & ~(RO_RENDER_NO_SKIP | RO_RENDER_AOV | RO_RENDER_ADAPTIVE_STEP | RO_RENDER_HOMOGENEOUS |
                             RO_RENDER_BRICKS | RO_RENDER_CHANNEL_RATES | RO_RENDER_NODES |
                             RO_RENDER_TRAVERSAL_DEPTH)),
             RO_E_ARG,
             "unknown render flags 0x%x", fd->flags);
    RO_CHECK(!(fd->flags & RO_RENDER_AOV) || fd->aov_dev, RO_E_ARG, "AOV requested without buffer");
    RO_CHECK(!(fd->flags & RO_RENDER_BRICKS) || fd->bricks_dev, RO_E_ARG, "required bricks requested without buffer");
    RO_CHECK(!(fd->flags & RO_RENDER_NODES) || fd->nodes_dev, RO_E_ARG, "node marks requested without buffer");
    RO_CHECK(!(fd->flags & RO_RENDER_CHANNEL_RATES) ||
                 ((fd->flags & RO_RENDER_ADAPTIVE_STEP) && !(fd->flags & RO_RENDER_HOMOGENEOUS)),
             RO_E_ARG, "per-channel rates need the adaptive step and exclude homogeneous nodes");
    RO_CHECK(!(fd->flags & RO_RENDER_TRAVERSAL_DEPTH) || (fd->flags & RO_RENDER_ADAPTIVE_STEP), RO_E_ARG,
             "a traversal depth from the step needs the adaptive step");
    uint32_t seen = 0;
    for (int j = 0; j < fd->n_vis; ++j) {
        RO_CHECK(fd->vis[j] >= 0 && fd->vis[j] < g.m, RO_E_ARG, "vis[%d] out of range", j);
        RO_CHECK(!(seen >> fd->vis[j] & 1u), RO_E_ARG, "channel %d listed twice", fd->vis[j]);
        seen |= 1u << fd->vis[j];
        RO_CHECK(fd->lod_lo[j] >= 0 && fd->lod_lo[j] <= fd->lod_hi[j] && fd->lod_hi[j] < g.L, RO_E_ARG,
                 "bad level range for visible slot %d", j);
        RO_CHECK(fd->win_lo[j] < fd->win_hi[j] && fd->win_hi[j] <= (uint32_t)(65535u * 256u),
                 RO_E_ARG, "bad window for visible slot %d", j);
    }
    return RO_OK;
}
}  // namespace ro

extern "C" ro_status ro_render(ro_octree *t, const ro_frame_desc *fd, float *rgba, void *stream) {
    ro_status st = validate_frame(t, fd, rgba);
    if (st) return st;
    return render_device(t, fd, rgba, (hipStream_t)stream);
}
