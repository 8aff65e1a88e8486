/*
 * resoct.h — C ABI of the residency-octree hot path on MI355X (gfx950).
 *
 * Implements ray-guided, mixed-resolution, multi-channel direct volume ray
 * casting over a residency octree (Herzberger et al., "Residency Octree: A
 * Hybrid Approach for Scalable Web-Based Multi-Volume Rendering",
 * arXiv 2309.04393), split along the paper's division of work: the CPU
 * dispatches rendering and memory-management commands, forwards requests
 * and uploads bricks; the GPU renders, records cache misses under a global
 * per-frame limit, and keeps page tables and the residency octree up to
 * date (Sec. 4 System Overview).
 *
 * Conventions
 *  - Every call returns ro_status: 0 on success, < 0 on error; ro_last_error()
 *    returns a thread-local message for the last failing call.  Arguments are
 *    validated before any work is enqueued, and a failing call leaves every
 *    state unchanged.  Device faults surface as RO_E_DEVICE at the next call
 *    that synchronises, carrying the HIP error string.
 *  - Handles are opaque, host-side and not thread-safe: one owner thread per
 *    handle.  Calls on a handle must use one stream (or be ordered by the
 *    caller across streams).
 *  - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *    null stream).  Work is enqueued asynchronously on that stream except
 *    where a call says it synchronises.
 *  - All device memory is owned by the caller: sizes come from the *_query
 *    calls, pointers are handed over at create time, and the library never
 *    frees them.  Destroy calls free host handle memory only.  Device buffers
 *    must be 256-byte aligned.
 *  - Brick IDs (Sec. 7): 32-bit, page-table ID c*k + l in bits 24-31 (c =
 *    cache channel, l = level, k = number of levels), brick z in bits 16-23,
 *    y in 8-15, x in 0-7.  Hence at most 256 bricks per axis per level and
 *    m*k <= 256 page tables.
 *  - Coordinates: L0 voxel i of an axis covers [i, i+1) and has its centre
 *    at i + 1/2; world position = L0 coordinate * spacing.  Level l scales
 *    each axis by a power-of-two factor f_l (axis a is halved from level l-1
 *    to l iff its spacing at l-1 is below twice the smallest spacing at l-1;
 *    halved dims are ceil(n/2)).  Brick b of level l holds level voxels
 *    [b*B, (b+1)*B) per axis and is stored with a one-voxel halo of its
 *    same-level neighbours, clamp-replicated at the level's borders:
 *    (B+2)^3 voxels, x fastest.
 */
#ifndef RESOCT_H
#define RESOCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ro_status;
#define RO_OK 0
#define RO_E_ARG (-1)      /* invalid argument */
#define RO_E_CAPACITY (-2) /* a size exceeds what IDs, buffers or tables can hold */
#define RO_E_NOMEM (-3)    /* host allocation failed */
#define RO_E_DEVICE (-4)   /* HIP error (launch, copy or an earlier asynchronous fault) */
#define RO_E_STATE (-5)    /* call not valid in the handle's current state */

#define RO_MAX_CHANNELS 16
#define RO_MAX_LEVELS 16
#define RO_MAX_DEPTH 20

typedef struct ro_volume ro_volume;
typedef struct ro_cache ro_cache;
typedef struct ro_octree ro_octree;

/* ---------------------------------------------------------------- volume */

/* Bricked multi-resolution multi-channel volume (Sec. 3 "Brick hierarchy";
 * Sec. 4 "Multi-channel data").  All channels share one brick size. */
typedef struct {
    int32_t dims[3];         /* L0 voxels per axis, each >= 1 */
    double spacing[3];       /* world units per L0 voxel, > 0 */
    int32_t n_channels;      /* m: channels referenced by cache and tree, 1..16 */
    int32_t bytes_per_voxel; /* 1 (uint8) or 2 (uint16); values are unsigned raw */
    int32_t brick;           /* B: interior brick edge, power of two in [4, 128] */
    int32_t n_levels;        /* k: resolution levels, 1..16 */
} ro_volume_desc;

/* Validates and derives the level schedule.  RO_E_CAPACITY when a level has
 * more than 256 bricks on an axis or m*k > 256 (brick-ID capacity, Sec. 7). */
ro_status ro_volume_create(const ro_volume_desc *desc, ro_volume **out);
void ro_volume_destroy(ro_volume *v);

/* Level geometry: dims_out[l*3+a], factor_out[l*3+a] (L0 voxels per level
 * voxel) and bricks_out[l*3+a] for l < k.  Any pointer may be NULL. */
ro_status ro_volume_levels(const ro_volume *v, int32_t *dims_out, int32_t *factor_out,
                           int32_t *bricks_out);

/* Total bricks over all channels and levels (= page-table entries). */
ro_status ro_volume_brick_count(const ro_volume *v, uint64_t *count);

/* Brick ID encode / decode (Sec. 7).  RO_E_ARG for out-of-range fields. */
ro_status ro_brick_id_encode(const ro_volume *v, uint32_t c, uint32_t l, const uint32_t b[3],
                             uint32_t *id);
ro_status ro_brick_id_decode(const ro_volume *v, uint32_t id, uint32_t *c, uint32_t *l,
                             uint32_t b[3]);

/* ----------------------------------------------------------------- cache */

/* Brick cache and multi-channel multi-resolution page tables (Sec. 5.1):
 * one pool of equal-size slots shared by all channels and levels. */
typedef struct {
    uint32_t n_slots;   /* S >= 1 */
    uint32_t max_batch; /* most uploads per ro_stream_bricks call, 1..8192 */
} ro_cache_desc;

/* Device buffers of a cache, each caller-allocated with the queried size.
 *  slots       S * slot_stride bytes: brick voxels, (B+2)^3 per slot
 *  page_table  one uint32 per brick: slot or 0xFFFFFFFF (not resident)
 *  counters    one uint32 per brick: cache-miss counts of the current frame;
 *              must be zero at create (the create call clears it)
 *  slot_brick  one uint32 per slot: brick index held, 0xFFFFFFFF if free
 *  stamps      one uint32 per slot: frame of last use or upload (LRU)
 *  seqs        one uint32 per slot: upload sequence number (LRU tie-break)
 *  scratch     work space of the streaming and compaction kernels */
typedef struct {
    size_t slots, page_table, counters, slot_brick, stamps, seqs, scratch;
    size_t slot_stride; /* bytes per slot (and per staged brick), multiple of 256 */
} ro_cache_sizes;

typedef struct {
    void *slots;
    uint32_t *page_table, *counters, *slot_brick, *stamps, *seqs;
    void *scratch;
} ro_cache_buffers;

ro_status ro_cache_query(const ro_volume *v, const ro_cache_desc *desc, ro_cache_sizes *out);

/* Clears page table, counters, slot map, stamps and seqs on `stream`. */
ro_status ro_cache_create(const ro_volume *v, const ro_cache_desc *desc,
                          const ro_cache_buffers *bufs, void *stream, ro_cache **out);
void ro_cache_destroy(ro_cache *c);

/* Upload one batch of bricks in frame `frame` (Sec. 5.3 "Updating residency
 * information", "LRU cache eviction").  ids_host[n] are brick IDs in the
 * policy's order; staged_dev holds n bricks, brick i at
 * staged_dev + i * slot_stride, halo included.  Slots are assigned on the
 * GPU: free slots first in ascending order, then resident slots in ascending
 * (stamp, seq) order, never a slot whose stamp equals `frame` (used this
 * frame).  An ID resident at the start of the batch, or repeated earlier in
 * it, gets flag 2 and its slot's stamp is set to `frame`; uploads that find
 * no eligible slot get flag 0; inserted ones flag 1 (inserted_host[n]).
 * Evicted and inserted bricks are recorded for ro_update_residency: the
 * page tables change at once, but the renderer picks a channel's level from
 * the octree's residency masks, so frames see the new bricks (and stop
 * substituting evicted ones) after ro_update_residency.  Until then a level
 * whose mask bit is stale and whose page-table entry is empty contributes
 * nothing at that sample (never an out-of-range read).
 * Synchronises on `stream` before returning (flags are host memory).
 * n <= max_batch; frame < 0xFFFFFFFF. */
ro_status ro_stream_bricks(ro_cache *c, uint32_t frame, uint32_t n, const uint32_t *ids_host,
                           const void *staged_dev, uint8_t *inserted_host, void *stream);

/* Cache-miss readback (Sec. 4: global limit on recorded misses per frame).
 * Compacts the per-brick counters into (id, count) pairs in ascending ID
 * order, returns at most `cap` of them, the number of distinct requested
 * bricks (*n_unique, may exceed cap) and the sum of all counts
 * (*total_missing), then zeroes the counters.  Synchronises. */
ro_status ro_read_requests(ro_cache *c, uint32_t cap, uint32_t *ids_host, uint32_t *counts_host,
                           uint32_t *n_unique, uint64_t *total_missing, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): the same readback
 * as ro_read_requests (same outputs, counters cleared the same way), with its
 * work space in a fixed device array of the library instead of the cache's
 * scratch buffer.  Allocates nothing.  Limits: cap <= RO_NOALLOC_MAX_PAIRS
 * and a volume of at most 2^26 bricks; beyond them RO_E_CAPACITY and nothing
 * is enqueued.  The array (about 2.5 MiB) exists once per GPU until the
 * process ends and keeps the last call's contents; every call on a GPU uses
 * that GPU's copy, so calls that overlap on one GPU (other threads or
 * streams) race.  Synchronises. */
#define RO_NOALLOC_MAX_PAIRS 262144u
ro_status ro_read_requests_noalloc(ro_cache *c, uint32_t cap, uint32_t *ids_host, uint32_t *counts_host,
                                   uint32_t *n_unique, uint64_t *total_missing, void *stream);

/* Slots read during frame `frame` (stamp == frame), ascending, at most cap;
 * *n_out receives the full count.  Synchronises. */
ro_status ro_read_usage(ro_cache *c, uint32_t frame, uint32_t cap, uint32_t *slots_host,
                        uint32_t *n_out, void *stream);

/* Checkpoint of the whole residency state (Sec. 4: the CPU holds the
 * state it needs to restart the GPU side): page table, miss counters, slot
 * map, LRU stamps and upload sequence numbers, node metadata, residency masks
 * and node flags of the octree and its cache, the cache's host mirrors
 * (page table, slot map, bricks awaiting a residency update, upload
 * counter), and with RO_SNAPSHOT_SLOTS the slot contents (slot_stride x
 * n_slots bytes).  ro_snapshot_size gives the blob size for the current
 * state; ro_snapshot writes it to host memory (RO_E_CAPACITY if cap is
 * smaller; *used = bytes written) and synchronises.  ro_restore brings an
 * octree and its cache of the same shapes back to the snapshot's state
 * (RO_E_ARG for a blob of another shape or size, nothing changed); without
 * RO_SNAPSHOT_SLOTS the slots must still hold what they held at the
 * snapshot.  Frames rendered after a restore are those rendered after the
 * snapshot.  Synchronises. */
#define RO_SNAPSHOT_SLOTS 1u
ro_status ro_snapshot_size(const ro_octree *t, uint32_t flags, size_t *bytes);
ro_status ro_snapshot(const ro_octree *t, uint32_t flags, void *host_blob, size_t cap, size_t *used,
                      void *stream);
ro_status ro_restore(ro_octree *t, const void *host_blob, size_t size, void *stream);

/* Run-time channel exchange (Sec. 5.2: when another data channel takes a
 * cache channel's place, what the cache holds for the old one is no longer
 * valid).  Every resident brick of cache channel `channel` leaves the cache:
 * its page-table entry is cleared and its slot becomes free (free slots are
 * taken first, in ascending index, by later uploads); the bricks join the
 * set awaiting ro_update_residency.  The caller then gives the channel the
 * new data's metadata (or [0, max] for unknown leaves), runs the residency
 * update and uploads the new bricks under the same channel's IDs.  Frames
 * rendered before the residency update read nothing of the channel's old
 * bricks (the page tables are already cleared).  RO_E_ARG if the channel is
 * out of range.  Queues one kernel; the host mirrors change at once. */
ro_status ro_cache_evict_channel(ro_cache *c, uint32_t channel, void *stream);

/* Channel map (Sec. 5.2: the octree and page tables reference m of the data
 * server's channels at a time; a cache channel can be given another data
 * channel at run time).  Host state of the cache: cache channel c shows
 * source channel map[c], the identity at create.  The GPU works in cache
 * channels only; the map names the data behind them, so requests read back
 * as brick IDs (cache channel, level, brick) are fetched from the server
 * through ro_cache_source_bricks.  Set it with the exchange
 * (ro_cache_evict_channel).  RO_E_ARG for a cache channel >= m. */
ro_status ro_cache_set_channel_map(ro_cache *c, uint32_t cache_channel, uint32_t source_channel);
/* map[m]: the source channel of every cache channel. */
ro_status ro_cache_get_channel_map(const ro_cache *c, uint32_t *map);
/* For each of ids[n]: out[5 i ..] = (source channel, level, bx, by, bz), the
 * brick as the data server names it.  RO_E_ARG, with nothing written, if an
 * ID is out of range. */
ro_status ro_cache_source_bricks(const ro_cache *c, uint32_t n, const uint32_t *ids, uint32_t *out);

/* Copy of the host mirror of the page table: brick index -> slot
 * (0xFFFFFFFF when not resident), `count` entries from ro_volume_brick_count. */
ro_status ro_cache_page_table_host(const ro_cache *c, uint32_t *out, uint64_t count);

/* Host-side state of a cache: page-table and slot-map mirrors, bricks
 * awaiting a residency update, channel map, upload counter.  Together with copies of the
 * caller-owned device buffers (page table, counters, slot map, stamps, seqs,
 * slots, node masks and metadata) it is a complete checkpoint: save, later
 * copy the device buffers back and load, and the cache continues exactly as
 * from the save point.  save/load do not touch device memory. */
ro_status ro_cache_state_size(const ro_cache *c, size_t *bytes);
ro_status ro_cache_save_state(const ro_cache *c, void *host, size_t cap);
/* RO_E_ARG if the blob was saved from a cache of another shape. */
ro_status ro_cache_load_state(ro_cache *c, const void *host, size_t size);

/* ---------------------------------------------------------------- octree */

/* Residency octree (Sec. 5.2): a full pointerless tree over the L0 domain
 * padded to a power of two number of leaves per axis.  Axis a needs s_a
 * splits (leaf_a * 2^s_a >= dims_a) and takes them at the last s_a of the
 * `depth` subdivision levels; node size at level d is
 * leaf_a << min(s_a, depth - d).  Leaf edges must be powers of two that
 * divide B, so a leaf lies inside exactly one brick of every level.  Each
 * node stores per channel the metadata [min, max] (uint16 each, packed
 * min | max << 16) and the mask of levels in which it is partially mapped
 * (uint16). */
typedef struct {
    int32_t leaf[3];     /* leaf edge in L0 voxels, powers of two dividing B */
    int32_t depth;       /* subdivision levels below the root, <= 20 */
    int32_t start_level; /* level where traversal starts each time a ray enters a leaf */
} ro_octree_desc;

/*  node_meta   n_nodes * m uint32 (min | max << 16)
 *  node_mask   n_nodes * m uint16
 *  node_flags  n_nodes bytes (propagation work flags)
 *  scratch     leaf-update work list
 *  leaf_level  n_leaves * m bytes: where each leaf's metadata came from (0 the
 *              server or level-0 bricks, l level-l bricks, 255 unknown) */
typedef struct {
    size_t node_meta, node_mask, node_flags, scratch, leaf_level;
    uint64_t n_nodes, n_leaves;
    int32_t leaf_grid[3]; /* leaves per axis (padded) */
} ro_octree_sizes;

typedef struct {
    uint32_t *node_meta;
    uint16_t *node_mask;
    uint8_t *node_flags;
    void *scratch;
    uint8_t *leaf_level;
} ro_octree_buffers;

ro_status ro_octree_query(const ro_volume *v, const ro_octree_desc *desc, ro_octree_sizes *out);

/* Clears metadata (to [0, 0]), masks and flags; every leaf's metadata level
 * is 255 (unknown).  The octree refers to the
 * cache's page tables; destroy it before the cache. */
ro_status ro_octree_create(ro_cache *c, const ro_octree_desc *desc,
                           const ro_octree_buffers *bufs, void *stream, ro_octree **out);
void ro_octree_destroy(ro_octree *t);

/* Leaf metadata of one channel from the data server (Sec. 4; Sec. 5.3
 * "Updating culling information"): leaf_minmax_dev[n_leaves][2] uint16
 * (min, max) over the padded leaf grid, x fastest.  Must be conservative
 * for every L0 voxel within one voxel of the leaf.  Inner nodes then get the
 * min of their children's minima and the max of their maxima.  The leaves'
 * metadata level becomes 0 (brick data do not replace them). */
ro_status ro_octree_set_leaf_metadata(ro_octree *t, uint32_t channel,
                                      const uint16_t *leaf_minmax_dev, void *stream);

/* Unknown leaves (Sec. 5.2: node information not yet initialised; Alg. 1
 * reportNodeRequest): every leaf of the channel gets [0, max raw value],
 * which no transfer function can call empty or homogeneous, and metadata
 * level 255, so the first brick data covering it (ro_octree_leaf_metadata_
 * from_bricks) give it metadata; inner nodes are reduced again. */
ro_status ro_octree_set_leaf_unknown(ro_octree *t, uint32_t channel, void *stream);

/* Leaf metadata computed from resident brick data (Sec. 5.3: a client whose
 * server has no metadata derives it from the voxels it fetched; the
 * application picks the resolution level).  ids_host[n]: brick IDs, each
 * resident (else RO_E_STATE) and in range (else RO_E_ARG); on either error
 * nothing changes.  Every leaf of the padded grid inside such a brick's
 * extent gets, for the brick's channel, [min, max] over the voxels of the
 * brick's level that overlap the leaf box dilated by one voxel of that level
 * and clamped to the level's grid ([0, 0] if nothing is left): at level 0
 * exactly the conservative metadata ro_octree_set_leaf_metadata asks for; at
 * coarser levels an estimate from fewer voxels, which may miss extremes.
 * A leaf takes a brick's values only when the brick's level is at most the
 * leaf's metadata level, which then becomes the brick's level: metadata are
 * refined by finer data and never replaced by coarser ones, across calls and
 * within one.  Leaves outside the given bricks keep their metadata: to keep
 * them from being skipped before their data arrive, make them unknown first
 * (ro_octree_set_leaf_unknown).  Inner nodes of the touched channels are
 * then reduced again.  Reads the slots: call it after the ro_stream_bricks
 * that uploaded them, on the same stream or after it has completed.  Returns
 * after the work is queued (it waits for its own copies of the work list). */
ro_status ro_octree_leaf_metadata_from_bricks(ro_octree *t, uint32_t n, const uint32_t *ids_host,
                                              void *stream);

/* Residency update for the bricks inserted or evicted since the last call
 * (Sec. 5.3): each leaf overlapping such a brick gets bit l of its channel's
 * mask set iff the level-l brick containing it is resident; then every
 * inner node whose children changed gets the OR of its children, level by
 * level, stopping where nothing changed. */
ro_status ro_update_residency(ro_octree *t, void *stream);

/* From-scratch recomputation of every mask from the page tables. */
ro_status ro_rebuild_residency(ro_octree *t, void *stream);

/* ---------------------------------------------------------------- render */

#define RO_PROJ_ORTHO 0
#define RO_PROJ_PERSP 1

#define RO_RENDER_NO_SKIP 1u /* evaluate every sample (results are identical) */
#define RO_RENDER_AOV 2u     /* write per-pixel per-level sample counts to aov_dev */
#define RO_RENDER_ADAPTIVE_STEP 4u /* LOD-adaptive sampling distance (see below) */
#define RO_RENDER_HOMOGENEOUS 8u   /* nodes homogeneous for all channels rendered from their values (see below) */
#define RO_RENDER_BRICKS 16u       /* write the bricks each pixel requires to bricks_dev (see below) */
#define RO_RENDER_CHANNEL_RATES 32u /* with the adaptive step: per-channel sampling rates (see below) */
#define RO_RENDER_NODES 64u        /* mark the nodes whose metadata the frame reads in nodes_dev */
#define RO_RENDER_TRAVERSAL_DEPTH 128u /* with the adaptive step: decision node from the step (see below) */

/* One frame (Sec. 6.1, Alg. 1; Sec. 6.2).  Pixel (i, j), row 0 at the top,
 * has a = (2i+1-W)/W, b = (H-2j-1)/H.  Orthographic: origin
 * eye + a*tx*right + b*ty*up, direction forward.  Perspective: origin eye,
 * direction normalize(forward + a*tx*right + b*ty*up).  Samples at
 * t_k = k*step along the ray (world units, k = 0, 1, ...), those outside
 * the volume are void.  For every sample and visible channel:
 *  - a leaf whose metadata make the channel's transfer function zero over
 *    every table entry reachable from [min, max] contributes nothing and
 *    requests nothing;
 *  - desired level l* = clamp(#{l >= 1 : t >= D_l}, lod_lo, lod_hi) with
 *    D_l = s_l / (lod_bias * 2 ty / H), s_l the level's x voxel size
 *    (orthographic views use the pixel size 2 ty / H in place of t * 2ty/H);
 *  - a missing desired brick adds one to its miss counter, and the finest
 *    resident level >= l* substitutes (none: the channel contributes
 *    nothing); every slot read gets its stamp set to `frame`;
 *  - value = trilinear interpolation in the slot; the transfer function maps
 *    v to clamp((v - win_lo/256) / ((win_hi - win_lo)/256), 0, 1) * 255
 *    and interpolates linearly in the channel's 256-entry RGBA table.
 * Channels mix per sample as alpha = 1 - prod(1 - alpha_c),
 * colour = alpha * sum(alpha_c rgb_c) / sum(alpha_c); samples composite
 * front to back (premultiplied), and a ray stops once its opacity reaches
 * term_alpha.  Empty-space skipping and the traversal start level change no
 * output.
 * RO_RENDER_ADAPTIVE_STEP (Sec. 6.1: the sampling distance may grow with the
 * resolution level): at sample k let l_s = clamp(#{l >= 1 : t >= D_l},
 * min lod_lo, min lod_hi), the finest desired level over the visible
 * channels, and r its x factor (a power of two).  The sample is evaluated
 * only when k is a multiple of r (so skipping resumes on the same grid), and
 * its mixed opacity becomes 1 - (1 - alpha)^r with the premultiplied colour
 * scaled by the same factor.  Where l_s = 0 the frame is unchanged.
 * RO_RENDER_CHANNEL_RATES (Sec. 6.1: a channel may need only every second
 * step; the channel needing the highest rate sets the step), only with
 * RO_RENDER_ADAPTIVE_STEP and not with RO_RENDER_HOMOGENEOUS: channel c takes
 * part in sample k only when k is a multiple of r_c, the x factor of its own
 * desired level clamp(l*, lod_lo[c], lod_hi[c]); there it stands for r_c base
 * steps, with transparency (1 - alpha_c)^r_c and colour weight r_c alpha_c,
 * and the sample's opacity is 1 - prod of those transparencies (no further
 * correction).  A channel's requests, reads and stamps come only from the
 * samples it takes part in.  With one level range for every channel the
 * frame is the adaptive one.
 * RO_RENDER_TRAVERSAL_DEPTH (Alg. 1 chooseTraversalDepth: the tree is not
 * traversed below a node the step would jump over), only with
 * RO_RENDER_ADAPTIVE_STEP: a sample taken with step factor r decides
 * emptiness and homogeneity at the deepest node whose smallest world extent
 * is at least r * step (the leaf when the leaf is that large), so a channel
 * not empty in that node samples its brick even where its own leaf is
 * empty; requests and substitution stay per sample (leaf masks).  Where
 * every step fits in a leaf the frame is the adaptive one.
 * RO_RENDER_HOMOGENEOUS (Alg. 1 isHomogeneous / renderAndSkipNode; Sec. 6.1:
 * a node is rendered from its value only when it is homogeneous for all
 * channels): a channel is homogeneous in a node whose metadata hold one value
 * (min == max).  A node in which every visible channel is empty or
 * homogeneous, and at least one is homogeneous, is rendered from those values
 * and skipped: each of its samples takes, per homogeneous channel, the node's
 * value through the transfer function, mixed and composited like a sampled
 * one; no brick is read, requested or stamped there, whatever is resident and
 * whatever level is desired.  Samples stay on the same grid, so early
 * termination falls on the same sample.  Every other node is rendered as
 * without the option (a channel homogeneous in a node that is not is sampled
 * from its brick).  Where level 0 is read and the metadata are exact, the
 * image is the same as without the option. */
typedef struct {
    uint32_t frame;     /* frame number written into slot stamps, < 0xFFFFFFFF */
    int32_t projection; /* RO_PROJ_ORTHO or RO_PROJ_PERSP */
    double eye[3], forward[3], right[3], up[3];
    double tx, ty;      /* ortho: half extents (world); perspective: tan of half angles */
    int32_t width, height;
    double step;        /* world distance between samples, > 0 */
    double lod_bias;    /* > 0 */
    int32_t n_vis;      /* visible channels, 1..m */
    int32_t vis[RO_MAX_CHANNELS];    /* cache channel of each visible slot, distinct */
    int32_t lod_lo[RO_MAX_CHANNELS]; /* per visible slot resolution range, lo <= hi < k */
    int32_t lod_hi[RO_MAX_CHANNELS];
    uint32_t win_lo[RO_MAX_CHANNELS]; /* window in raw units, 24.8 fixed point, lo < hi */
    uint32_t win_hi[RO_MAX_CHANNELS];
    const float *tf_dev;  /* device [n_vis][256][4] RGBA, alpha >= 0 */
    float term_alpha;     /* in (0, 1] */
    int32_t start_level;  /* traversal start level (Sec. 7, implementation), -1: the octree's */
    uint32_t flags;       /* RO_RENDER_*; other bits are rejected (RO_E_ARG) */
    uint32_t *aov_dev;    /* RO_RENDER_AOV: device [H][W][k] uint32, zeroed by the caller */
    unsigned long long *stats_dev; /* optional device [8], accumulated (not cleared): [0] ray
                                      samples evaluated, [1] channel samples read from bricks,
                                      [2] channel samples whose desired brick was missing,
                                      [3] (leaf, level) visits, [4] channel samples in leaves
                                      that are not empty for the channel, [5] lane slots of
                                      the wave stepping iterations ([0] / [5] = share of
                                      lanes busy), [6] ray samples rendered from
                                      homogeneous nodes; [7] zero */
    uint32_t *bricks_dev; /* RO_RENDER_BRICKS: device [H][W][1 + n_vis] uint32; word 0 of a
                             pixel receives the number of bricks the pixel requires (Sec. 8,
                             bricks required to be resident per pixel): the distinct desired
                             bricks (channel, l*, brick) of its samples in leaves where the
                             channel is not empty, outside nodes rendered from their values,
                             up to its early termination, resident or not; words 1..n_vis
                             are the kernel's work space.  Needs no clearing. */
    uint8_t *nodes_dev;   /* RO_RENDER_NODES: device [n_nodes] uint8, zeroed by the caller; every
                             node whose metadata the frame's descents read gets 1 (the tree's
                             part of the frame's memory traffic) */
} ro_frame_desc;

/* Renders into rgba_dev[H][W][4] (float, premultiplied) and updates the
 * miss counters and slot stamps.  Asynchronous.  The kernel's work queue
 * counters live in the octree's scratch buffer, so frames of one octree are
 * rendered one at a time (in stream order); use the server below for
 * concurrent requests. */
ro_status ro_render(ro_octree *t, const ro_frame_desc *fd, float *rgba_dev, void *stream);

/* ------------------------------------------------------------- predictor */

/* Brick-request predictor: an addition to the paper's method that only
 * changes which bricks a policy streams, never the image rendered from a
 * given cache state.  A perceptron 24 -> 64 -> 64 -> 9 with ReLU hidden
 * layers and one logit per resolution level:
 *   h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), z = h2 W3 + b3,
 * trained with binary cross-entropy on the logits, masked per (row, level),
 * mean over unmasked entries, by Adam (beta 0.9 / 0.999, eps 1e-8) on FP32
 * master weights.  Products run on MFMA with FP16 operands and FP32
 * accumulation.  Device layouts: features x [rows][32] FP16 (features
 * 0..23, the rest zero); logits z [rows][16] FP32 (0..8 used); labels y and
 * mask [rows][16] uint8 0/1.  Host weight layout (FP32, input-major):
 * W1[24][64], b1[64], W2[64][64], b2[64], W3[64][9], b3[9] (6217 floats). */
typedef struct ro_mlp ro_mlp;
ro_status ro_mlp_query(size_t *param_bytes, size_t *workspace_bytes);
ro_status ro_mlp_create(void *params_dev, void *workspace_dev, ro_mlp **out);
void ro_mlp_destroy(ro_mlp *n);
/* Loads weights and resets the optimiser state.  Synchronises. */
ro_status ro_mlp_set_weights(ro_mlp *n, const float *host, void *stream);
ro_status ro_mlp_get_weights(const ro_mlp *n, float *host, void *stream); /* synchronises */
ro_status ro_mlp_forward(ro_mlp *n, const uint16_t *x_dev, uint32_t rows, float *z_dev, void *stream);
/* Gradient of the loss at the current weights (host layout above) and the
 * loss; no update.  Synchronises. */
ro_status ro_mlp_gradients(ro_mlp *n, const uint16_t *x_dev, const uint8_t *y_dev, const uint8_t *mask_dev,
                           uint32_t rows, float *grads_host, float *loss_host, void *stream);
/* One Adam step; *loss_host (if not NULL) receives the loss before the step
 * (then the call synchronises). */
ro_status ro_mlp_train_step(ro_mlp *n, const uint16_t *x_dev, const uint8_t *y_dev, const uint8_t *mask_dev,
                            uint32_t rows, float lr, float *loss_host, void *stream);

/* Predictor rows and bookkeeping.  Rows: one per (cache channel c, L0 brick
 * position p), row = c * P + p, p = (z * nby + y) * nbx + x over the L0
 * brick grid (P positions, m * P rows).  History: one byte per brick, bits
 * 0-3 requested in the last four frames (bit 0 = latest), bits 4-7 read in
 * them.  Features (24 per row, FP16, written into x_dev[rows][32]): brick
 * edge in pixels and distance relative to the first level threshold (log2),
 * desired level, frustum flag, projected position, depth, fraction of the
 * brick's leaves not empty under the channel's transfer function (0 when the
 * channel is not visible), request and read history of the L0 brick,
 * residency of the bricks covering it at levels 0..7.  Labels: level l of a
 * row is 1 iff the level-l brick covering the row's position was requested
 * or read in the last four frames (use with features from four frames
 * before); mask = 1 for existing levels (at most 9). */
typedef struct ro_prefetch ro_prefetch;
ro_status ro_pf_query(const ro_octree *t, uint32_t *rows, size_t *hist_bytes, size_t *score_bytes);
/* hist_dev and score_dev are caller-allocated device buffers of the queried
 * sizes; both are cleared. */
ro_status ro_pf_create(ro_octree *t, uint8_t *hist_dev, uint32_t *score_dev, void *stream, ro_prefetch **out);
void ro_pf_destroy(ro_prefetch *p);
/* Shift the history and record this frame's requests (miss counters, so call
 * after ro_render and before ro_read_requests) and reads (stamp == frame). */
ro_status ro_pf_record(ro_prefetch *p, uint32_t frame, void *stream);
ro_status ro_pf_features(ro_prefetch *p, const ro_frame_desc *fd, uint16_t *x_dev, void *stream);
ro_status ro_pf_labels(ro_prefetch *p, uint8_t *y_dev, uint8_t *mask_dev, void *stream);
/* Bricks not resident whose predicted probability sigmoid(z) exceeds
 * `threshold` for some row (z_dev [rows][16] logits), with the best
 * probability per brick, in ascending ID order; at most cap returned,
 * *n_out = all of them.  Synchronises. */
ro_status ro_pf_candidates(ro_prefetch *p, const float *z_dev, float threshold, uint32_t cap, uint32_t *ids_host,
                           float *prob_host, uint32_t *n_out, void *stream);

/* --------------------------------------------------------------- serving */

/* Batched rendering for a serving loop (an addition to the paper's method):
 * one persistent kernel renders up to 64 frame requests of different
 * viewports, channel subsets, transfer functions and cameras over the shared
 * cache and octree; its workgroups pop work items (up to 96 blocks of 8 x 8
 * pixels of one request; ro_serve_work_items counts them) from a device
 * queue.  Each pixel runs the same code as ro_render, so a request's image is
 * the same alone and in any batch.
 *
 * A server owns pinned host memory for two batches ("halves", used
 * alternately) and two non-blocking streams of default priority, one per
 * half; the caller owns the device buffer (size from ro_serve_query, 256-byte
 * aligned) that holds the halves' device copies and queue counters.  Batches
 * from different halves may run concurrently.  The serving kernel reads the
 * cache and octree and adds to the request counters; the caller must not
 * stream bricks or update residency while a batch is in flight (wait for its
 * ticket), and usage stamps written by overlapping batches of different frame
 * numbers end with either value.  Not thread-safe. */
#define RO_SERVE_GRAPH 1u
typedef struct ro_server ro_server;
ro_status ro_serve_query(uint32_t max_requests, uint32_t max_tiles, size_t *device_bytes);
/* Work items of a width x height request. */
ro_status ro_serve_work_items(int32_t width, int32_t height, uint32_t *items);
/* max_requests in 1..64 per batch; max_tiles (work items) in 1..2^24 per
 * batch. */
ro_status ro_serve_create(ro_octree *t, uint32_t max_requests, uint32_t max_tiles, void *device_buf,
                          ro_server **out);
/* Waits for outstanding batches, then frees the server's resources. */
void ro_serve_destroy(ro_server *s);
/* Host side of a batch: fds[n] as for ro_render (no AOV), rgba_dev[n] output
 * images ([H][W][4] float, 256-byte aligned).  Writes the next half after
 * waiting for that half's previous batch to finish.  full_channels != 0
 * selects the 16-channel kernel whatever the batch holds, which graph
 * submission requires.  RO_E_CAPACITY when n or the batch's tiles exceed the
 * server's limits, RO_E_STATE when a prepared batch is still unsubmitted;
 * nothing is submitted on error. */
ro_status ro_serve_prepare(ro_server *s, uint32_t n, const ro_frame_desc *fds, float *const *rgba_dev,
                           int32_t full_channels);
/* Device side: on the half's stream, copy the prepared half to its device
 * copy, reset its queue and run the kernel.  With RO_SERVE_GRAPH the sequence
 * is captured into a graph on the half's first such submission and replayed
 * afterwards (it depends only on the half).  *ticket (may be null) names the
 * batch for ro_serve_poll / ro_serve_wait. */
ro_status ro_serve_submit(ro_server *s, uint32_t flags, uint64_t *ticket);
/* *done = 1 when the batch has finished (its images and counters are
 * written), else 0. */
ro_status ro_serve_poll(ro_server *s, uint64_t ticket, int32_t *done);
/* *done = 1 when request r (its index in the batch) of the batch has
 * finished: the kernel posts each request's completion to mapped host
 * memory as soon as its last work item is written, before the batch ends. */
ro_status ro_serve_request_done(ro_server *s, uint64_t ticket, uint32_t r, int32_t *done);
ro_status ro_serve_wait(ro_server *s, uint64_t ticket);
/* prepare (kernel chosen by the batch's largest channel count) + submit. */
ro_status ro_serve_launch(ro_server *s, uint32_t n, const ro_frame_desc *fds, float *const *rgba_dev,
                          uint64_t *ticket);

/* Continuous admission (an addition to the paper's method, next to the
 * batches above): requests are admitted one at a time, whenever the caller
 * likes, also while others render.  The server appends the request's work
 * items to a ring of max_tiles (rounded up to a power of two) entries in
 * mapped pinned host memory and publishes them; the workgroups of every
 * running serving kernel take the next published item as they free up, and
 * each call also launches a kernel (the 16-channel instance, at most one
 * workgroup per compute unit, alternating between two non-blocking streams
 * of default priority) for the compute units that have emptied.  A kernel's
 * workgroups leave as soon as no published item is left: no kernel ever
 * waits for the host.  The same per-ray code as ro_render runs, so the image
 * is the same as the frame kernel's.  Up to max_requests requests are
 * unfinished at once (one descriptor slot each).
 *
 * ro_serve_enqueue: fd as for ro_serve_prepare (no diagnostic outputs, no
 * homogeneous nodes, rates or traversal depths), rgba_dev the [H][W][4]
 * float output (256-byte aligned).  RO_E_CAPACITY, with nothing admitted,
 * when every slot holds an unfinished request or the ring has no room for
 * the request's items (retry after completions).  *ticket names the request
 * for ro_serve_done.  The caller keeps the output and the transfer-function
 * tables alive until the request has finished.  Batches and continuous
 * admission may be mixed (their queues are separate); the same rules on
 * streaming and residency updates apply (no changes while requests are
 * unfinished).  Tickets are 32-bit serials from 1 on (a server admits fewer
 * than 2^32 requests). */
ro_status ro_serve_enqueue(ro_server *s, const ro_frame_desc *fd, float *rgba_dev, uint64_t *ticket);
/* *done = 1 once the request's last work item is written (the kernel posts
 * it to mapped host memory), else 0.  RO_E_ARG for a ticket never issued. */
ro_status ro_serve_done(ro_server *s, uint64_t ticket, int32_t *done);
/* Waits until every admitted request has finished and its kernels ended. */
ro_status ro_serve_drain(ro_server *s);

/* Thread-local message of the last failing call ("" if none). */
const char *ro_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
