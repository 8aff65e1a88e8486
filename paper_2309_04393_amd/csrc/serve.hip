// Multi-request rendering for the serving loop (an addition to the paper's
// method): one persistent kernel renders a batch of frame requests of
// different viewports, channel subsets and transfer functions over the
// shared cache and octree.  Workgroups pop work items (up to 96 blocks of
// 8 x 8 pixels of one request) from a device queue; when an item belongs to
// another request than the previous one, the workgroup stages that
// request's descriptor and tables in LDS.  Every pixel runs the same per-ray
// code as the frame kernel, so a request's image does not depend on what
// else is in the batch.
//
// The host prepares descriptors and the work list in pinned host memory owned
// by the server.  There are two halves used alternately, each with its own
// device copy, queue counter and stream, so a batch can be prepared while the
// previous one renders and the tail of one batch overlaps the head of the
// next.  A submission copies the prepared half to the device and launches the
// kernel with arguments that depend only on the half; with the 16-channel
// kernel this sequence is captured once per half as a graph and replayed.
#include <math.h>
#include <string.h>

#include <new>

#include "render_core.h"

namespace ro {

// Batch header (device copy of the prepared half).
struct ServeHeader {
    uint32_t n_tiles;
    uint32_t n_req;
    uint32_t seq;              // batch ticket (low 32 bits), posted per finished request
    uint32_t pad0;
    uint32_t *done;            // device [max_req] finished work items per request
    volatile uint32_t *flags;  // mapped host [max_req] completion tickets
    uint32_t pad[56];
};

// Work items of a W x H request: its 8 x 8 blocks (16 per 32 x 32 tile) in
// groups of kSegBlocks.
__host__ __device__ inline uint32_t serve_segments(int W, int H) {
    const uint64_t blocks = (uint64_t)((W + 31) / 32) * (uint64_t)((H + 31) / 32) * 16u;
    return (uint32_t)((blocks + kSegBlocks - 1) / kSegBlocks);
}


// Renders work item `seg` (kSegBlocks consecutive 8 x 8-pixel blocks, the
// blocks of a 32 x 32 tile consecutive, tiles in raster order) of the
// request staged in sA.  The workgroup's waves take the item's blocks from
// the LDS counter *s_next (zero on entry) one at a time, so waves that
// finish early take more blocks.
template <int NV, int BPV, int EC>
__device__ __forceinline__ void serve_item(const RenderArgs &sA, uint32_t seg, uint32_t *s_next, const float4 *s_tf,
                                           const ChanLds *s_ch, const uint32_t *s_runs, const LevLds *s_lv,
                                           const NodeLds *s_nd) {
    const uint32_t tiles_x = ((uint32_t)sA.W + 31) / 32, tiles_y = ((uint32_t)sA.H + 31) / 32;
    const uint32_t first = seg * kSegBlocks, n_blk = tiles_x * tiles_y * 16;
    BlockQueue q;
    q.counter = s_next;
    q.n_blocks = min(kSegBlocks, n_blk - first);
    q.offset = first;
    q.tiles_x = tiles_x;
    q.n_queues = 1;
    q.chunk = 1;
    q.W = sA.W;
    q.H = sA.H;
    q.min_idle = 64;
    uint32_t st[7] = {0, 0, 0, 0, 0, 0, 0};
    const LdsSlots sl{(uint32_t *)(s_tf + kTfStride * NV) + threadIdx.x, (uint32_t)kRenderLanes};
    render_rays<NV, BPV, false, EC, true, 0>(sA, q, s_tf, s_ch, s_runs, s_lv, s_nd, st, sl);
    if (sA.stats) {
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            uint32_t v = st[j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if ((threadIdx.x & 63) == 0 && v) atomicAdd(&sA.stats[j], (unsigned long long)v);
        }
    }
}

// A workgroup takes a work item, stages the request's tables if it changed,
// renders the item and waits for its slowest wave once per item.
template <int NV, int BPV, int EC>
__global__ void __launch_bounds__(kRenderLanes) __attribute__((amdgpu_waves_per_eu(kRenderLanes / 256)))
    k_serve(const ServeHeader *__restrict__ hdr, const RenderArgs *__restrict__ descs,
            const uint32_t *__restrict__ segs, uint32_t *__restrict__ queue) {
    extern __shared__ float4 s_tf[];  // [NV][kTfStride] tables, then [NV][kRenderLanes] slot words
    __shared__ RenderArgs sA;
    __shared__ ChanLds s_ch[NV];
    __shared__ uint32_t s_runs[NV * kMaxRuns];
    __shared__ LevLds s_lv[kMaxL];
    __shared__ NodeLds s_nd[kMaxD + 1];
    __shared__ uint32_t s_seg, s_next;
    const uint32_t n_segs = hdr->n_tiles;
    int cur = -1;
    for (;;) {
        if (threadIdx.x == 0) {
            s_seg = atomicAdd(queue, 1u);
            s_next = 0;
        }
        __syncthreads();
        const uint32_t seg = s_seg;
        if (seg >= n_segs) break;
        const uint32_t sw = segs[seg];
        const int req = (int)(sw >> 26);
        if (req != cur) {
            const uint32_t *src = (const uint32_t *)(descs + req);
            uint32_t *dst = (uint32_t *)&sA;
            for (unsigned i = threadIdx.x; i < sizeof(RenderArgs) / 4; i += blockDim.x) dst[i] = src[i];
            __syncthreads();
            stage_frame<NV>(sA, s_tf, s_ch, s_runs, s_lv, s_nd);
            cur = req;
        }
        serve_item<NV, BPV, EC>(sA, sw & 0x3FFFFFFu, &s_next, s_tf, s_ch, s_runs, s_lv, s_nd);
        __threadfence();  // this item's pixels are visible device-wide before it is counted
        __syncthreads();  // sA, the LDS tables, s_seg and s_next are reused by the next segment
        if (threadIdx.x == 0) {
            // the request's last work item posts its completion to the host:
            // its pixels (and those of every other item, each fenced before
            // its count) are written before the flag
            const uint32_t c = atomicAdd(hdr->done + req, 1u) + 1u;
            if (c == serve_segments(sA.W, sA.H)) {
                __threadfence_system();
                hdr->flags[req] = hdr->seq;
            }
        }
    }
}

// Continuous admission.  Requests are appended one at a time to a ring of
// work items in mapped host memory (entry: request serial, slot << 26 |
// item); the host publishes them by raising the ring's tail.  A launch is
// open until one of its workgroups finds no unclaimed item: while open, its
// workgroups claim the next item (compare-and-swap on the device head,
// only while head < tail), so a request appended meanwhile is taken as
// workgroups free up, in arrival order, without a new launch.  The
// workgroup that finds the ring empty closes the launch (the device's
// closed generation, and a record of the launch and the head in host
// memory): the launch's workgroups leave after their current item, and the
// host starts a new launch for items published after the close.  No
// workgroup ever waits for the host.  Host memory is read with system-scope
// relaxed loads, which go to memory without invalidating the caches (the
// bricks stay in L2): the tail is read first, and the entry and the
// descriptor the host wrote before it only after the tail's value has
// arrived.  A request's last item resets its slot's count and posts the
// serial to the host.
struct RingCtl {
    uint32_t tail;  // items published (host: release store)
    uint32_t pad[63];
};
constexpr uint32_t kCloseRecords = 1024;  // host records of closed launches, by launch number

__device__ __forceinline__ uint32_t sys_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int NV, int BPV, int EC>
__global__ void __launch_bounds__(kRenderLanes) __attribute__((amdgpu_waves_per_eu(kRenderLanes / 256)))
    k_serve_ring(const RingCtl *ctl, const RenderArgs *descs, const uint2 *ring, uint32_t mask, uint32_t *head,
                 uint32_t *closed, unsigned long long *records, uint32_t launch, uint32_t *done, uint32_t *flags) {
    extern __shared__ float4 s_tf[];
    __shared__ RenderArgs sA;
    __shared__ ChanLds s_ch[NV];
    __shared__ uint32_t s_runs[NV * kMaxRuns];
    __shared__ LevLds s_lv[kMaxL];
    __shared__ NodeLds s_nd[kMaxD + 1];
    __shared__ uint2 s_item;
    __shared__ uint32_t s_ok, s_next;
    uint32_t cur = 0;  // serial of the staged request (serials start at 1)
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t ok = 0;
            // this launch (or a later one) closed: leave
            if ((int32_t)(__hip_atomic_load(closed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - launch) < 0) {
                uint32_t h = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (;;) {
                    const uint32_t t = sys_load(&ctl->tail);
                    if ((int32_t)(t - h) <= 0) {
                        // nothing unclaimed: close the launch
                        atomicMax(closed, launch);
                        __hip_atomic_store(records + (launch & (kCloseRecords - 1)),
                                           ((unsigned long long)launch << 32) | h, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                        break;
                    }
                    const uint32_t prev = atomicCAS(head, h, h + 1u);
                    if (prev == h) {
                        ok = 1;
                        break;
                    }
                    h = prev;  // another workgroup took h
                }
                if (ok) {
                    const uint32_t *e = (const uint32_t *)(ring + (h & mask));
                    s_item = make_uint2(sys_load(e), sys_load(e + 1));
                }
            }
            s_ok = ok;
            s_next = 0;
        }
        __syncthreads();
        if (!s_ok) break;
        const uint2 it = s_item;
        const uint32_t slot = it.y >> 26;
        if (it.x != cur) {
            const uint32_t *src = (const uint32_t *)(descs + slot);
            uint32_t *dst = (uint32_t *)&sA;
            for (unsigned i = threadIdx.x; i < sizeof(RenderArgs) / 4; i += blockDim.x) dst[i] = sys_load(src + i);
            __syncthreads();
            stage_frame<NV>(sA, s_tf, s_ch, s_runs, s_lv, s_nd);
            cur = it.x;
        }
        serve_item<NV, BPV, EC>(sA, it.y & 0x3FFFFFFu, &s_next, s_tf, s_ch, s_runs, s_lv, s_nd);
        __threadfence();
        __syncthreads();  // sA, the LDS tables, s_item and s_next are reused by the next item
        if (threadIdx.x == 0) {
            const uint32_t c = atomicAdd(done + slot, 1u) + 1u;
            if (c == serve_segments(sA.W, sA.H)) {
                // the slot's next request is published only after the host
                // has seen this serial, so the reset comes first
                atomicExch(done + slot, 0u);
                __threadfence_system();
                __hip_atomic_store(flags + slot, it.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
}

__global__ void k_zero(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__global__ void k_serve_reset(uint32_t *queue, uint32_t *done, uint32_t n) {
    if (threadIdx.x == 0) *queue = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) done[i] = 0;
}

ro_status build_render_args(ro_octree *tr, const ro_frame_desc *fd, float *rgba, RenderArgs &A);

}  // namespace ro

using namespace ro;

struct ro_server {
    ro_octree *tree;
    uint32_t max_req, max_tiles;
    int ncu;
    uint8_t *host;        // pinned host memory: 2 halves
    uint32_t *flags;      // mapped pinned host memory: [2][max_req] completion tickets
    uint32_t *flags_dev;  // its device address
    uint8_t *dev;         // caller-owned device buffer: 2 halves, 2 queue counters, [2][max_req] counts
    size_t half;          // bytes per half
    int cur;              // half the next prepare writes
    int ready;            // half prepared and not yet submitted (-1: none)
    int nv[2];            // channel template of each half's batch
    uint64_t ticket[2];   // last ticket submitted from each half
    uint64_t next_ticket;
    hipStream_t stream[2];
    hipEvent_t ev[2];
    hipGraph_t graph[2];
    hipGraphExec_t exec[2];
    // continuous admission: one mapped coherent host block holding RingCtl,
    // the completion flags, max_req descriptor slots and the ring
    uint8_t *rhost;
    uint8_t *rdev;          // its device address
    RingCtl *rctl;
    volatile uint32_t *rflags;
    RenderArgs *rdescs;
    uint2 *rring;
    uint32_t rcap;          // ring entries (a power of two)
    uint32_t rtail;         // items published
    uint32_t rserial[64];   // request in each slot (0: never used)
    uint32_t rfirst[64];    // its first ring index
    uint32_t next_serial;
    volatile unsigned long long *rrecords;  // close records: launch << 32 | head at the close
    int rnext;              // stream of the next launch
    uint32_t rlaunch;       // number of the latest launch (0: none yet)
    hipEvent_t rev[2];      // end of each stream's latest launch
    int rlast;              // stream of the latest launch
    hipStream_t rstream[2];
};

extern "C" ro_status ro_serve_work_items(int32_t width, int32_t height, uint32_t *items) {
    RO_CHECK(items && width > 0 && height > 0, RO_E_ARG, "bad argument");
    *items = serve_segments(width, height);
    return RO_OK;
}

static size_t serve_half_bytes(uint32_t max_req, uint32_t max_tiles) {
    size_t b = sizeof(ServeHeader) + (size_t)max_req * sizeof(RenderArgs) + 4 * (size_t)max_tiles;
    return (b + 4095) / 4096 * 4096;
}

static uint32_t ring_entries(uint32_t max_tiles) {
    uint32_t c = 1;
    while (c < max_tiles) c <<= 1;
    return c;
}

// host block: RingCtl, completion flags [64], close records, descriptor
// slots [max_req], ring [cap]
static size_t ring_off_records() { return sizeof(RingCtl) + 256; }
static size_t ring_off_descs() { return ring_off_records() + 8 * (size_t)kCloseRecords; }
static size_t ring_off_ring(uint32_t max_req) { return ring_off_descs() + (size_t)max_req * sizeof(RenderArgs); }
static size_t ring_host_bytes(uint32_t max_req, uint32_t cap) {
    return ring_off_ring(max_req) + (size_t)cap * sizeof(uint2);
}

// device head counter, closed launch and per-slot counts of continuous
// admission (512 bytes, zero at creation)
static inline uint32_t *ring_head(const ro_server *s) { return (uint32_t *)(s->dev + 2 * s->half + 1024); }
static inline uint32_t *ring_closed(const ro_server *s) { return (uint32_t *)(s->dev + 2 * s->half + 1028); }
static inline uint32_t *ring_done(const ro_server *s) { return (uint32_t *)(s->dev + 2 * s->half + 1280); }

static inline uint32_t *serve_queue(const ro_server *s, int h) {
    return (uint32_t *)(s->dev + 2 * s->half + 256 * (size_t)h);
}

// per-request finished work-item counts of half h (max_req <= 64 words)
static inline uint32_t *serve_done(const ro_server *s, int h) {
    return (uint32_t *)(s->dev + 2 * s->half + 512 + 256 * (size_t)h);
}

template <int NV, int BPV, int EC>
static hipError_t serve_attr1() {
    return hipFuncSetAttribute((const void *)k_serve<NV, BPV, EC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)render_lds_bytes(NV));
}

template <int NV, int BPV>
static hipError_t serve_attr() {
    hipError_t e = serve_attr1<NV, BPV, 0>();
    if (e == hipSuccess) e = serve_attr1<NV, BPV, 18>();
    if (e == hipSuccess) e = serve_attr1<NV, BPV, 34>();
    return e;
}

template <int BPV>
static hipError_t ring_attr() {
    hipError_t e = hipSuccess;
    for (const void *f : {(const void *)k_serve_ring<16, BPV, 0>, (const void *)k_serve_ring<16, BPV, 18>,
                          (const void *)k_serve_ring<16, BPV, 34>})
        if (e == hipSuccess)
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)render_lds_bytes(16));
    return e;
}

template <int BPV, int EC>
static void ring_launch_e(const ro_server *s, uint32_t launch, hipStream_t st) {
    const uint8_t *d = s->rdev;
    const RingCtl *ctl = (const RingCtl *)d;
    uint32_t *flags = (uint32_t *)(d + sizeof(RingCtl));
    unsigned long long *records = (unsigned long long *)(d + ring_off_records());
    const RenderArgs *descs = (const RenderArgs *)(d + ring_off_descs());
    const uint2 *ring = (const uint2 *)(d + ring_off_ring(s->max_req));
    hipLaunchKernelGGL((k_serve_ring<16, BPV, EC>), dim3(s->ncu), dim3(kRenderLanes), render_lds_bytes(16), st, ctl,
                       descs, ring, s->rcap - 1, ring_head(s), ring_closed(s), records, launch, ring_done(s),
                       flags);
}

static hipError_t ring_launch(const ro_server *s, uint32_t launch, hipStream_t st) {
    const int E = s->tree->cache->vol->g.E;
    const bool b1 = s->tree->cache->vol->g.bpv == 1;
    if (E == 34) b1 ? ring_launch_e<1, 34>(s, launch, st) : ring_launch_e<2, 34>(s, launch, st);
    else if (E == 18) b1 ? ring_launch_e<1, 18>(s, launch, st) : ring_launch_e<2, 18>(s, launch, st);
    else b1 ? ring_launch_e<1, 0>(s, launch, st) : ring_launch_e<2, 0>(s, launch, st);
    return hipGetLastError();
}

template <int NV, int BPV, int EC>
static void serve_launch_e(const ro_server *s, int h, hipStream_t st) {
    const uint8_t *d = s->dev + (size_t)h * s->half;
    const ServeHeader *dh = (const ServeHeader *)d;
    const RenderArgs *dd = (const RenderArgs *)(d + sizeof(ServeHeader));
    const uint32_t *dt = (const uint32_t *)(d + sizeof(ServeHeader) + (size_t)s->max_req * sizeof(RenderArgs));
    uint32_t *q = serve_queue(s, h);
    hipLaunchKernelGGL(k_serve_reset, dim3(1), dim3(64), 0, st, q, serve_done(s, h), s->max_req);
    hipLaunchKernelGGL((k_serve<NV, BPV, EC>), dim3(s->ncu), dim3(kRenderLanes), render_lds_bytes(NV), st, dh, dd, dt,
                       q);
}

// compile-time brick edge for 32^3 and 16^3 bricks (see the frame kernel)
template <int NV, int BPV>
static void serve_launch_t(const ro_server *s, int h, hipStream_t st) {
    const int E = s->tree->cache->vol->g.E;
    if (E == 34) serve_launch_e<NV, BPV, 34>(s, h, st);
    else if (E == 18) serve_launch_e<NV, BPV, 18>(s, h, st);
    else serve_launch_e<NV, BPV, 0>(s, h, st);
}

// Device work of one submission from half h: copy, queue reset, kernel.
static hipError_t serve_enqueue(const ro_server *s, int h, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(s->dev + (size_t)h * s->half, s->host + (size_t)h * s->half, s->half,
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    const bool b1 = s->tree->cache->vol->g.bpv == 1;
    switch (s->nv[h]) {
        case 4: b1 ? serve_launch_t<4, 1>(s, h, st) : serve_launch_t<4, 2>(s, h, st); break;
        case 8: b1 ? serve_launch_t<8, 1>(s, h, st) : serve_launch_t<8, 2>(s, h, st); break;
        default: b1 ? serve_launch_t<16, 1>(s, h, st) : serve_launch_t<16, 2>(s, h, st); break;
    }
    return hipGetLastError();
}

extern "C" ro_status ro_serve_query(uint32_t max_requests, uint32_t max_tiles, size_t *device_bytes) {
    RO_CHECK(device_bytes, RO_E_ARG, "null argument");
    *device_bytes = 2 * serve_half_bytes(max_requests, max_tiles) + 1536;
    return RO_OK;
}

extern "C" void ro_serve_destroy(ro_server *s) {
    if (!s) return;
    for (int h = 0; h < 2; ++h) {
        if (s->stream[h]) (void)hipStreamSynchronize(s->stream[h]);
        if (s->exec[h]) (void)hipGraphExecDestroy(s->exec[h]);
        if (s->graph[h]) (void)hipGraphDestroy(s->graph[h]);
        if (s->ev[h]) (void)hipEventDestroy(s->ev[h]);
        if (s->stream[h]) (void)hipStreamDestroy(s->stream[h]);
        if (s->rstream[h]) {
            (void)hipStreamSynchronize(s->rstream[h]);
            (void)hipStreamDestroy(s->rstream[h]);
        }
        if (s->rev[h]) (void)hipEventDestroy(s->rev[h]);
    }
    if (s->rhost) (void)hipHostFree(s->rhost);
    if (s->host) (void)hipHostFree(s->host);
    if (s->flags) (void)hipHostFree(s->flags);
    delete s;
}

extern "C" ro_status ro_serve_create(ro_octree *t, uint32_t max_requests, uint32_t max_tiles, void *device_buf,
                                     ro_server **out) {
    RO_CHECK(t && device_buf && out, RO_E_ARG, "null argument");
    RO_CHECK(((uintptr_t)device_buf & 255u) == 0, RO_E_ARG, "device buffer must be 256-byte aligned");
    RO_CHECK(max_requests >= 1 && max_requests <= 64, RO_E_ARG, "max_requests not in 1..64");
    RO_CHECK(max_tiles >= 1 && max_tiles <= (1u << 24), RO_E_ARG, "max_tiles not in 1..2^24");
    ro_server *s = new (std::nothrow) ro_server();
    RO_CHECK(s, RO_E_NOMEM, "out of host memory");
    s->tree = t;
    s->max_req = max_requests;
    s->max_tiles = max_tiles;
    s->half = serve_half_bytes(max_requests, max_tiles);
    s->dev = (uint8_t *)device_buf;
    s->ready = -1;
    s->nv[0] = s->nv[1] = 16;
    s->next_ticket = 1;
    hipError_t e = hipSuccess;
    int dev = 0;
    void *h = nullptr;
    const char *what = "server set-up";
    do {
        if ((e = hipGetDevice(&dev)) != hipSuccess) break;
        if ((e = hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) break;
        if ((e = hipHostMalloc(&h, 2 * s->half, hipHostMallocDefault)) != hipSuccess) {
            what = "hipHostMalloc";
            break;
        }
        s->host = (uint8_t *)h;
        memset(h, 0, 2 * s->half);
        void *f = nullptr;
        if ((e = hipHostMalloc(&f, 2 * sizeof(uint32_t) * max_requests, hipHostMallocMapped)) != hipSuccess) {
            what = "hipHostMalloc (mapped)";
            break;
        }
        s->flags = (uint32_t *)f;
        memset(f, 0, 2 * sizeof(uint32_t) * max_requests);
        void *fd = nullptr;
        if ((e = hipHostGetDevicePointer(&fd, f, 0)) != hipSuccess) {
            what = "hipHostGetDevicePointer";
            break;
        }
        s->flags_dev = (uint32_t *)fd;
        for (int k = 0; k < 2 && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&s->stream[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev[k], hipEventDisableTiming);
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->rstream[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s->rev[k], hipEventDisableTiming);
        }
        if (e != hipSuccess) break;
        // continuous admission: coherent mapped host block (the device reads
        // the tail, ring and descriptors while the host appends)
        s->rcap = ring_entries(max_tiles);
        void *rh = nullptr;
        const size_t rb = ring_host_bytes(max_requests, s->rcap);
        if ((e = hipHostMalloc(&rh, rb, hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess) {
            what = "hipHostMalloc (ring)";
            break;
        }
        s->rhost = (uint8_t *)rh;
        memset(rh, 0, rb);
        void *rd = nullptr;
        if ((e = hipHostGetDevicePointer(&rd, rh, 0)) != hipSuccess) {
            what = "hipHostGetDevicePointer (ring)";
            break;
        }
        s->rdev = (uint8_t *)rd;
        s->rctl = (RingCtl *)rh;
        s->rflags = (volatile uint32_t *)(s->rhost + sizeof(RingCtl));
        s->rrecords = (volatile unsigned long long *)(s->rhost + ring_off_records());
        s->rdescs = (RenderArgs *)(s->rhost + ring_off_descs());
        s->rring = (uint2 *)(s->rhost + ring_off_ring(max_requests));
        s->next_serial = 1;
        // the head, the generation and the slots' counts start at zero
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(128), 0, s->rstream[0], ring_head(s), 128u);
        if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s->rstream[0])) != hipSuccess) {
            what = "ring reset";
            break;
        }
        // dynamic LDS limits are set here: attribute calls are not made
        // while a stream is being captured
        if ((e = serve_attr<4, 1>()) != hipSuccess || (e = serve_attr<4, 2>()) != hipSuccess ||
            (e = serve_attr<8, 1>()) != hipSuccess || (e = serve_attr<8, 2>()) != hipSuccess ||
            (e = serve_attr<16, 1>()) != hipSuccess || (e = serve_attr<16, 2>()) != hipSuccess ||
            (e = ring_attr<1>()) != hipSuccess || (e = ring_attr<2>()) != hipSuccess)
            break;
    } while (0);
    if (e != hipSuccess) {
        ro_serve_destroy(s);
        return hip_fail(e, what);
    }
    *out = s;
    return RO_OK;
}

extern "C" ro_status ro_serve_prepare(ro_server *s, uint32_t n, const ro_frame_desc *fds, float *const *rgba,
                                      int32_t full_channels) {
    RO_CHECK(s && fds && rgba && n >= 1, RO_E_ARG, "null argument");
    RO_CHECK(n <= s->max_req, RO_E_CAPACITY, "%u requests exceed the server's %u", n, s->max_req);
    RO_CHECK(s->ready < 0, RO_E_STATE, "a prepared batch has not been submitted");
    uint32_t nt = 0;
    int maxvis = 1;
    for (uint32_t r = 0; r < n; ++r) {
        ro_status vs = validate_frame(s->tree, &fds[r], rgba[r]);
        if (vs) return vs;
        RO_CHECK(!(fds[r].flags & (RO_RENDER_AOV | RO_RENDER_BRICKS | RO_RENDER_NODES)), RO_E_ARG,
                 "diagnostic outputs are not served");
        RO_CHECK(!(fds[r].flags & (RO_RENDER_HOMOGENEOUS | RO_RENDER_CHANNEL_RATES | RO_RENDER_TRAVERSAL_DEPTH)),
                 RO_E_ARG, "homogeneous nodes, per-channel rates and traversal depths are not served");
        RO_CHECK(fds[r].width <= 65536 && fds[r].height <= 65536, RO_E_ARG, "viewport too large");
        const uint32_t ns = serve_segments(fds[r].width, fds[r].height);
        RO_CHECK(ns <= s->max_tiles - nt, RO_E_CAPACITY, "batch exceeds %u work items", s->max_tiles);
        nt += ns;
        maxvis = fds[r].n_vis > maxvis ? fds[r].n_vis : maxvis;
    }
    // the half being written was submitted two batches ago: wait for it
    const int h = s->cur;
    RO_HIP(hipEventSynchronize(s->ev[h]));
    uint8_t *base = s->host + (size_t)h * s->half;
    ServeHeader *hh = (ServeHeader *)base;
    RenderArgs *hd = (RenderArgs *)(base + sizeof(ServeHeader));
    uint32_t *ht = (uint32_t *)(base + sizeof(ServeHeader) + (size_t)s->max_req * sizeof(RenderArgs));
    nt = 0;
    for (uint32_t r = 0; r < n; ++r) {
        RenderArgs A;
        ro_status st = build_render_args(s->tree, &fds[r], rgba[r], A);
        if (st) {
            hh->n_tiles = 0;
            return st;
        }
        memcpy(&hd[r], &A, sizeof(A));
        // a request's segments are consecutive: a workgroup re-stages its
        // LDS tables only when it crosses into the next request
        const uint32_t ns = serve_segments(fds[r].width, fds[r].height);
        for (uint32_t i = 0; i < ns; ++i) ht[nt++] = (r << 26) | i;
    }
    hh->n_tiles = nt;
    hh->n_req = n;
    hh->seq = (uint32_t)s->next_ticket;  // the ticket the next submission assigns
    hh->done = serve_done(s, h);
    hh->flags = s->flags_dev + (size_t)h * s->max_req;
    s->nv[h] = full_channels ? 16 : (maxvis <= 4 ? 4 : (maxvis <= 8 ? 8 : 16));
    s->ready = h;
    return RO_OK;
}

extern "C" ro_status ro_serve_submit(ro_server *s, uint32_t flags, uint64_t *ticket) {
    RO_CHECK(s, RO_E_ARG, "null argument");
    RO_CHECK(s->ready >= 0, RO_E_STATE, "no prepared batch");
    const int h = s->ready;
    hipStream_t st = s->stream[h];
    if (flags & RO_SERVE_GRAPH) {
        RO_CHECK(s->nv[h] == 16, RO_E_ARG, "graph submission needs a batch prepared with full_channels");
        if (!s->exec[h]) {
            RO_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            hipError_t e = serve_enqueue(s, h, st);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(st, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(e != hipSuccess ? e : e2, "graph capture");
            }
            e = hipGraphInstantiate(&s->exec[h], g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                s->exec[h] = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
            s->graph[h] = g;
        }
        RO_HIP(hipGraphLaunch(s->exec[h], st));
    } else {
        RO_HIP(serve_enqueue(s, h, st));
    }
    RO_HIP(hipEventRecord(s->ev[h], st));
    s->ticket[h] = s->next_ticket++;
    if (ticket) *ticket = s->ticket[h];
    s->cur = h ^ 1;
    s->ready = -1;
    return RO_OK;
}

static ro_status serve_ticket_half(const ro_server *s, uint64_t ticket, int *h) {
    RO_CHECK(ticket >= 1 && ticket < s->next_ticket, RO_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    *h = -1;  // older than both halves' last submissions: finished
    for (int k = 0; k < 2; ++k)
        if (s->ticket[k] == ticket) *h = k;
    return RO_OK;
}

extern "C" ro_status ro_serve_poll(ro_server *s, uint64_t ticket, int32_t *done) {
    RO_CHECK(s && done, RO_E_ARG, "null argument");
    int h;
    ro_status st = serve_ticket_half(s, ticket, &h);
    if (st) return st;
    if (h < 0) {
        *done = 1;
        return RO_OK;
    }
    hipError_t e = hipEventQuery(s->ev[h]);
    if (e == hipErrorNotReady) {
        *done = 0;
        return RO_OK;
    }
    RO_HIP(e);
    *done = 1;
    return RO_OK;
}

extern "C" ro_status ro_serve_request_done(ro_server *s, uint64_t ticket, uint32_t r, int32_t *done) {
    RO_CHECK(s && done, RO_E_ARG, "null argument");
    int h;
    ro_status st = serve_ticket_half(s, ticket, &h);
    if (st) return st;
    RO_CHECK(r < s->max_req, RO_E_ARG, "request index %u out of range", r);
    if (h < 0) {
        *done = 1;
        return RO_OK;
    }
    const volatile uint32_t *f = s->flags + (size_t)h * s->max_req;
    *done = f[r] == (uint32_t)ticket ? 1 : 0;
    return RO_OK;
}

extern "C" ro_status ro_serve_wait(ro_server *s, uint64_t ticket) {
    RO_CHECK(s, RO_E_ARG, "null argument");
    int h;
    ro_status st = serve_ticket_half(s, ticket, &h);
    if (st) return st;
    if (h >= 0) RO_HIP(hipEventSynchronize(s->ev[h]));
    return RO_OK;
}

extern "C" ro_status ro_serve_launch(ro_server *s, uint32_t n, const ro_frame_desc *fds, float *const *rgba,
                                     uint64_t *ticket) {
    ro_status st = ro_serve_prepare(s, n, fds, rgba, 0);
    if (st) return st;
    return ro_serve_submit(s, 0, ticket);
}

// ---------------------------------------------------------------- continuous admission

// Starts a launch when published items may be left with no open launch to
// take them: none yet, the latest launch's close record says it closed
// before them, or the latest launch has ended (then the device head is
// read).  An open launch takes what is published while it runs.
static ro_status ring_kick(ro_server *s) {
    uint32_t h;
    if (s->rlaunch == 0) {
        h = 0;
    } else {
        const unsigned long long rec = s->rrecords[s->rlaunch & (kCloseRecords - 1)];
        if ((uint32_t)(rec >> 32) == s->rlaunch) {
            h = (uint32_t)rec;
        } else {
            const hipError_t q = hipEventQuery(s->rev[s->rlast]);
            if (q == hipErrorNotReady) return RO_OK;  // open and running
            RO_HIP(q);
            // ended without a record seen (overwritten): ask the device
            RO_HIP(hipMemcpyAsync(&h, ring_head(s), 4, hipMemcpyDeviceToHost, s->rstream[s->rlast]));
            RO_HIP(hipStreamSynchronize(s->rstream[s->rlast]));
        }
    }
    if ((int32_t)(s->rtail - h) <= 0) return RO_OK;  // nothing unclaimed
    const uint32_t launch = s->rlaunch + 1 == 0 ? 1 : s->rlaunch + 1;
    const int k = s->rnext;
    RO_HIP(ring_launch(s, launch, s->rstream[k]));
    RO_HIP(hipEventRecord(s->rev[k], s->rstream[k]));
    s->rlaunch = launch;
    s->rlast = k;
    s->rnext ^= 1;
    return RO_OK;
}

// The slot's request has finished (or the slot was never used).
static inline bool ring_slot_free(const ro_server *s, uint32_t j) {
    return s->rserial[j] == 0 || s->rflags[j] == s->rserial[j];
}

extern "C" ro_status ro_serve_enqueue(ro_server *s, const ro_frame_desc *fd, float *rgba, uint64_t *ticket) {
    RO_CHECK(s && fd && rgba, RO_E_ARG, "null argument");
    ro_status vs = validate_frame(s->tree, fd, rgba);
    if (vs) return vs;
    RO_CHECK(!(fd->flags & (RO_RENDER_AOV | RO_RENDER_BRICKS | RO_RENDER_NODES)), RO_E_ARG,
             "diagnostic outputs are not served");
    RO_CHECK(!(fd->flags & (RO_RENDER_HOMOGENEOUS | RO_RENDER_CHANNEL_RATES | RO_RENDER_TRAVERSAL_DEPTH)), RO_E_ARG,
             "homogeneous nodes, per-channel rates and traversal depths are not served");
    RO_CHECK(fd->width <= 65536 && fd->height <= 65536, RO_E_ARG, "viewport too large");
    const uint32_t n = serve_segments(fd->width, fd->height);
    RO_CHECK(n <= s->rcap, RO_E_CAPACITY, "a request of %u work items exceeds the ring of %u", n, s->rcap);
    // a free slot, and the oldest ring entry still owned by an unfinished request
    int slot = -1;
    uint32_t lowest = s->rtail;
    for (uint32_t j = 0; j < s->max_req; ++j) {
        if (ring_slot_free(s, j)) {
            if (slot < 0) slot = (int)j;
        } else if ((int32_t)(s->rfirst[j] - lowest) < 0) {
            lowest = s->rfirst[j];
        }
    }
    RO_CHECK(slot >= 0, RO_E_CAPACITY, "all %u request slots are in use", s->max_req);
    RO_CHECK(s->rtail + n - lowest <= s->rcap, RO_E_CAPACITY, "the ring has no room for %u work items", n);
    RenderArgs A;
    ro_status st = build_render_args(s->tree, fd, rgba, A);
    if (st) return st;
    const uint32_t serial = s->next_serial;
    memcpy(&s->rdescs[slot], &A, sizeof(A));
    for (uint32_t i = 0; i < n; ++i) {
        uint2 &e = s->rring[(s->rtail + i) & (s->rcap - 1)];
        e.x = serial;
        e.y = ((uint32_t)slot << 26) | i;
    }
    s->rserial[slot] = serial;
    s->rfirst[slot] = s->rtail;
    s->rtail += n;
    // descriptor and entries are written before the tail that publishes them
    __atomic_store_n(&s->rctl->tail, s->rtail, __ATOMIC_RELEASE);
    s->next_serial = serial + 1 == 0 ? 1 : serial + 1;
    if (ticket) *ticket = serial;
    return ring_kick(s);
}

extern "C" ro_status ro_serve_done(ro_server *s, uint64_t ticket, int32_t *done) {
    RO_CHECK(s && done, RO_E_ARG, "null argument");
    RO_CHECK(ticket >= 1 && ticket < s->next_serial, RO_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    *done = 1;  // a ticket no slot holds any more has finished
    for (uint32_t j = 0; j < s->max_req; ++j)
        if (s->rserial[j] == (uint32_t)ticket) *done = s->rflags[j] == (uint32_t)ticket ? 1 : 0;
    // polling drives progress: items published just as the latest launch
    // closed get a launch here
    return *done ? RO_OK : ring_kick(s);
}

extern "C" ro_status ro_serve_drain(ro_server *s) {
    RO_CHECK(s, RO_E_ARG, "null argument");
    for (;;) {
        for (int k = 0; k < 2; ++k) RO_HIP(hipStreamSynchronize(s->rstream[k]));
        bool open = false;
        for (uint32_t j = 0; j < s->max_req; ++j) open = open || !ring_slot_free(s, j);
        if (!open) return RO_OK;
        // every launch has ended with requests unfinished: their items were
        // published after the last close; start a launch for them
        const uint32_t before = s->rlaunch;
        ro_status st = ring_kick(s);
        if (st) return st;
        RO_CHECK(s->rlaunch != before, RO_E_STATE, "unfinished requests with no unclaimed work item");
    }
}
