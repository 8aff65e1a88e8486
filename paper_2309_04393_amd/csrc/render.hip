// Ray-guided mixed-resolution multi-channel ray casting over the residency
// octree (Sec. 6.1, Alg. 1; Sec. 6.2; Sec. 7 implementation notes).
//
// One lane per ray; persistent 768-lane workgroups (one per CU) whose waves
// take 8 x 8-pixel blocks from per-XCD queues.
// Sample positions and every integer decision derived from them (box, leaf,
// brick, level) are computed in FP64; interpolation, transfer functions and
// the channel mix in FP32; the compositing state in FP64.  Per lane, the
// state of the current (leaf, level) visit is cached: which channels are
// empty there, the slot each channel samples, and which channels miss their
// desired brick; misses are counted once per visit with the visit's sample
// count (one atomic per visit and channel).
//
// Every table a lane indexes with a lane-dependent value (channel
// parameters, zero-alpha runs, per-level brick grid and LOD thresholds,
// per-level node grid, transfer functions) is staged in LDS at workgroup
// start; kernel arguments are only read with uniform indices.
#include <math.h>
#include <string.h>

#include "render_core.h"

namespace ro {

// Workgroups of kRenderLanes lanes (768: 3 waves per SIMD, up to 168 VGPRs),
// one per CU: one copy of the frame's LDS tables plus the per-lane slot
// words.  The 16-channel instantiations for 16-bit 32^3 and 16^3 bricks
// without the options keep nothing in scratch; the other 16-channel ones up
// to 40 bytes per lane, three 8-channel ones 12.  1024 lanes (4 waves per
// SIMD, 128 VGPRs) spill more and measured 1-10 % slower, 512 lanes 35 %
// slower.

// Lanes refill only when the whole wave is idle: a wave then takes a whole
// new 8 x 8 block and its rays start together.  Refilling single lanes as
// their rays end keeps more lanes busy (91 % against 70 %) but spreads a
// wave's samples over different depths and cache lines, and measured 3.4x
// slower on the 16-channel 1080p frame; refilling from 16 idle lanes 1.5x
// slower.
#ifndef RO_MIN_IDLE
#define RO_MIN_IDLE 64
#endif

// Per-XCD block queues: blocks are dealt to them in chunks of RO_CHUNK
// consecutive blocks (16 chunks per queue at 1080p).  On the 16-channel
// 1080p frame chunks of 256 measured 0.6 % faster than 64, 16 0.7 % slower,
// 1024 as 256, and 4096 (one region per XCD) 4 % slower.
#ifndef RO_QUEUES
#define RO_QUEUES 8
#endif
#ifndef RO_CHUNK
#define RO_CHUNK 256
#endif

// Persistent grid (one workgroup per CU) whose waves take 8 x 8-pixel blocks
// from a device counter independently of each other, so a CU never waits
// for the slowest wave of a workgroup before taking new work.
template <int NV, int BPV, bool AOV, int EC, int EXT>
__global__ void __launch_bounds__(kRenderLanes) __attribute__((amdgpu_waves_per_eu(kRenderLanes / 256)))
    k_render(const RenderArgs A, uint32_t *counter, uint32_t n_blocks, uint32_t tiles_x) {
    extern __shared__ float4 s_tf[];  // [NV][kTfStride] tables, then [NV][kRenderLanes] slot words
    __shared__ ChanLds s_ch[NV];
    __shared__ uint32_t s_runs[NV * kMaxRuns];
    __shared__ LevLds s_lv[kMaxL];
    __shared__ NodeLds s_nd[kMaxD + 1];

    stage_frame<NV>(A, s_tf, s_ch, s_runs, s_lv, s_nd);

    BlockQueue q;
    q.counter = counter;
    q.n_blocks = n_blocks;
    q.offset = 0;
    q.tiles_x = tiles_x;
    q.n_queues = RO_QUEUES;
    q.chunk = RO_CHUNK;
    q.W = A.W;
    q.H = A.H;
    q.min_idle = RO_MIN_IDLE;
    uint32_t st[7] = {0, 0, 0, 0, 0, 0, 0};
    const LdsSlots sl{(uint32_t *)(s_tf + kTfStride * NV) + threadIdx.x, (uint32_t)kRenderLanes};
    render_rays<NV, BPV, AOV, EC, EC == 0, EXT>(A, q, s_tf, s_ch, s_runs, s_lv, s_nd, st, sl);
    if (A.stats) {
        // every lane of the workgroup is here: reduce over the wave, one atomic per wave
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            uint32_t v = st[j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if ((threadIdx.x & 63) == 0 && v) atomicAdd(&A.stats[j], (unsigned long long)v);
        }
    }
}

struct QueueLaunch {
    dim3 grid;
    uint32_t *counter;
    uint32_t n_blocks, tiles_x;
};

template <int NV, int BPV, bool AOV, int EC, int EXT = 0>
static hipError_t launch_one(const RenderArgs &A, const QueueLaunch &Q, hipStream_t s) {
    const size_t lds = render_lds_bytes(NV, (EXT & 1) != 0);
    hipError_t e = hipFuncSetAttribute((const void *)k_render<NV, BPV, AOV, EC, EXT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_render<NV, BPV, AOV, EC, EXT>), Q.grid, dim3(kRenderLanes), lds, s, A, Q.counter, Q.n_blocks,
                       Q.tiles_x);
    return hipGetLastError();
}

// Compile-time brick edges: 32^3 and 16^3 bricks with their halo (the AOV
// diagnostic output and the LOD-adaptive step take the generic kernel).
// Render-and-skip of homogeneous nodes (EXT bit 0) and per-channel sampling
// rates (EXT bit 1) have instantiations of their own, so the kernels that do
// not take them carry none of their code.
template <int NV, int BPV>
static hipError_t launch_nv(const RenderArgs &A, bool aov, const QueueLaunch &Q, hipStream_t s) {
    if (aov) return launch_one<NV, BPV, true, 0, 3>(A, Q, s);
    if (A.flags & RO_RENDER_ADAPTIVE_STEP) {
        if (A.flags & RO_RENDER_HOMOGENEOUS) return launch_one<NV, BPV, false, 0, 1>(A, Q, s);
        if (A.flags & RO_RENDER_CHANNEL_RATES) return launch_one<NV, BPV, false, 0, 2>(A, Q, s);
        return launch_one<NV, BPV, false, 0>(A, Q, s);
    }
    if (A.flags & RO_RENDER_HOMOGENEOUS) {
        if (A.E == 34) return launch_one<NV, BPV, false, 34, 1>(A, Q, s);
        if (A.E == 18) return launch_one<NV, BPV, false, 18, 1>(A, Q, s);
        return launch_one<NV, BPV, false, 0, 1>(A, Q, s);
    }
    if (A.E == 34) return launch_one<NV, BPV, false, 34>(A, Q, s);
    if (A.E == 18) return launch_one<NV, BPV, false, 18>(A, Q, s);
    return launch_one<NV, BPV, false, 0>(A, Q, s);
}

template <int BPV>
static hipError_t launch_bpv(const RenderArgs &A, bool aov, const QueueLaunch &Q, hipStream_t s) {
    if (A.nvis <= 1) return launch_nv<1, BPV>(A, aov, Q, s);
    if (A.nvis <= 2) return launch_nv<2, BPV>(A, aov, Q, s);
    if (A.nvis <= 4) return launch_nv<4, BPV>(A, aov, Q, s);
    if (A.nvis <= 8) return launch_nv<8, BPV>(A, aov, Q, s);
    return launch_nv<16, BPV>(A, aov, Q, s);
}

// Kernel arguments of one frame (validated by the caller).
ro_status build_render_args(ro_octree *tr, const ro_frame_desc *fd, float *rgba, RenderArgs &A) {
    const ro_cache *c = tr->cache;
    const VolGeo &g = c->vol->g;
    const TreeGeo &T = tr->t;
    memset(&A, 0, sizeof(A));
    for (int k = 0; k < 3; ++k) {
        A.dims[k] = g.dims[k];
        A.sp[k] = g.spacing[k];
        A.eye[k] = fd->eye[k];
        A.F[k] = fd->forward[k];
        A.R[k] = fd->right[k];
        A.U[k] = fd->up[k];
    }
    A.m = g.m;
    A.L = g.L;
    A.Blog = g.Blog;
    A.E = g.E;
    A.depth = T.depth;
    A.start_level = fd->start_level >= 0 ? fd->start_level : tr->desc.start_level;
    A.per_channel = g.per_channel;
    A.slot_stride = g.slot_stride;
    A.tx = fd->tx;
    A.ty = fd->ty;
    A.step = fd->step;
    A.proj = fd->projection;
    A.W = fd->width;
    A.H = fd->height;
    for (int l = 0; l < g.L; ++l) {
        A.lsh[l] = (uint32_t)g.lshift[l][0] | ((uint32_t)g.lshift[l][1] << 8) | ((uint32_t)g.lshift[l][2] << 16);
        A.loff[l] = g.loff[l];
        A.nbx[l] = (uint32_t)g.nb[l][0];
        A.nby[l] = (uint32_t)g.nb[l][1];
    }
    for (int d = 0; d <= T.depth; ++d) {
        A.nsh[d] = (uint32_t)T.nshift[d][0] | ((uint32_t)T.nshift[d][1] << 8) | ((uint32_t)T.nshift[d][2] << 16);
        A.nlg[d] = (uint32_t)T.nlog[d][0] | ((uint32_t)T.nlog[d][1] << 8) | ((uint32_t)T.nlog[d][2] << 16);
        A.noff[d] = T.noff[d];
    }
    // desired level thresholds: level l from the first sample k with
    // k * step >= D_l, D_l = s_l / (lod_bias * 2 ty / H)
    const double pix = 2.0 * fd->ty / fd->height;
    for (int l = 0; l < kMaxL; ++l) A.K[l] = kInvalid;
    A.K[0] = 0;
    for (int l = 1; l < g.L; ++l) {
        const double s_l = (double)(1 << g.lshift[l][0]) * g.spacing[0];
        if (fd->projection == RO_PROJ_ORTHO) {
            A.K[l] = fd->lod_bias * pix >= s_l ? 0u : kInvalid;
        } else {
            const double Dl = s_l / (fd->lod_bias * pix);
            const double q = ceil(Dl / fd->step);
            if (!(q < 4.0e9)) {
                A.K[l] = kInvalid;
                continue;
            }
            long long kk = (long long)q;
            while (kk > 0 && (double)(kk - 1) * fd->step >= Dl) --kk;
            while ((double)kk * fd->step < Dl) ++kk;
            A.K[l] = kk < 0xFFFFFFFFll ? (uint32_t)kk : kInvalid;
        }
    }
    // traversal depth from the step (Alg. 1 chooseTraversalDepth): for the
    // step of level l, the deepest node whose smallest world extent is at
    // least the distance between samples, f_l * step
    for (int l = 0; l < kMaxL; ++l) A.dd[l] = (uint32_t)T.depth;
    if ((fd->flags & RO_RENDER_TRAVERSAL_DEPTH) && (fd->flags & RO_RENDER_ADAPTIVE_STEP)) {
        for (int l = 0; l < g.L; ++l) {
            const double dist = (double)(1 << g.lshift[l][0]) * fd->step;
            int d = T.depth;
            while (d > 0) {
                double ext = INFINITY;
                for (int a = 0; a < 3; ++a) ext = fmin(ext, (double)(1ll << T.nshift[d][a]) * g.spacing[a]);
                if (ext >= dist) break;
                --d;
            }
            A.dd[l] = (uint32_t)d;
        }
    }
    A.nvis = fd->n_vis;
    A.ident = fd->n_vis == g.m && g.m % 4 == 0;
    for (int j = 0; j < fd->n_vis; ++j) A.ident = A.ident && fd->vis[j] == j;
    A.uni = 1;
    for (int j = 0; j < fd->n_vis; ++j) A.uni = A.uni && fd->lod_lo[j] == fd->lod_lo[0] && fd->lod_hi[j] == fd->lod_hi[0];
    // min_c clamp(l, lo_c, hi_c) = clamp(l, min_c lo_c, min_c hi_c)
    A.step_lo = A.step_hi = kMaxL;
    for (int j = 0; j < fd->n_vis; ++j) {
        A.step_lo = fd->lod_lo[j] < A.step_lo ? fd->lod_lo[j] : A.step_lo;
        A.step_hi = fd->lod_hi[j] < A.step_hi ? fd->lod_hi[j] : A.step_hi;
    }
    for (int j = 0; j < fd->n_vis; ++j) {
        A.vis[j] = fd->vis[j];
        A.lo[j] = fd->lod_lo[j];
        A.hi[j] = fd->lod_hi[j];
        A.W0[j] = fd->win_lo[j];
        A.W1[j] = fd->win_hi[j];
        A.w0[j] = (float)(fd->win_lo[j] / 256.0);
        A.iw[j] = (float)(256.0 / ((double)fd->win_hi[j] - (double)fd->win_lo[j]));
    }
    A.term = fd->term_alpha;
    A.frame = fd->frame;
    A.flags = fd->flags;
    A.slots = (const uint8_t *)c->b.slots;
    A.pt = c->b.page_table;
    A.cnt = c->b.counters;
    A.stamp = c->b.stamps;
    A.meta = tr->b.node_meta;
    A.mask = tr->b.node_mask;
    A.tf = (const float4 *)fd->tf_dev;
    A.rgba = rgba;
    A.aov = (fd->flags & RO_RENDER_AOV) ? fd->aov_dev : nullptr;
    A.reqb = (fd->flags & RO_RENDER_BRICKS) ? fd->bricks_dev : nullptr;
    A.nodes = (fd->flags & RO_RENDER_NODES) ? fd->nodes_dev : nullptr;
    A.stats = fd->stats_dev;
    return RO_OK;
}

ro_status render_device(ro_octree *tr, const ro_frame_desc *fd, float *rgba, hipStream_t s) {
    const VolGeo &g = tr->cache->vol->g;
    RenderArgs A;
    ro_status st = build_render_args(tr, fd, rgba, A);
    if (st) return st;
    int dev = 0, ncu = 0;
    RO_HIP(hipGetDevice(&dev));
    RO_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    QueueLaunch Q;
    const uint32_t tiles_x = (uint32_t)(fd->width + 31) / 32, tiles_y = (uint32_t)(fd->height + 31) / 32;
    Q.tiles_x = tiles_x;
    Q.n_blocks = tiles_x * tiles_y * 16;
    // the block counter is in the last 256 bytes of the octree's scratch
    // buffer (residency work items use the rest); cleared by a kernel, not a
    // memset
    Q.counter = (uint32_t *)((uint8_t *)tr->b.scratch + tr->scratch_bytes - 256);
    Q.grid = dim3((unsigned)(ncu > 0 ? ncu : 256));
    static_assert(RO_QUEUES * kQueueStride * 4 <= 256, "queue counters exceed the scratch tail");
    st = launch_fill_u32(Q.counter, (uint64_t)RO_QUEUES * kQueueStride, 0u, s);
    if (st) return st;
    // the diagnostic outputs (per-level reads, required bricks) take the AOV kernel
    const bool aov = (fd->flags & (RO_RENDER_AOV | RO_RENDER_BRICKS | RO_RENDER_NODES)) != 0;
    RO_HIP(g.bpv == 1 ? launch_bpv<1>(A, aov, Q, s) : launch_bpv<2>(A, aov, Q, s));
    return RO_OK;
}

}  // namespace ro
