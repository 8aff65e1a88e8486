// Per-ray core of the residency-octree ray caster, shared by the frame kernel
// (render.hip) and the multi-request serving kernel (serve.hip).
#pragma once

#include <math.h>

#include <type_traits>

#include "common.h"

namespace ro {

struct RenderArgs {
    // scalars
    int32_t dims[3];
    double sp[3];
    int32_t m, L, Blog, E, depth, start_level;
    uint32_t per_channel, slot_stride;
    double eye[3], F[3], R[3], U[3];
    double tx, ty, step;
    int32_t proj, W, H;
    int32_t nvis;
    float term;
    uint32_t frame, flags;
    int32_t ident;  // visible slot j shows channel j for every channel, and m % 4 == 0
    int32_t uni;    // every visible channel has the same level range (lo[0], hi[0])
    int32_t step_lo, step_hi;  // adaptive step: the finest desired level is clamped to these
    // uniform tables copied to LDS by the workgroup
    int32_t vis[kMaxC], lo[kMaxC], hi[kMaxC];
    uint32_t W0[kMaxC], W1[kMaxC];
    float w0[kMaxC], iw[kMaxC];
    uint32_t lsh[kMaxL];   // per level: packed log2 factors x | y << 8 | z << 16
    uint32_t loff[kMaxL];  // brick offset of the level inside a channel
    uint32_t nbx[kMaxL], nby[kMaxL];
    uint32_t K[kMaxL];     // level l is desired from sample index K[l] on
    uint32_t dd[kMaxL];    // traversal depth for the step of level l (the tree depth without the option)
    uint32_t nsh[kMaxD + 1];   // per tree level: packed log2 node edge
    uint32_t nlg[kMaxD + 1];   // per tree level: packed log2 node count
    uint32_t noff[kMaxD + 1];  // node offset of the level
    // device buffers
    const uint8_t *slots;
    const uint32_t *pt;
    uint32_t *cnt;
    uint32_t *stamp;
    const uint32_t *meta;
    const uint16_t *mask;
    const float4 *tf;
    float *rgba;
    uint32_t *aov;   // per-level reads (AOV kernel), or null
    uint32_t *reqb;  // required bricks per pixel, [H][W][1 + nvis] (AOV kernel), or null
    uint8_t *nodes;  // nodes whose metadata the frame reads, [n_nodes] (AOV kernel), or null
    unsigned long long *stats;
};

struct ChanLds {
    int c, lo, hi, nruns;
    float w0, iw;
    uint32_t ehi;     // one zero-opacity run starting at raw value 0: its last raw value, else ~0
    uint32_t single;  // same in every entry: every visible channel has such a run
};

struct LevLds {
    uint32_t sh;   // packed shifts (level factor + brick) per axis
    uint32_t raw;  // packed level factor shifts
    uint32_t loff, nbx, nbxy, K;
    uint32_t dd;   // decision depth when this level sets the step
};

struct NodeLds {
    uint32_t nsh, nlg, noff;
};

__device__ __forceinline__ uint32_t field(uint32_t p, int a) { return (p >> (8 * a)) & 255u; }

// A pointer into device memory, marked as such: accesses through it are
// global (not flat) memory operations also where the frame's arguments were
// read from LDS (the serve kernels), where the compiler cannot tell.  The
// address goes through an integer: a cast to the global address space and
// straight back would be folded away.
template <class T>
__device__ __forceinline__ T *gmem(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)reinterpret_cast<uintptr_t>(p);
}

// Zero-alpha runs of a channel's table as raw-value bounds (lo | hi << 16):
// the range [mn, mx] is empty iff some run has mn >= lo and mx <= hi.  Raw
// values are at most 65535, so runs whose lower bound exceeds that are
// dropped and upper bounds are clamped to 65535.  Bounds from the window
// (24.8 fixed point, den = W1 - W0):
// floor(255 (256 r - W0) / den) >= a  <=>  r >= ceil((255 W0 + a den) / 65280)
// ceil (255 (256 r - W0) / den) <= b  <=>  r <= floor((255 W0 + b den) / 65280)
__device__ inline int build_runs(const float4 *tf, uint32_t W0, uint32_t W1, uint32_t *runs) {
    int n = 0, e = 0;
    const uint64_t den = (uint64_t)W1 - (uint64_t)W0;
    while (e < 256) {
        if (tf[e].w != 0.0f) {
            ++e;
            continue;
        }
        const int a = e;
        while (e < 256 && tf[e].w == 0.0f) ++e;
        const int b = e - 1;
        uint64_t rlo = a == 0 ? 0 : (255ull * W0 + (uint64_t)a * den + 65279ull) / 65280ull;
        uint64_t rhi = b == 255 ? 65535ull : (255ull * W0 + (uint64_t)b * den) / 65280ull;
        if (rhi > 65535ull) rhi = 65535ull;
        if (rlo <= rhi && n < kMaxRuns) runs[n++] = (uint32_t)rlo | ((uint32_t)rhi << 16);
    }
    return n;
}

__device__ __forceinline__ bool range_empty(uint32_t mm, const uint32_t *runs, int nr) {
    const uint32_t mn = mm & 0xFFFFu, mx = mm >> 16;
    for (int r = 0; r < nr; ++r) {
        const uint32_t q = runs[r];
        if (mn >= (q & 0xFFFFu) && mx <= (q >> 16)) return true;
    }
    return false;
}

// A channel's transfer-function table in LDS: its 256 entries and a copy of
// the last, so the interpolation's upper entry needs no clamp.
constexpr int kTfStride = 257;

// Transfer function of a visible channel at raw value v: window, table
// position, linear interpolation of the LDS table (tf = the channel's
// entries; at the top end the weight of the copy is zero).
__device__ __forceinline__ void classify(float v, const ChanLds &ch, const float4 *tf, float &al, float &r, float &g,
                                         float &b) {
    float x = (v - ch.w0) * ch.iw;
    x = fminf(fmaxf(x, 0.0f), 1.0f);
    const float p = x * 255.0f;
    const int e = (int)p;  // 0 .. 255
    const float f = p - (float)e;
    const float4 ta = tf[e], tb = tf[e + 1];
    al = ta.w + (tb.w - ta.w) * f;
    r = ta.x + (tb.x - ta.x) * f;
    g = ta.y + (tb.y - ta.y) * f;
    b = ta.z + (tb.z - ta.z) * f;
}

// Two horizontally adjacent voxels (x, x + 1) in one load; the voxel grid
// is only 1- or 2-byte aligned, which global loads allow on this target.
template <int BPV>
__device__ __forceinline__ uint32_t vpair(const uint8_t *p) {
    if (BPV == 1) {
        uint16_t v;
        __builtin_memcpy(&v, p, 2);
        return v;
    }
    uint32_t v;
    __builtin_memcpy(&v, p, 4);
    return v;
}

template <int BPV>
__device__ __forceinline__ void unpack(uint32_t w, float v[2]) {
    if (BPV == 1) {
        v[0] = (float)(w & 0xFFu);
        v[1] = (float)((w >> 8) & 0xFFu);
    } else {
        v[0] = (float)(w & 0xFFFFu);
        v[1] = (float)(w >> 16);
    }
}

__device__ __forceinline__ uint32_t brick_dense(const LevLds &lv, uint32_t c, uint32_t per_channel, int bx,
                                                int by, int bz) {
    return c * per_channel + lv.loff + (uint32_t)bz * lv.nbxy + (uint32_t)by * lv.nbx + (uint32_t)bx;
}

__device__ __forceinline__ uint32_t node_at(const NodeLds &nd, int x, int y, int z) {
    return nd.noff + ((((uint32_t)z << field(nd.nlg, 1)) + (uint32_t)y) << field(nd.nlg, 0)) + (uint32_t)x;
}

// Lanes per workgroup of the render and serve kernels.
#ifndef RO_LANES
#define RO_LANES 768
#endif
#ifndef RO_GROUP
#define RO_GROUP 4
#endif
constexpr int kRenderLanes = RO_LANES;
// Serving work items: up to kSegBlocks 8 x 8-pixel blocks of one request.
constexpr uint32_t kSegBlocks = 96;

// A lane's span of a node that is homogeneous for every visible channel:
// the transparency of one taken sample, the transparency when the span
// began, and the constant mix's summed opacity and opacity-weighted colour.
struct HomLane {
    double tau, t0;
    float hsa, hsr, hsg, hsb;
};

// Dynamic LDS of a workgroup: NV transfer-function tables, then one slot
// word per lane and visible channel, then (kernels with render-and-skip)
// one HomLane per lane.
__host__ __device__ constexpr size_t render_lds_bytes(int nv, bool homog = false) {
    return (size_t)nv * kTfStride * 16 + (size_t)nv * kRenderLanes * 4 + (homog ? kRenderLanes * sizeof(HomLane) : 0);
}

// Slot of each visible channel for a lane's current visit, kept in LDS (one
// word per lane and channel, lane-minor so a wave's accesses are
// conflict-free) rather than in registers.
struct LdsSlots {
    uint32_t *p;      // this lane's first word
    uint32_t stride;  // lanes in the workgroup
    __device__ __forceinline__ uint32_t &operator[](int j) { return p[(uint32_t)j * stride]; }
};

// Pixel source of the stepping loop (first pixel of each lane, further
// pixels when lanes of the wave are idle).
//
// BlockQueue: waves take 8 x 8-pixel blocks from device counters (blocks of
// a 32 x 32 tile are consecutive, tiles in raster order).  With n_queues = 1
// one counter hands out the blocks in order.  With n_queues > 1 the blocks
// are dealt in chunks of `chunk` consecutive blocks, chunk c to queue
// c mod n_queues; a workgroup starts on queue (workgroup index mod
// n_queues), which with workgroups dealt to the XCDs in turn is its XCD's,
// and takes from the next queues once its own is used up.  The XCDs then
// work on separate neighbouring chunks (their L2s hold different lines)
// while all of them still sweep the image together (the Infinity Cache is
// shared).  Lanes whose ray ended take the next pixels of the wave's block,
// in lane order of a ballot of the idle lanes (prefix ranks), once at least
// min_idle lanes are idle.  Counter reads and block state are wave-uniform.
constexpr int kQueueStride = 8;  // words between queue counters (32 bytes)
struct BlockQueue {
    static constexpr bool kRefill = true;
    uint32_t *counter;  // n_queues counters kQueueStride words apart, zero at launch (device or LDS)
    uint32_t n_blocks;  // blocks this queue hands out: offset .. offset + n_blocks - 1
    uint32_t offset, tiles_x;
    uint32_t n_queues, chunk;
    int W, H;
    int min_idle;     // refill when at least this many lanes are idle
    uint32_t block;   // current block (wave-uniform)
    uint32_t used;    // its pixels handed out
    bool exhausted;
    uint32_t q, tried;  // current queue, queues found used up (wave-uniform)

    __device__ __forceinline__ uint32_t pop() {
        uint32_t b = n_blocks;
        if ((threadIdx.x & 63) == 0) {
            if (n_queues == 1) {
                b = atomicAdd(counter, 1u);
            } else {
                while (tried < n_queues) {
                    const uint32_t i = atomicAdd(counter + q * kQueueStride, 1u);
                    const uint64_t c = (uint64_t)(i / chunk) * n_queues + q;
                    const uint64_t bb = c * chunk + i % chunk;
                    if (bb < n_blocks) {
                        b = (uint32_t)bb;
                        break;
                    }
                    q = (q + 1) % n_queues;
                    ++tried;
                }
            }
        }
        q = (uint32_t)__shfl((int)q, 0, 64);
        tried = (uint32_t)__shfl((int)tried, 0, 64);
        return (uint32_t)__shfl((int)b, 0, 64);
    }
    __device__ __forceinline__ void pixel(uint32_t b, uint32_t i, int &x, int &y, bool &v) const {
        b += offset;
        const uint32_t t = b >> 4;
        x = (int)((t % tiles_x) * 32 + (b & 3u) * 8 + (i & 7u));
        y = (int)((t / tiles_x) * 32 + ((b >> 2) & 3u) * 8 + (i >> 3));
        v = x < W && y < H;
    }
    __device__ __forceinline__ bool more() const { return !exhausted; }
    __device__ __forceinline__ bool first(int &x, int &y, bool &v) {
        q = blockIdx.x % n_queues;
        tried = 0;
        block = pop();
        used = 64;
        exhausted = block >= n_blocks;
        if (exhausted) return false;
        pixel(block, threadIdx.x & 63, x, y, v);
        return true;
    }
    // want: ballot of the idle lanes; returns whether this lane got a pixel
    __device__ __forceinline__ bool refill(uint64_t want, int &x, int &y, bool &v) {
        if (exhausted || __popcll(want) < (unsigned)min_idle) return false;
        const uint32_t ln = threadIdx.x & 63;
        const bool me = (want >> ln) & 1ull;
        const uint32_t r = (uint32_t)__popcll(want & ((1ull << ln) - 1ull));
        const uint32_t n = (uint32_t)__popcll(want);
        const uint32_t left = 64 - used;
        bool got = false;
        if (me && r < left) {
            pixel(block, used + r, x, y, v);
            got = true;
        }
        if (n > left) {
            const uint32_t nb = pop();
            if (nb >= n_blocks) {
                exhausted = true;
                used = 64;
            } else {
                if (me && r >= left) {
                    pixel(nb, r - left, x, y, v);
                    got = true;
                }
                block = nb;
                used = n - left;
            }
        } else {
            used += n;
        }
        return got;
    }
};

// Slot bytes of a brick of edge e (halo included): rounded up to 256 bytes,
// as the cache lays out its slots.
__host__ __device__ constexpr size_t slot_bytes(int e, int bpv) {
    return ((size_t)e * e * e * bpv + 255) / 256 * 256;
}

// EC: the brick edge with halo known at compile time (0: read from A).  A
// constant edge turns the four gather offsets into instruction immediates.
// ADAPT: whether the LOD-adaptive step is compiled in; EXT: bit 0
// render-and-skip of nodes homogeneous for all channels, bit 1 per-channel
// sampling rates (frames that ask for them go to a kernel that has them).
template <int NV, int BPV, bool AOV, int EC, bool ADAPT, int EXT, class Source>
__device__ __forceinline__ void render_rays(const RenderArgs &A, Source &src, const float4 *s_tf,
                                            const ChanLds *s_ch, const uint32_t *s_runs, const LevLds *s_lv,
                                            const NodeLds *s_nd, uint32_t stats[7], LdsSlots slot) {
    constexpr bool HOMOG = (EXT & 1) != 0;
    constexpr bool RATES = ADAPT && (EXT & 2) != 0;
    const int nvis = A.nvis;
    const int D = A.depth;
    const int L = A.L;
    const int m = A.m;
    constexpr int kGroup = NV < RO_GROUP ? NV : RO_GROUP;  // channels whose loads are in flight together
    const double one_minus_term = 1.0 - (double)A.term;
    const uint32_t vismask = (nvis >= 32) ? 0xFFFFFFFFu : ((1u << nvis) - 1u);
    const int s0 = A.start_level;
    const bool noskip = (A.flags & RO_RENDER_NO_SKIP) != 0;
    const bool adaptive = ADAPT && (A.flags & RO_RENDER_ADAPTIVE_STEP) != 0;
    const bool homog = HOMOG && (A.flags & RO_RENDER_HOMOGENEOUS) != 0;
    // per-channel sampling rates (with the adaptive step): a channel takes part
    // only in samples k that are multiples of its own level's x factor
    const bool rates = RATES && adaptive && (A.flags & RO_RENDER_CHANNEL_RATES) != 0;
    // traversal depth from the step (with the adaptive step): emptiness and
    // homogeneity are decided at the node of depth dd of the step's level
    const bool tdepth = ADAPT && adaptive && (A.flags & RO_RENDER_TRAVERSAL_DEPTH) != 0;
    const NodeLds leafl = s_nd[D];
    const bool single = s_ch[0].single != 0;
    uint32_t st_samples = 0, st_reads = 0, st_miss = 0, st_visits = 0, st_nonempty = 0, st_iters = 0, st_hom = 0;

    // ---- per-ray state
    int px = 0, py = 0;
    bool has = false;  // the lane holds a ray (finished or not)
    double o[3] = {0, 0, 0}, d[3] = {0, 0, 0};
    double Cr = 0, Cg = 0, Cb = 0, Tr = 1.0;
    float *out = nullptr;
    bool done = true;
    long long k = 0, kend = -1, skip_to = 0;  // the lane is inside an empty node while k < skip_to
    int rpace = 0;  // adaptive step: log2 of the lane's last sampling distance (its pace while skipping)
    uint32_t cur_leaf = kInvalid;
    int cur_lod = -1, lod = 0;
    uint32_t emask = 0, missmask = 0;
    uint64_t lvpack = 0;
    uint32_t nvisit = 0;
    int lc[3] = {-1, -1, -1};  // L0 origin of the last visited leaf or skipped node (none yet)
    int lcd = 0;                // its depth: the nodes above it are known not to be skipped
    uint32_t last_key = kInvalid;  // (level, cell) of the last visit when uniform
    uint32_t have = 0;             // channels with a slot from the last visit
    uint32_t stamped = 0;          // with rates: channels whose current slot carries this frame's stamp
    uint64_t rpk = 0;              // with rates: each channel's rate shift in the current visit (4 bits)
    // render-and-skip: the lane composites a homogeneous span, one taken
    // sample per wave iteration, until skip_to (its state in LDS)
    bool hom_on = false;
    HomLane *hl = nullptr;
    if constexpr (HOMOG) hl = (HomLane *)((uint32_t *)(s_tf + kTfStride * NV) + NV * kRenderLanes) + threadIdx.x;

    // ray set-up in L0 voxel units, box interval, first sample index
    auto start = [&](int x, int y, bool valid) {
        px = x;
        py = y;
        has = true;
        const double a = (double)(2 * px + 1 - A.W) / (double)A.W;
        const double b = (double)(A.H - 2 * py - 1) / (double)A.H;
        double ow[3], dw[3];
        if (A.proj == RO_PROJ_ORTHO) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                ow[q] = A.eye[q] + a * A.tx * A.R[q] + b * A.ty * A.U[q];
                dw[q] = A.F[q];
            }
        } else {
            double n = 0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                ow[q] = A.eye[q];
                dw[q] = A.F[q] + a * A.tx * A.R[q] + b * A.ty * A.U[q];
                n += dw[q] * dw[q];
            }
            n = sqrt(n);
#pragma unroll
            for (int q = 0; q < 3; ++q) dw[q] = dw[q] / n;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            o[q] = ow[q] / A.sp[q];
            d[q] = dw[q] / A.sp[q];
        }
        Cr = Cg = Cb = 0.0;
        Tr = 1.0;
        out = valid ? gmem(A.rgba) + ((size_t)py * A.W + px) * 4 : nullptr;
        if (AOV && A.reqb && valid) {
            // required bricks: the count, then each channel's last desired brick
            uint32_t *rb = A.reqb + ((size_t)py * A.W + px) * (1 + nvis);
            rb[0] = 0;
            for (int j = 0; j < nvis; ++j) rb[1 + j] = kInvalid;
        }
        double t0 = -INFINITY, t1 = INFINITY;
        bool hit = true;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (d[q] == 0.0) {
                if (o[q] < 0.0 || o[q] >= (double)A.dims[q]) hit = false;
                continue;
            }
            double u = (0.0 - o[q]) / d[q], v = ((double)A.dims[q] - o[q]) / d[q];
            if (u > v) {
                const double sw = u;
                u = v;
                v = sw;
            }
            t0 = fmax(t0, u);
            t1 = fmin(t1, v);
        }
        done = !valid || !hit || t0 > t1;
        k = done ? 0 : (long long)floor(t0 / A.step) - 1;
        if (k < 0) k = 0;
        kend = done ? -1 : (long long)ceil(t1 / A.step) + 1;
        skip_to = 0;
        cur_leaf = kInvalid;
        cur_lod = -1;
        lod = 0;
        rpace = 0;
        while (lod + 1 < L && (unsigned long long)k >= s_lv[lod + 1].K) ++lod;
        emask = missmask = 0;
        lvpack = 0;
        nvisit = 0;
        lc[0] = lc[1] = lc[2] = -1;
        lcd = 0;
        last_key = kInvalid;
        have = 0;
        stamped = 0;
        hom_on = false;
#pragma unroll
        for (int j = 0; j < NV; ++j) slot[j] = kInvalid;
    };

    auto flush = [&]() {
        if (missmask && nvisit) {
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                if (j < nvis && ((missmask >> j) & 1u)) {
                    const ChanLds ch = s_ch[j];
                    const int ls = min(max(cur_lod, ch.lo), ch.hi);
                    const LevLds lv = s_lv[ls];
                    const int bx = lc[0] >> field(lv.sh, 0), by = lc[1] >> field(lv.sh, 1),
                              bz = lc[2] >> field(lv.sh, 2);
                    atomicAdd(&gmem(A.cnt)[brick_dense(lv, (uint32_t)ch.c, A.per_channel, bx, by, bz)], nvisit);
                    st_miss += nvisit;
                }
            }
        }
        nvisit = 0;
    };

    auto finish = [&]() {
        flush();
        if (out) {
            out[0] = (float)Cr;
            out[1] = (float)Cg;
            out[2] = (float)Cb;
            out[3] = (float)(1.0 - Tr);
        }
        has = false;
    };

    {
        int x = 0, y = 0;
        bool v = false;
        if (src.first(x, y, v)) start(x, y, v);
    }

    // Wave-coherent stepping: lanes advance one sample per iteration, so the
    // lanes of a wave (neighbouring pixels) sample at the same t and share
    // cache lines; a lane inside an empty node idles, and the wave jumps
    // ahead only by the smallest skip over its active lanes.  The samples a
    // lane evaluates are exactly those it would evaluate on its own.  A lane
    // whose ray ended writes its pixel and, with a refilling source, starts
    // the next pixel of the wave's block.
    while (true) {
        if (has && (done || k > kend)) finish();
        if (Source::kRefill) {
            const uint64_t want = __ballot(!has);
            if (want) {
                int x = 0, y = 0;
                bool v = false;
                if (src.refill(want, x, y, v)) start(x, y, v);
            }
        }
        const bool active = has && !done && k <= kend;
        const long long gap = skip_to - k;
        uint32_t need = !active ? 0xFFFFFFFFu : (gap > 0 ? (gap < 0x7FFFFFFFll ? (uint32_t)gap : 0x7FFFFFFFu) : 0u);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) need = min(need, (uint32_t)__shfl_xor((int)need, o, 64));
        if (need == 0xFFFFFFFFu) {
            // no lane is stepping: the wave ends once no lane holds a ray and
            // the source has nothing more (rays that just ended retire above)
            if (!__any(has) && !src.more()) break;
            continue;
        }
        if (need > 0) {
            // every active lane is in an empty node or a homogeneous span:
            // the wave jumps; a lane in a span composites the span's samples
            // it passes, one transparency factor each (a few instructions
            // per sample, all lanes at once)
            if constexpr (HOMOG) {
                if (active && hom_on) {
                    const long long rr = ADAPT ? (1ll << rpace) : 1;
                    const long long m = ((long long)need + rr - 1) / rr;
                    const double tau = hl->tau;
                    bool term = false;
                    long long i = 0;
                    while (i < m && !term) {
                        Tr *= tau;
                        ++i;
                        term = Tr <= one_minus_term;
                    }
                    st_samples += (uint32_t)i;
                    st_hom += (uint32_t)i;
                    k += i * rr;
                    if (term || k >= skip_to) {
                        const double sc = (hl->t0 - Tr) / (double)hl->hsa;
                        Cr += sc * (double)hl->hsr;
                        Cg += sc * (double)hl->hsg;
                        Cb += sc * (double)hl->hsb;
                        hom_on = false;
                        done = term;
                    }
                    continue;
                }
            }
            k += need;
            continue;
        }
        ++st_iters;  // a stepping iteration of the wave (lane busy or idle)
        if (!active) continue;
        if constexpr (HOMOG) {
            if (hom_on) {
                // the next taken sample of the span: one transparency factor,
                // as sample by sample (early termination falls on the same
                // sample); the colour is summed in closed form at the end
                Tr *= hl->tau;
                ++st_samples;
                ++st_hom;
                const bool term = Tr <= one_minus_term;
                k += ADAPT ? (1ll << rpace) : 1;
                if (term || k >= skip_to) {
                    const double sc = (hl->t0 - Tr) / (double)hl->hsa;
                    Cr += sc * (double)hl->hsr;
                    Cg += sc * (double)hl->hsg;
                    Cb += sc * (double)hl->hsb;
                    hom_on = false;
                    done = term;
                }
                continue;
            }
        }
        if (k < skip_to) {
            // a skipping lane keeps the pace of the sampling lanes (one base
            // step, or the band's distance with the adaptive step) so the
            // wave's lanes stay at neighbouring depths
            k = ADAPT ? min(skip_to, k + (1ll << rpace)) : k + 1;
            continue;
        }
        const double t = (double)k * A.step;
        double u[3];
        bool inside = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u[a] = o[a] + t * d[a];
            inside = inside && (u[a] >= 0.0) && (u[a] < (double)A.dims[a]);
        }
        if (!inside) {
            ++k;
            continue;
        }
        const int iu[3] = {(int)u[0], (int)u[1], (int)u[2]};
        while (lod + 1 < L && (unsigned long long)k >= s_lv[lod + 1].K) ++lod;
        // LOD-adaptive step: the finest desired level over the visible
        // channels sets the sampling distance, r = its x factor; only samples
        // with k a multiple of r are evaluated
        int rsh = 0, dend = D;
        if (adaptive) {
            const LevLds slv = s_lv[min(max(lod, A.step_lo), A.step_hi)];
            rsh = (int)field(slv.raw, 0);
            if (tdepth) dend = (int)slv.dd;
            rpace = rsh;
            const long long rm = (1ll << rsh) - 1;
            if (k & rm) {
                skip_to = (k | rm) + 1;
                continue;
            }
        }
        const uint32_t leaf = node_at(leafl, iu[0] >> field(leafl.nsh, 0), iu[1] >> field(leafl.nsh, 1),
                                      iu[2] >> field(leafl.nsh, 2));
        if (leaf != cur_leaf || lod != cur_lod) {
            flush();
            // with a traversal depth the decision node depends on the level too
            if (leaf != cur_leaf || (tdepth && lod != cur_lod)) {
                // Descend from the start level and skip the first node that
                // is empty for every visible channel (the leaf included).
                // Every ancestor of a visited leaf is non-empty, so levels
                // whose node also holds the last visited leaf are known
                // non-empty and the test starts below them (the same node
                // is skipped either way).  With HOMOG the first node in which
                // every visible channel is empty or holds one value (and one
                // holds a value) is rendered from those values and skipped
                // (Alg. 1 renderAndSkipNode, Sec. 6.1: homogeneous for all
                // channels): its samples are composited and the ray goes on
                // past the node.  Ancestors of a visited leaf are never such
                // nodes either (metadata nest, so their descendants would be),
                // and the ancestors of a skipped node were tested and found
                // not to be skipped: the shared levels above the last visited
                // leaf or skipped node are not tested again.
                int d0 = noskip ? dend : min(s0, dend);
                if (lc[0] >= 0 && !noskip && !tdepth) {
                    while (d0 < lcd) {
                        const uint32_t sh = s_nd[d0].nsh;
                        if (((iu[0] ^ lc[0]) >> field(sh, 0)) | ((iu[1] ^ lc[1]) >> field(sh, 1)) |
                            ((iu[2] ^ lc[2]) >> field(sh, 2)))
                            break;
                        ++d0;
                    }
                }
                bool skipped = false;
                long long rs_end = 0;   // render-and-skip: the first sample past the node or the volume,
                uint32_t rs_node = 0;   // the node,
                uint32_t rs_mask = 0;   // its homogeneous channels (none: no such node)
                for (int dl = d0; dl <= dend; ++dl) {
                    const NodeLds nd = s_nd[dl];
                    const uint32_t node = node_at(nd, iu[0] >> field(nd.nsh, 0), iu[1] >> field(nd.nsh, 1),
                                                  iu[2] >> field(nd.nsh, 2));
                    // the node's metadata, kGroup channels per batch of loads
                    uint32_t em = 0, hm = 0;
                    const uint32_t *nm = gmem(A.meta) + (size_t)node * m;
                    if (AOV && A.nodes) A.nodes[node] = 1;
#pragma unroll
                    for (int g = 0; g < NV; g += kGroup) {
                        if (g >= nvis) break;
                        uint32_t mm[kGroup];
                        if (kGroup == 4 && A.ident) {
                            // channels g..g+3 are one aligned 16-byte load
                            const uint4 v = *(const uint4 *)(nm + g);
                            mm[0] = v.x;
                            mm[kGroup > 1 ? 1 : 0] = v.y;
                            mm[kGroup > 2 ? 2 : 0] = v.z;
                            mm[kGroup > 3 ? 3 : 0] = v.w;
                        } else {
#pragma unroll
                            for (int jj = 0; jj < kGroup; ++jj) mm[jj] = g + jj < nvis ? nm[s_ch[g + jj].c] : 0u;
                        }
                        if (single) {
                            // one zero run [0, ehi] per channel: empty iff the maximum is within it
#pragma unroll
                            for (int jj = 0; jj < kGroup; ++jj) {
                                const int j = g + jj;
                                if (j < nvis && (mm[jj] >> 16) <= s_ch[j].ehi) em |= 1u << j;
                            }
                        } else {
#pragma unroll
                            for (int jj = 0; jj < kGroup; ++jj) {
                                const int j = g + jj;
                                if (j < nvis && range_empty(mm[jj], s_runs + j * kMaxRuns, s_ch[j].nruns)) em |= 1u << j;
                            }
                        }
                        if (homog) {
#pragma unroll
                            for (int jj = 0; jj < kGroup; ++jj) {
                                const int j = g + jj;
                                if (j < nvis && (mm[jj] & 0xFFFFu) == (mm[jj] >> 16)) hm |= 1u << j;
                            }
                        }
                        asm volatile("" ::: "memory");
                    }
                    hm &= ~em;
                    if (dl == dend) emask = em;
                    const bool all_empty = em == vismask;
                    const bool rskip = homog && hm && (em | hm) == vismask;
                    // (without skipping, empty nodes are stepped through;
                    // render-and-skip changes the image, so it stays on)
                    if ((all_empty && !noskip) || rskip) {
                        // exit of the node (and, for render-and-skip, of the
                        // volume: a node may reach past it, and void samples
                        // are not composited)
                        double te = INFINITY;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            if (d[a] == 0.0) continue;
                            const int sh = (int)field(nd.nsh, a);
                            const double lo_a = (double)((iu[a] >> sh) << sh);
                            const double bound = d[a] > 0.0 ? lo_a + (double)(1 << sh) : lo_a;
                            te = fmin(te, (bound - o[a]) / d[a]);
                            if (!all_empty) te = fmin(te, ((d[a] > 0.0 ? (double)A.dims[a] : 0.0) - o[a]) / d[a]);
                        }
                        // samples before kb lie a whole step inside; kb itself
                        // is inside when the sampling path's own position test
                        // (same arithmetic) puts it in the node and the volume
                        const long long kb = (long long)floor(te / A.step);
                        bool in = kb > k;
                        if (in) {
                            const double tk = (double)kb * A.step;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                const double ua = o[a] + tk * d[a];
                                in = in && ua >= 0.0 && ua < (double)A.dims[a] &&
                                     ((((int)ua) ^ iu[a]) >> field(nd.nsh, a)) == 0;
                            }
                        }
                        const long long kx = in ? kb + 1 : kb;  // first sample that may lie outside
#pragma unroll
                        for (int a = 0; a < 3; ++a) lc[a] = (iu[a] >> field(nd.nsh, a)) << field(nd.nsh, a);
                        lcd = dl;
                        if (all_empty) {
                            skip_to = kx > k + 1 ? kx : k + 1;
                            ++k;
                            skipped = true;
                        } else if constexpr (HOMOG) {
                            // render-and-skip: composited after the descent
                            rs_end = kx;
                            rs_node = node;
                            rs_mask = hm;
                        }
                        break;
                    }
                }
                if constexpr (HOMOG) {
                    if (rs_mask) {
                        // The constant mix of the homogeneous channels (in
                        // visible-channel order, as sampled values mix) for the
                        // taken samples k, k + r, .. of the span: up to the
                        // node's exit, the volume's exit (the node may reach
                        // beyond the volume, whose samples are void) and, with
                        // the adaptive step, the next level threshold (r may
                        // change there).  The lane composites them one per
                        // wave iteration from here on, without gathers, then
                        // goes on past the node.
                        float hp = 1.0f, hsa = 0.0f, hsr = 0.0f, hsg = 0.0f, hsb = 0.0f;
                        const uint32_t *rm = gmem(A.meta) + (size_t)rs_node * m;
                        for (int j = 0; j < nvis; ++j) {
                            if (!((rs_mask >> j) & 1u)) continue;
                            const ChanLds ch = s_ch[j];
                            float al, r, gg, bb;
                            classify((float)(rm[ch.c] & 0xFFFFu), ch, s_tf + j * kTfStride, al, r, gg, bb);
                            hp *= 1.0f - al;
                            hsa += al;
                            hsr += al * r;
                            hsg += al * gg;
                            hsb += al * bb;
                        }
                        // samples before rs_end lie in the node and the
                        // volume; those from the next level threshold on are
                        // not taken
                        long long end = rs_end;
                        if (adaptive && lod + 1 < L && (long long)s_lv[lod + 1].K < end) end = s_lv[lod + 1].K;
                        const long long rr = 1ll << rsh;
                        long long n = (end - k + rr - 1) / rr;
                        if (n < 1) n = 1;
                        skip_to = k + n * rr;
                        if (hsa > 0.0f) {
                            double tau = (double)hp;
                            for (int q = 0; q < rsh; ++q) tau *= tau;
                            hl->tau = tau;
                            hl->t0 = Tr;
                            hl->hsa = hsa;
                            hl->hsr = hsr;
                            hl->hsg = hsg;
                            hl->hsb = hsb;
                            hom_on = true;
                        } else {
                            // nothing to composite: the span is skipped
                            st_samples += (uint32_t)n;
                            st_hom += (uint32_t)n;
                            ++k;
                        }
                        skipped = true;
                    }
                }
                if (skipped) {
                    cur_leaf = kInvalid;
                    continue;
                }
                cur_leaf = leaf;
#pragma unroll
                for (int a = 0; a < 3; ++a) lc[a] = (iu[a] >> field(leafl.nsh, a)) << field(leafl.nsh, a);
                lcd = D;
            }
            cur_lod = lod;
            ++st_visits;
            missmask = 0;
            lvpack = 0;
            if (rates) {
                // the rate of each channel's clamped desired level (fixed within a visit)
                rpk = 0;
                for (int j = 0; j < nvis; ++j) {
                    const ChanLds ch = s_ch[j];
                    rpk |= (uint64_t)field(s_lv[min(max(lod, ch.lo), ch.hi)].raw, 0) << (4 * j);
                }
            }
            // Residency masks of the leaf give each channel the level it
            // samples (finest resident at or above the desired one).
            const uint16_t *lm = gmem(A.mask) + (size_t)leaf * m;
            uint32_t look = 0;  // channels with a resident brick to look up
            bool all_at = false;  // every non-empty channel resident at the common desired level
            int lsu = 0;
            if (NV >= 4 && A.ident && A.uni) {
                // one desired level for every channel: AND the masks of all
                // channels (two per word) and test its bit
                lsu = min(max(lod, A.lo[0]), A.hi[0]);
                uint32_t andm = 0xFFFFFFFFu;
#pragma unroll
                for (int g = 0; g < NV; g += 4) {
                    if (g >= nvis) break;
                    const uint2 v = *(const uint2 *)(lm + g);
                    andm &= v.x & v.y;
                }
                andm &= andm >> 16;
                all_at = ((andm >> lsu) & 1u) != 0;
            }
            if (all_at) {
                look = vismask & ~emask;
                lvpack = 0;
#pragma unroll
                for (int j = 0; j < NV; ++j)
                    if ((look >> j) & 1u) lvpack |= (uint64_t)lsu << (4 * j);
            } else {
#pragma unroll
                for (int g = 0; g < NV; g += kGroup) {
                    if (g >= nvis) break;
                    uint32_t mk[kGroup];
                    if (kGroup == 4 && A.ident) {
                        const uint2 v = *(const uint2 *)(lm + g);
                        mk[0] = v.x & 0xFFFFu;
                        mk[kGroup > 1 ? 1 : 0] = v.x >> 16;
                        mk[kGroup > 2 ? 2 : 0] = v.y & 0xFFFFu;
                        mk[kGroup > 3 ? 3 : 0] = v.y >> 16;
                    } else {
#pragma unroll
                        for (int jj = 0; jj < kGroup; ++jj) mk[jj] = g + jj < nvis ? (uint32_t)lm[s_ch[g + jj].c] : 0u;
                    }
#pragma unroll
                    for (int jj = 0; jj < kGroup; ++jj) {
                        const int j = g + jj;
                        if (j < nvis && !((emask >> j) & 1u)) {
                            const ChanLds ch = s_ch[j];
                            const int ls = min(max(lod, ch.lo), ch.hi);
                            const uint32_t mj = mk[jj] >> ls;
                            if (!(mj & 1u)) missmask |= 1u << j;
                            if (mj) {
                                lvpack |= (uint64_t)(ls + __builtin_ctz(mj)) << (4 * j);
                                look |= 1u << j;
                            }
                        }
                    }
                }
            }
            // When every looked-up channel samples one level, its bricks are
            // the same grid cell in each channel: if that cell and level are
            // those of the previous visit, the slots found then still hold
            // (the page table does not change during a frame).
            uint32_t key = kInvalid;
            if (look) {
                int lu0 = lsu;
                bool uniform = true;
                if (!all_at) {
                    lu0 = (int)((lvpack >> (4 * __builtin_ctz(look))) & 15u);
#pragma unroll
                    for (int j = 0; j < NV; ++j)
                        if (((look >> j) & 1u) && (int)((lvpack >> (4 * j)) & 15u) != lu0) uniform = false;
                }
                if (uniform) {
                    const LevLds lv = s_lv[lu0];
                    key = brick_dense(lv, 0u, 0u, iu[0] >> field(lv.sh, 0), iu[1] >> field(lv.sh, 1),
                                      iu[2] >> field(lv.sh, 2)) |
                          ((uint32_t)lu0 << 28);
                }
            }
            const uint32_t reuse = (key != kInvalid && key == last_key) ? have : 0u;
            uint32_t nhave = reuse & look;
            // channels whose slot changes: looked up anew, or no longer sampled
            if ((look & ~reuse) | (have & ~look)) {
                nhave = 0;
#pragma unroll
                for (int g = 0; g < NV; g += kGroup) {
                    if (g >= nvis) break;
                    uint32_t ns[kGroup];
#pragma unroll
                    for (int jj = 0; jj < kGroup; ++jj) {
                        const int j = g + jj;
                        ns[jj] = kInvalid;
                        if ((look >> j) & 1u) {
                            if ((reuse >> j) & 1u) {
                                ns[jj] = slot[j];
                            } else {
                                const int lu = (int)((lvpack >> (4 * j)) & 15u);
                                const LevLds lv = s_lv[lu];
                                ns[jj] = gmem(A.pt)[brick_dense(lv, (uint32_t)s_ch[j].c, A.per_channel,
                                                          iu[0] >> field(lv.sh, 0), iu[1] >> field(lv.sh, 1),
                                                          iu[2] >> field(lv.sh, 2))];
                            }
                        }
                    }
#pragma unroll
                    for (int jj = 0; jj < kGroup; ++jj) {
                        const int j = g + jj;
                        if (j >= nvis) break;
                        if (ns[jj] == kInvalid) {
                            lvpack &= ~((uint64_t)15u << (4 * j));
                        } else {
                            nhave |= 1u << j;
                            if (ns[jj] != slot[j]) {
                                // with rates the stamp waits for a sample the channel takes part in
                                if (rates) stamped &= ~(1u << j);
                                else gmem(A.stamp)[ns[jj]] = A.frame;
                            }
                        }
                        slot[j] = ns[jj];
                    }
                    asm volatile("" ::: "memory");
                }
            }
            have = nhave;
            last_key = key;
        }
        ++st_samples;
        float prod = 1.0f, sa = 0.0f, sr = 0.0f, sg = 0.0f, sbl = 0.0f;
        // channels taking part in this sample (all of them without rates)
        uint32_t part = vismask;
        if (rates) {
            part = 0;
            for (int j = 0; j < nvis; ++j) {
                const int rs = (int)((rpk >> (4 * j)) & 15u);
                if (!(k & ((1ll << rs) - 1))) part |= 1u << j;
            }
            // misses and stamps per sample (a visit's samples differ in which
            // channels take part)
            uint32_t mp = missmask & part;
            while (mp) {
                const int j = __builtin_ctz(mp);
                mp &= mp - 1u;
                const ChanLds ch = s_ch[j];
                const LevLds lv = s_lv[min(max(lod, ch.lo), ch.hi)];
                atomicAdd(&gmem(A.cnt)[brick_dense(lv, (uint32_t)ch.c, A.per_channel, iu[0] >> field(lv.sh, 0),
                                             iu[1] >> field(lv.sh, 1), iu[2] >> field(lv.sh, 2))],
                          1u);
                ++st_miss;
            }
            uint32_t sp = have & part & ~stamped;
            while (sp) {
                const int j = __builtin_ctz(sp);
                sp &= sp - 1u;
                gmem(A.stamp)[slot[j]] = A.frame;
            }
            stamped |= have & part;
        } else {
            ++nvisit;
        }
        if (AOV && A.reqb) {
            // Bricks required per pixel: the desired brick of each channel not
            // empty here that takes part in the sample (a leaf lies in one
            // brick per level).  Along a ray the desired level never decreases
            // and a brick's samples are one interval, so each required brick is
            // one run of equal keys: count the changes.
            uint32_t *rb = A.reqb + ((size_t)py * A.W + px) * (1 + nvis);
            for (int j = 0; j < nvis; ++j) {
                if (((emask >> j) & 1u) || !((part >> j) & 1u)) continue;
                const ChanLds ch = s_ch[j];
                const LevLds lv = s_lv[min(max(lod, ch.lo), ch.hi)];
                const uint32_t key = brick_dense(lv, 0u, 0u, iu[0] >> field(lv.sh, 0), iu[1] >> field(lv.sh, 1),
                                                 iu[2] >> field(lv.sh, 2));
                if (rb[1 + j] != key) {
                    rb[1 + j] = key;
                    rb[0] += 1;
                }
            }
        }
        st_nonempty += __popc(vismask & ~emask & part);
        st_reads += __popc(have & part);  // the channels gathered below (those with a slot)
        // ---- sample every visible channel
        // In-brick coordinates depend only on the level a channel samples
        // (bricks of one level share their grid), so they are computed once
        // per distinct level of the sample.  Channels are gathered in groups
        // of kGroup: the group's loads are all issued before any of them is
        // used, and two horizontally adjacent voxels come in one load.
        int lprev = -1;
        uint32_t idx = 0;
        float fr0 = 0.0f, fr1 = 0.0f, fr2 = 0.0f;
        const uint32_t E = EC ? (uint32_t)EC : (uint32_t)A.E;
        const size_t stride = EC ? slot_bytes(EC, BPV) : (size_t)A.slot_stride;
        // in-brick voxel index and fractions of the sample at level lu
        auto in_brick = [&](int lu) {
            const LevLds lv = s_lv[lu];
            uint32_t i0[3];
            float fr[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int sft = (int)field(lv.raw, a);
                const double ul = ldexp(u[a], -sft);
                const int bo = (iu[a] >> field(lv.sh, a)) << A.Blog;
                const double q = ul + 0.5 - (double)bo;
                const int qi = (int)q;
                i0[a] = (uint32_t)qi;
                fr[a] = (float)(q - (double)qi);
            }
            idx = (i0[2] * E + i0[1]) * E + i0[0];
            fr0 = fr[0];
            fr1 = fr[1];
            fr2 = fr[2];
            lprev = lu;
        };
        // Gather, interpolate, classify and mix every channel with a slot.
        // With UNI every such channel reads the visit's one level, whose
        // coordinates are computed before the loop, so the FP64 position is
        // not live across the channels.
        auto sample_channels = [&](auto uni_c) {
            constexpr bool UNI = decltype(uni_c)::value;
            // the channel count and the slot pool (the same in every lane:
            // kernel arguments, or the workgroup's staged request) as scalar
            // values of this sample: the group tests stay scalar compares and
            // the pool address stays in registers instead of being hoisted
            // out of the ray loop
            // (the builtin returns int: each half is taken back to uint32_t
            // before widening, so the low half is not sign-extended)
            int nvs = __builtin_amdgcn_readfirstlane(nvis);
            const uint64_t pa = reinterpret_cast<uint64_t>(A.slots);
            const uint32_t phi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(pa >> 32));
            const uint32_t plo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)pa);
            uint64_t pv = ((uint64_t)phi << 32) | (uint64_t)plo;
            asm volatile("" : "+s"(nvs), "+s"(pv));
            const uint8_t *pool = (const uint8_t *)(const __attribute__((address_space(1))) uint8_t *)pv;
#pragma unroll
        for (int g = 0; g < NV; g += kGroup) {
            if (g >= nvs) break;
            uint32_t w[kGroup][4];
            float fq[kGroup][3];
            bool ok[kGroup];
#pragma unroll
            for (int jj = 0; jj < kGroup; ++jj) {
                const int j = g + jj;
                // the slot words of channels past nvis stay invalid
                ok[jj] = slot[j] != kInvalid;
                if (rates) ok[jj] = ok[jj] && ((part >> j) & 1u);
                if constexpr (!UNI) {
                    const int lu = (int)((lvpack >> (4 * j)) & 15u);
                    if (ok[jj] && lu != lprev) in_brick(lu);
                }
                fq[jj][0] = fr0;
                fq[jj][1] = fr1;
                fq[jj][2] = fr2;
                // a channel without a slot reads offset 0 of slot 0 (always
                // inside the pool) and its result is discarded
                const uint8_t *base = pool + (ok[jj] ? (size_t)slot[j] * stride + (size_t)idx * BPV : 0);
                w[jj][0] = vpair<BPV>(base);
                w[jj][1] = vpair<BPV>(base + (size_t)E * BPV);
                w[jj][2] = vpair<BPV>(base + (size_t)E * E * BPV);
                w[jj][3] = vpair<BPV>(base + (size_t)(E * E + E) * BPV);
            }
#pragma unroll
            for (int jj = 0; jj < kGroup; ++jj) {
                const int j = g + jj;
                if (!ok[jj]) continue;
                const float f0 = fq[jj][0], f1 = fq[jj][1], f2 = fq[jj][2];
                float v00[2], v10[2], v01[2], v11[2];
                unpack<BPV>(w[jj][0], v00);
                unpack<BPV>(w[jj][1], v10);
                unpack<BPV>(w[jj][2], v01);
                unpack<BPV>(w[jj][3], v11);
                const float c00 = v00[0] + (v00[1] - v00[0]) * f0;
                const float c10 = v10[0] + (v10[1] - v10[0]) * f0;
                const float c01 = v01[0] + (v01[1] - v01[0]) * f0;
                const float c11 = v11[0] + (v11[1] - v11[0]) * f0;
                const float e0 = c00 + (c10 - c00) * f1;
                const float e1 = c01 + (c11 - c01) * f1;
                const float v = e0 + (e1 - e0) * f2;
                float al, r, gg, bb;
                classify(v, s_ch[j], s_tf + j * kTfStride, al, r, gg, bb);
                if (rates) {
                    // the channel stands for r_c base steps: transparency
                    // (1 - alpha)^r_c, colour weight r_c alpha
                    const int rs = (int)((rpk >> (4 * j)) & 15u);
                    float tr = 1.0f - al;
                    for (int q = 0; q < rs; ++q) tr *= tr;
                    const float w = (float)(1 << rs) * al;
                    prod *= tr;
                    sa += w;
                    sr += w * r;
                    sg += w * gg;
                    sbl += w * bb;
                } else {
                    prod *= 1.0f - al;
                    sa += al;
                    sr += al * r;
                    sg += al * gg;
                    sbl += al * bb;
                }
                if (AOV && A.aov) A.aov[((size_t)py * A.W + px) * L + (int)((lvpack >> (4 * j)) & 15u)] += 1;
            }
            // the next group's loads are issued after this group is used:
            // bounds the registers held by loads in flight
            asm volatile("" ::: "memory");
        }
        };
        if (last_key != kInvalid) {
            // one level for every channel with a slot (the visit's lookup key)
            in_brick((int)(last_key >> 28));
            sample_channels(std::true_type{});
        } else {
            sample_channels(std::false_type{});
        }
        if (sa > 0.0f) {
            if (rsh == 0 || rates) {
                const float as = 1.0f - prod;
                const float sc = as / sa;
                Cr += Tr * (double)(sr * sc);
                Cg += Tr * (double)(sg * sc);
                Cb += Tr * (double)(sbl * sc);
                Tr *= 1.0 - (double)as;
            } else {
                // opacity correction for a sample standing for r base steps:
                // transparency prod^r, colour scaled with the opacity
                double tr = (double)prod;
                for (int q = 0; q < rsh; ++q) tr *= tr;
                const double sc = (1.0 - tr) / (double)sa;
                Cr += Tr * ((double)sr * sc);
                Cg += Tr * ((double)sg * sc);
                Cb += Tr * ((double)sbl * sc);
                Tr *= tr;
            }
            if (Tr <= one_minus_term) done = true;
        }
        // the next sample: with the adaptive step the next multiple of r (the
        // level only grows along the ray, so no grid point lies in between);
        // each lane keeps its own phase and samples on every iteration
        k += 1ll << rsh;
    }
    stats[0] = st_samples;
    stats[1] = st_reads;
    stats[2] = st_miss;
    stats[3] = st_visits;
    stats[4] = st_nonempty;
    stats[5] = st_iters;
    stats[6] = st_hom;
}

// Workgroup set-up: stage the frame's transfer functions, zero-alpha runs,
// channel parameters, per-level brick tables and per-level node tables in
// LDS.  Ends with a workgroup barrier.
template <int NV>
__device__ __forceinline__ void stage_frame(const RenderArgs &A, float4 *s_tf, ChanLds *s_ch, uint32_t *s_runs,
                                            LevLds *s_lv, NodeLds *s_nd) {
    const int nvis = A.nvis;
    for (int i = threadIdx.x; i < nvis * kTfStride; i += blockDim.x) {
        const int t = i / kTfStride, e = i - t * kTfStride;
        s_tf[i] = A.tf[t * 256 + (e < 256 ? e : 255)];
    }
    const unsigned t = threadIdx.x;
    if (t < (unsigned)A.L) {
        LevLds lv;
        lv.raw = A.lsh[t];
        lv.sh = lv.raw + (uint32_t)A.Blog * 0x010101u;
        lv.loff = A.loff[t];
        lv.nbx = A.nbx[t];
        lv.nbxy = A.nbx[t] * A.nby[t];
        lv.K = A.K[t];
        lv.dd = A.dd[t];
        s_lv[t] = lv;
    }
    if (t >= 64 && t < 64u + (unsigned)A.depth + 1u) {
        const unsigned dl = t - 64;
        NodeLds nd;
        nd.nsh = A.nsh[dl];
        nd.nlg = A.nlg[dl];
        nd.noff = A.noff[dl];
        s_nd[dl] = nd;
    }
    __syncthreads();
    if (t < (unsigned)nvis) {
        ChanLds ch;
        ch.c = A.vis[t];
        ch.lo = A.lo[t];
        ch.hi = A.hi[t];
        ch.w0 = A.w0[t];
        ch.iw = A.iw[t];
        ch.nruns = build_runs(s_tf + t * kTfStride, A.W0[t], A.W1[t], s_runs + t * kMaxRuns);
        const uint32_t r0 = s_runs[t * kMaxRuns];
        ch.ehi = (ch.nruns == 1 && (r0 & 0xFFFFu) == 0) ? (r0 >> 16) : 0xFFFFFFFFu;
        ch.single = 0;
        s_ch[t] = ch;
    }
    __syncthreads();
    if (t < (unsigned)nvis) {
        uint32_t all = 1;
        for (int j = 0; j < nvis; ++j) all &= s_ch[j].ehi != 0xFFFFFFFFu ? 1u : 0u;
        s_ch[t].single = all;
    }
    __syncthreads();

}

}  // namespace ro
