// Streaming kernels: request compaction, usage readback, LRU slot
// selection, page-table update and brick scatter (Sec. 4: requests copied to
// the CPU under a global limit; Sec. 5.3: slot selection with LRU eviction).
#include <string.h>

#include <mutex>

#include "common.h"

namespace ro {

// ------------------------------------------------------------------- fills

template <typename T>
__global__ void k_fill(T *__restrict__ p, uint64_t n, T v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

template <typename T>
static ro_status fill(T *p, uint64_t n, T v, hipStream_t s) {
    if (n == 0) return RO_OK;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    RO_HIP(hipGetLastError());
    return RO_OK;
}

ro_status launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) { return fill(p, n, v, s); }
ro_status launch_fill_u16(uint16_t *p, uint64_t n, uint16_t v, hipStream_t s) { return fill(p, n, v, s); }
ro_status launch_fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s) { return fill(p, n, v, s); }

// ------------------------------------------------------ block-level helpers

// Exclusive prefix sum over the block (blockDim.x == 256, 4 waves of 64):
// wave-level via ballot-free shuffles, then across waves through LDS.
__device__ inline uint32_t block_excl_scan_256(uint32_t v, uint32_t *lds4, uint32_t *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds4[wid] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t t = lds4[w];
        if (w < wid) base += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// ------------------------------------------------------ request compaction

// Per block of 1024 counters: number of nonzero counters and the sum of all.
__global__ void __launch_bounds__(256) k_req_count(const uint32_t *__restrict__ cnt, uint64_t n,
                                                   uint32_t *__restrict__ blk,
                                                   unsigned long long *__restrict__ total) {
    __shared__ uint32_t lds[4];
    uint64_t base = (uint64_t)blockIdx.x * 1024 + threadIdx.x * 4;
    uint32_t nz = 0;
    unsigned long long sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint64_t i = base + k;
        if (i < n) {
            uint32_t v = cnt[i];
            nz += v != 0;
            sum += v;
        }
    }
    uint32_t tot;
    block_excl_scan_256(nz, lds, &tot);
    // wave-reduce the sums, one atomic per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if ((threadIdx.x & 63) == 0 && sum) atomicAdd(total, sum);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

// Exclusive scan of nblk block counts by one block; writes offsets and the
// grand total at offs[nblk].
__global__ void __launch_bounds__(256) k_scan_blocks(const uint32_t *__restrict__ blk, uint32_t nblk,
                                                     uint32_t *__restrict__ offs) {
    __shared__ uint32_t lds[4];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nblk; b0 += 256) {
        uint32_t i = b0 + threadIdx.x;
        uint32_t v = i < nblk ? blk[i] : 0;
        uint32_t tot;
        uint32_t e = block_excl_scan_256(v, lds, &tot);
        if (i < nblk) offs[i] = carry + e;
        carry += tot;
    }
    if (threadIdx.x == 0) offs[nblk] = carry;
}

// Writes the ID and count of every nonzero counter at its ascending rank r
// (out_ids[r], out_vals[r], only for r < lim) and clears every nonzero
// counter, whatever its rank.
__global__ void __launch_bounds__(256) k_req_write(uint32_t *__restrict__ cnt, uint64_t n,
                                                   const uint32_t *__restrict__ offs, VolGeo g,
                                                   uint32_t *__restrict__ out_ids, uint32_t *__restrict__ out_vals,
                                                   uint32_t lim) {
    __shared__ uint32_t lds[4];
    uint64_t base = (uint64_t)blockIdx.x * 1024 + threadIdx.x * 4;
    uint32_t v[4], nz = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint64_t i = base + k;
        v[k] = i < n ? cnt[i] : 0;
        nz += v[k] != 0;
    }
    uint32_t tot;
    uint32_t r = offs[blockIdx.x] + block_excl_scan_256(nz, lds, &tot);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (v[k]) {
            if (r < lim) {
                out_ids[r] = dense_to_id(g, (uint32_t)(base + k));
                out_vals[r] = v[k];
            }
            cnt[base + k] = 0;
            ++r;
        }
    }
}

ro_status read_requests_device(ro_cache *c, uint32_t cap, uint32_t *ids, uint32_t *counts,
                               uint32_t *n_unique, uint64_t *total, hipStream_t s) {
    return compact_dense(c, c->b.counters, cap, ids, counts, n_unique, total, s);
}

// Work space of one compaction of n entries: nblk = ceil(n / 1024) block
// counts, nblk + 1 offsets, the 64-bit sum, and lim output IDs and values.
size_t compact_scratch_bytes(uint64_t n, uint32_t lim) {
    const uint64_t nblk = (n + 1023) / 1024;
    return 256 + (((2 * nblk + 1) * 4 + 255) / 256) * 256 + 2 * (((uint64_t)lim * 4 + 255) / 256) * 256;
}

// Compaction of the dense per-brick array arr (g.total entries) in the work
// space ws (compact_scratch_bytes(g.total, lim) bytes, 256-byte aligned):
// copies the first min(cap, lim) (ID, value) pairs in ascending ID order to
// the host, with the distinct count and the sum, and clears the array.
// Clears its counters with a fill kernel (no memset).  Synchronises.
ro_status compact_dense_ws(const VolGeo &g, uint32_t *arr, uint8_t *ws, uint32_t lim, uint32_t cap, uint32_t *ids,
                           uint32_t *counts, uint32_t *n_unique, uint64_t *total, hipStream_t s) {
    const uint32_t nblk = (uint32_t)((g.total + 1023) / 1024);
    unsigned long long *tot = (unsigned long long *)ws;
    uint32_t *blk = (uint32_t *)(ws + 256);
    uint32_t *offs = blk + nblk;
    uint32_t *out_ids = (uint32_t *)(ws + 256 + (((2 * (uint64_t)nblk + 1) * 4 + 255) / 256) * 256);
    uint32_t *out_vals = out_ids + (((uint64_t)lim * 4 + 255) / 256) * 64;
    ro_status st = launch_fill_u32((uint32_t *)tot, 2, 0u, s);
    if (st) return st;
    hipLaunchKernelGGL(k_req_count, dim3(nblk), dim3(256), 0, s, arr, g.total, blk, tot);
    RO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(256), 0, s, blk, nblk, offs);
    RO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_req_write, dim3(nblk), dim3(256), 0, s, arr, g.total, offs, g, out_ids, out_vals, lim);
    RO_HIP(hipGetLastError());
    uint32_t nu = 0;
    unsigned long long t = 0;
    RO_HIP(hipMemcpyAsync(&nu, offs + nblk, 4, hipMemcpyDeviceToHost, s));
    RO_HIP(hipMemcpyAsync(&t, tot, 8, hipMemcpyDeviceToHost, s));
    RO_HIP(hipStreamSynchronize(s));
    uint32_t k = nu < cap ? nu : cap;
    k = k < lim ? k : lim;
    if (k) {
        RO_HIP(hipMemcpyAsync(ids, out_ids, 4 * (size_t)k, hipMemcpyDeviceToHost, s));
        RO_HIP(hipMemcpyAsync(counts, out_vals, 4 * (size_t)k, hipMemcpyDeviceToHost, s));
        RO_HIP(hipStreamSynchronize(s));
    }
    *n_unique = nu;
    *total = t;
    return RO_OK;
}

// Compaction in the cache's own scratch buffer (room for every brick).
ro_status compact_dense(ro_cache *c, uint32_t *arr, uint32_t cap, uint32_t *ids, uint32_t *counts,
                        uint32_t *n_unique, uint64_t *total, hipStream_t s) {
    const VolGeo &g = c->vol->g;
    return compact_dense_ws(g, arr, (uint8_t *)c->b.scratch + c->sc.compact, (uint32_t)g.total, cap, ids, counts,
                            n_unique, total, s);
}

// ------------------------------------- request readback without allocation

// Fixed work space of ro_read_requests_noalloc: room for the compaction of
// up to kNoAllocMaxBricks counters returning up to kNoAllocMaxPairs pairs.
// One copy per GPU, held until the process ends; every call on a GPU uses
// that GPU's copy, so calls that overlap on one GPU race.
constexpr uint64_t kNoAllocMaxBricks = 1ull << 26;
constexpr uint32_t kNoAllocMaxPairs = RO_NOALLOC_MAX_PAIRS;
constexpr size_t kNoAllocBytes = 256 + (((2 * (kNoAllocMaxBricks / 1024) + 1) * 4 + 255) / 256) * 256 +
                                 2 * (((size_t)kNoAllocMaxPairs * 4 + 255) / 256) * 256;

}  // namespace ro

static __device__ __align__(256) uint8_t scratch[ro::kNoAllocBytes];

namespace ro {

// Device address of this GPU's copy of `scratch` (the host-side name is not
// a device address): taken once per device with that device current.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static ro_status noalloc_scratch(uint8_t **out) {
    int dev = -1;
    RO_HIP(hipGetDevice(&dev));
    RO_CHECK(dev >= 0 && dev < kMaxDevices, RO_E_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        RO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        RO_CHECK(p != nullptr, RO_E_DEVICE, "no device address for the fixed work space");
        g_scratch_ptr[dev] = p;
    }
    *out = (uint8_t *)g_scratch_ptr[dev];
    return RO_OK;
}

ro_status read_requests_noalloc_device(ro_cache *c, uint32_t cap, uint32_t *ids, uint32_t *counts,
                                       uint32_t *n_unique, uint64_t *total, hipStream_t s) {
    const VolGeo &g = c->vol->g;
    RO_CHECK(g.total <= kNoAllocMaxBricks, RO_E_CAPACITY,
             "volume has %llu bricks; the fixed work space holds counters of at most %llu",
             (unsigned long long)g.total, (unsigned long long)kNoAllocMaxBricks);
    RO_CHECK(cap <= kNoAllocMaxPairs, RO_E_CAPACITY, "cap %u exceeds the fixed work space's %u pairs", cap,
             kNoAllocMaxPairs);
    uint8_t *ws = nullptr;
    ro_status st = noalloc_scratch(&ws);
    if (st) return st;
    return compact_dense_ws(g, c->b.counters, ws, kNoAllocMaxPairs, cap, ids, counts, n_unique, total, s);
}

// -------------------------------------------------------- usage readback

__global__ void __launch_bounds__(256) k_use_count(const uint32_t *__restrict__ stamp,
                                                   const uint32_t *__restrict__ slot_brick, uint32_t n,
                                                   uint32_t f, uint32_t *__restrict__ blk) {
    __shared__ uint32_t lds[4];
    uint32_t base = blockIdx.x * 1024 + threadIdx.x * 4, nz = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) nz += (base + k < n) && stamp[base + k] == f && slot_brick[base + k] != kInvalid;
    uint32_t tot;
    block_excl_scan_256(nz, lds, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_use_write(const uint32_t *__restrict__ stamp,
                                                   const uint32_t *__restrict__ slot_brick, uint32_t n,
                                                   uint32_t f, const uint32_t *__restrict__ offs,
                                                   uint32_t *__restrict__ out) {
    __shared__ uint32_t lds[4];
    uint32_t base = blockIdx.x * 1024 + threadIdx.x * 4, nz = 0;
    bool hit[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        hit[k] = (base + k < n) && stamp[base + k] == f && slot_brick[base + k] != kInvalid;
        nz += hit[k];
    }
    uint32_t tot;
    uint32_t r = offs[blockIdx.x] + block_excl_scan_256(nz, lds, &tot);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (hit[k]) out[r++] = base + k;
}

ro_status read_usage_device(ro_cache *c, uint32_t frame, uint32_t cap, uint32_t *slots,
                            uint32_t *n_out, hipStream_t s) {
    uint8_t *sc = (uint8_t *)c->b.scratch;
    uint32_t S = c->desc.n_slots;
    uint32_t nblk = (S + 1023) / 1024;
    // the request-compaction block arrays are large enough: total >= 1 brick
    // per slot is not guaranteed, so use the candidate-key area when needed
    uint32_t *blk = (uint32_t *)(sc + c->sc.keys);  // n_slots * 8 bytes >= 2 * nblk + 1 words
    uint32_t *offs = blk + nblk + 1;
    uint32_t *out = (uint32_t *)(sc + c->sc.outpairs);
    hipLaunchKernelGGL(k_use_count, dim3(nblk), dim3(256), 0, s, c->b.stamps, c->b.slot_brick, S, frame, blk);
    RO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(256), 0, s, blk, nblk, offs);
    RO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_use_write, dim3(nblk), dim3(256), 0, s, c->b.stamps, c->b.slot_brick, S, frame,
                       offs, out);
    RO_HIP(hipGetLastError());
    uint32_t n = 0;
    RO_HIP(hipMemcpyAsync(&n, offs + nblk, 4, hipMemcpyDeviceToHost, s));
    RO_HIP(hipStreamSynchronize(s));
    uint32_t k = n < cap ? n : cap;
    if (k) {
        RO_HIP(hipMemcpyAsync(slots, out, 4 * (size_t)k, hipMemcpyDeviceToHost, s));
        RO_HIP(hipStreamSynchronize(s));
    }
    *n_out = n;
    return RO_OK;
}

// ------------------------------------------------------- LRU slot choice

// Select state words.
enum { SEL_ELIG = 0, SEL_KEFF = 1, SEL_KREM = 2, SEL_NCAND = 3, SEL_PREFIX = 4 /* u64 at 4..5 */ };

__global__ void k_touch(uint32_t *__restrict__ stamp, const uint32_t *__restrict__ slots, uint32_t n,
                        uint32_t f) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) stamp[slots[i]] = f;
}

// LRU key per slot: free slots first in ascending index (key = slot), then
// occupied slots by (stamp, seq) (key = (stamp + 1) << 32 | seq); slots used
// in the current frame are not eligible (key = ~0).  Keys are unique.
__global__ void __launch_bounds__(256) k_keys(const uint32_t *__restrict__ slot_brick,
                                              const uint32_t *__restrict__ stamp,
                                              const uint32_t *__restrict__ seq, uint32_t S, uint32_t f,
                                              unsigned long long *__restrict__ keys,
                                              uint32_t *__restrict__ sel) {
    __shared__ uint32_t lds[4];
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    uint32_t elig = 0;
    if (i < S) {
        unsigned long long k;
        if (slot_brick[i] == kInvalid) {
            k = i;
            elig = 1;
        } else if (stamp[i] == f) {
            k = ~0ull;
        } else {
            k = ((unsigned long long)(stamp[i] + 1u) << 32) | seq[i];
            elig = 1;
        }
        keys[i] = k;
    }
    uint32_t tot;
    block_excl_scan_256(elig, lds, &tot);
    if (threadIdx.x == 0 && tot) atomicAdd(&sel[SEL_ELIG], tot);
}

__global__ void k_sel_init(uint32_t *sel, uint32_t n_new) {
    uint32_t k = sel[SEL_ELIG] < n_new ? sel[SEL_ELIG] : n_new;
    sel[SEL_KEFF] = k;
    sel[SEL_KREM] = k;
    sel[SEL_NCAND] = 0;
    sel[SEL_PREFIX] = 0;
    sel[SEL_PREFIX + 1] = 0;
}

// Radix-select pass: histogram of the digit at `shift` over keys whose
// higher digits equal the prefix chosen so far.
__global__ void __launch_bounds__(256) k_hist(const unsigned long long *__restrict__ keys, uint32_t S,
                                              const uint32_t *__restrict__ sel, int shift,
                                              uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    if (sel[SEL_KREM] == 0) return;
    h[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long prefix = ((unsigned long long)sel[SEL_PREFIX + 1] << 32) | sel[SEL_PREFIX];
    int hs = shift + 8;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < S; i += gridDim.x * 256) {
        unsigned long long k = keys[i];
        if (hs < 64 && (k >> hs) != (prefix >> hs)) continue;
        atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void __launch_bounds__(256) k_pick(uint32_t *__restrict__ hist, uint32_t *__restrict__ sel,
                                              int shift) {
    __shared__ uint32_t lds[4];
    uint32_t krem = sel[SEL_KREM];
    uint32_t v = hist[threadIdx.x];
    hist[threadIdx.x] = 0;
    if (krem == 0) return;
    uint32_t tot;
    uint32_t before = block_excl_scan_256(v, lds, &tot);
    if (before < krem && krem <= before + v) {
        unsigned long long prefix = ((unsigned long long)sel[SEL_PREFIX + 1] << 32) | sel[SEL_PREFIX];
        prefix |= (unsigned long long)threadIdx.x << shift;
        sel[SEL_PREFIX] = (uint32_t)prefix;
        sel[SEL_PREFIX + 1] = (uint32_t)(prefix >> 32);
        sel[SEL_KREM] = krem - before;
    }
}

// Collect the k_eff smallest keys (all keys <= the selected threshold).
__global__ void __launch_bounds__(256) k_collect(const unsigned long long *__restrict__ keys, uint32_t S,
                                                 uint32_t *__restrict__ sel,
                                                 unsigned long long *__restrict__ cand,
                                                 uint32_t *__restrict__ cand_slot, uint32_t cap) {
    if (sel[SEL_KEFF] == 0) return;
    unsigned long long thr = ((unsigned long long)sel[SEL_PREFIX + 1] << 32) | sel[SEL_PREFIX];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < S; i += gridDim.x * 256) {
        unsigned long long k = keys[i];
        if (k <= thr) {
            uint32_t at = atomicAdd(&sel[SEL_NCAND], 1u);
            if (at < cap) {  // exactly k_eff keys qualify (keys are unique)
                cand[at] = k;
                cand_slot[at] = i;
            }
        }
    }
}

// Order the candidates: rank = number of smaller keys (keys are unique).
__global__ void __launch_bounds__(256) k_rank(const unsigned long long *__restrict__ cand,
                                              const uint32_t *__restrict__ cand_slot,
                                              const uint32_t *__restrict__ sel,
                                              uint32_t *__restrict__ victims) {
    __shared__ unsigned long long tile[256];
    uint32_t n = sel[SEL_KEFF];
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    unsigned long long mine = i < n ? cand[i] : 0;
    uint32_t rank = 0;
    for (uint32_t t0 = 0; t0 < n; t0 += 256) {
        __syncthreads();
        if (t0 + threadIdx.x < n) tile[threadIdx.x] = cand[t0 + threadIdx.x];
        __syncthreads();
        uint32_t lim = n - t0 < 256 ? n - t0 : 256;
        for (uint32_t j = 0; j < lim; ++j) rank += tile[j] < mine;
    }
    if (i < n) victims[rank] = cand_slot[i];
}

// Page-table update: evict the victim's brick, insert the upload.
__global__ void k_pt_update(const uint32_t *__restrict__ sel, const uint32_t *__restrict__ victims,
                            const uint32_t *__restrict__ uploads, uint32_t *__restrict__ pt,
                            uint32_t *__restrict__ slot_brick, uint32_t *__restrict__ stamp,
                            uint32_t *__restrict__ seq, uint32_t *__restrict__ evicted, uint32_t f,
                            uint32_t seq_base) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sel[SEL_KEFF]) return;
    uint32_t slot = victims[i];
    uint32_t old = slot_brick[slot];
    if (old != kInvalid) pt[old] = kInvalid;
    evicted[i] = old;
    uint32_t b = uploads[i];
    pt[b] = slot;
    slot_brick[slot] = b;
    stamp[slot] = f;
    seq[slot] = seq_base + i;
}

// Brick scatter: staged brick src[i] -> slot victims[i], 16-byte vectors.
__global__ void __launch_bounds__(256) k_scatter(const uint32_t *__restrict__ sel,
                                                 const uint32_t *__restrict__ victims,
                                                 const uint32_t *__restrict__ src,
                                                 const uint4 *__restrict__ staged, uint4 *__restrict__ slots,
                                                 uint32_t vec_per_slot) {
    uint32_t i = blockIdx.y;
    if (i >= sel[SEL_KEFF]) return;
    const uint4 *from = staged + (size_t)src[i] * vec_per_slot;
    uint4 *to = slots + (size_t)victims[i] * vec_per_slot;
    for (uint32_t v = blockIdx.x * 256 + threadIdx.x; v < vec_per_slot; v += gridDim.x * 256)
        to[v] = from[v];
}

ro_status stream_bricks_device(ro_cache *c, uint32_t frame, uint32_t n_new, uint32_t n_touch,
                               const void *staged, hipStream_t s, uint32_t *k_eff_host,
                               uint32_t *victims_host, uint32_t *evicted_host) {
    const VolGeo &g = c->vol->g;
    uint8_t *sc = (uint8_t *)c->b.scratch;
    uint32_t S = c->desc.n_slots;
    unsigned long long *keys = (unsigned long long *)(sc + c->sc.keys);
    uint32_t *hist = (uint32_t *)(sc + c->sc.hist);
    uint32_t *sel = (uint32_t *)(sc + c->sc.sel);
    unsigned long long *cand = (unsigned long long *)(sc + c->sc.cand);
    uint32_t *victims = (uint32_t *)(sc + c->sc.victims);
    uint32_t *evicted = (uint32_t *)(sc + c->sc.evicted);
    uint32_t *uploads = (uint32_t *)(sc + c->sc.uploads);
    uint32_t *srcidx = (uint32_t *)(sc + c->sc.srcidx);
    uint32_t *touch = (uint32_t *)(sc + c->sc.touch);
    // candidate slots share the evicted array's space until the update
    uint32_t *cand_slot = (uint32_t *)(sc + c->sc.outpairs);
    if (n_touch) {
        hipLaunchKernelGGL(k_touch, dim3((n_touch + 255) / 256), dim3(256), 0, s, c->b.stamps, touch, n_touch,
                           frame);
        RO_HIP(hipGetLastError());
    }
    *k_eff_host = 0;
    if (n_new == 0) return RO_OK;
    RO_HIP(hipMemsetAsync(sel, 0, 64, s));
    RO_HIP(hipMemsetAsync(hist, 0, 1024, s));
    uint32_t nb = (S + 255) / 256;
    hipLaunchKernelGGL(k_keys, dim3(nb), dim3(256), 0, s, c->b.slot_brick, c->b.stamps, c->b.seqs, S, frame,
                       keys, sel);
    RO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1), 0, s, sel, n_new);
    RO_HIP(hipGetLastError());
    uint32_t hb = nb < 1024 ? nb : 1024;
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_hist, dim3(hb), dim3(256), 0, s, keys, S, sel, shift, hist);
        RO_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(256), 0, s, hist, sel, shift);
        RO_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_collect, dim3(hb), dim3(256), 0, s, keys, S, sel, cand, cand_slot, n_new);
    RO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rank, dim3((n_new + 255) / 256), dim3(256), 0, s, cand, cand_slot, sel, victims);
    RO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pt_update, dim3((n_new + 255) / 256), dim3(256), 0, s, sel, victims, uploads,
                       c->b.page_table, c->b.slot_brick, c->b.stamps, c->b.seqs, evicted, frame,
                       c->seq_next);
    RO_HIP(hipGetLastError());
    uint32_t vps = g.slot_stride / 16;
    uint32_t gx = (vps + 255) / 256;
    hipLaunchKernelGGL(k_scatter, dim3(gx, n_new), dim3(256), 0, s, sel, victims, srcidx,
                       (const uint4 *)staged, (uint4 *)c->b.slots, vps);
    RO_HIP(hipGetLastError());
    uint32_t selh[8];
    RO_HIP(hipMemcpyAsync(selh, sel, 32, hipMemcpyDeviceToHost, s));
    RO_HIP(hipMemcpyAsync(victims_host, victims, 4 * (size_t)n_new, hipMemcpyDeviceToHost, s));
    RO_HIP(hipMemcpyAsync(evicted_host, evicted, 4 * (size_t)n_new, hipMemcpyDeviceToHost, s));
    RO_HIP(hipStreamSynchronize(s));
    *k_eff_host = selh[SEL_KEFF];
    return RO_OK;
}


// Every resident brick whose dense index lies in [lo, hi) leaves the cache:
// its page-table entry and its slot's brick are cleared, so the slot is free.
__global__ void k_evict_range(uint32_t *__restrict__ slot_brick, uint32_t *__restrict__ pt, uint32_t S,
                              uint32_t lo, uint32_t hi) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const uint32_t b = slot_brick[i];
    if (b != kInvalid && b >= lo && b < hi) {
        pt[b] = kInvalid;
        slot_brick[i] = kInvalid;
    }
}

ro_status cache_evict_channel(ro_cache *c, uint32_t ch, hipStream_t s) {
    const VolGeo &g = c->vol->g;
    const uint32_t lo = ch * g.per_channel, hi = lo + g.per_channel;
    const uint32_t S = c->desc.n_slots;
    hipLaunchKernelGGL(k_evict_range, dim3((S + 255) / 256), dim3(256), 0, s, c->b.slot_brick, c->b.page_table, S,
                       lo, hi);
    RO_HIP(hipGetLastError());
    // the host mirrors follow; the evicted bricks await the residency update
    for (uint32_t i = 0; i < S; ++i) {
        const uint32_t b = c->slot_host[i];
        if (b != kInvalid && b >= lo && b < hi) {
            c->pt_host[b] = kInvalid;
            c->slot_host[i] = kInvalid;
            c->dirty.push_back(b);
        }
    }
    return RO_OK;
}

}  // namespace ro
