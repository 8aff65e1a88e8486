// Brick-request predictor: a 24-64-64-9 perceptron (ReLU hidden layers, one
// logit per resolution level) trained with masked binary cross-entropy.
// This network is an addition to the paper's method; it only changes which
// bricks are streamed, never how a frame is rendered from a cache state.
//
// All three layers run on MFMA (v_mfma_f32_16x16x16_f16: FP16 operands,
// FP32 accumulation).  A wave owns 16 rows at a time.  Layer shapes with
// padding: X [rows][32] (24 features), W1 [32][64], W2 [64][64],
// W3 [64][16] (9 logits), Z [rows][16].  Operand lane layout of the 16x16x16
// instruction (wave64, lane l, i = 0..3):
//   A (16 x 16, row-major M x K):  A[l % 16][4 (l / 16) + i]
//   B (16 x 16, K x N):            B[4 (l / 16) + i][l % 16]
//   C/D (16 x 16, M x N):          D[4 (l / 16) + i][l % 16]
// Activations move from the D layout to the A layout through a per-wave LDS
// tile.  Training recomputes the forward pass per tile, backpropagates with
// the loss scaled by the number of unmasked entries (so FP16 operands stay
// in range), accumulates weight gradients in FP32 per wave, reduces the
// per-wave partials in a fixed order (deterministic) and applies Adam to FP32
// master weights, refreshing the FP16 copies.
#include <math.h>
#include <string.h>

#include "common.h"

namespace ro {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// FP32 parameter block layout (floats), padded shapes.
constexpr int kW1 = 0, kB1 = kW1 + 32 * 64, kW2 = kB1 + 64, kB2 = kW2 + 64 * 64, kW3 = kB2 + 64,
              kB3 = kW3 + 64 * 16, kNP = kB3 + 16;  // 7312
// FP16 copies (halves): W1h [32][64], W2h [64][64], W3h [64][16]
constexpr int kH1 = 0, kH2 = kH1 + 32 * 64, kH3 = kH2 + 64 * 64, kNH = kH3 + 64 * 16;  // 7168
constexpr int kWaves = 4;            // waves per workgroup
constexpr int kTrainBlocks = 64;     // workgroups of the gradient kernel (fixed: deterministic sums)
constexpr int kPartials = kTrainBlocks * kWaves;
constexpr int kStat = 4;             // per-wave scalars: loss sum, mask count

__device__ __forceinline__ f4_t mfma16(half4_t a, half4_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

struct MlpLds {
    _Float16 w[kNH];
    float b1[64], b2[64], b3[16];
    _Float16 h1[kWaves][16 * 64];  // per-wave activation tiles [row][unit]
    _Float16 h2[kWaves][16 * 64];
    _Float16 t16[kWaves][16 * 64];  // per-wave gradient tiles
    _Float16 x[kWaves][16 * 32];
};

__device__ void load_weights(MlpLds &S, const _Float16 *wh, const float *p) {
    for (int i = threadIdx.x; i < kNH; i += blockDim.x) S.w[i] = wh[i];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        S.b1[i] = p[kB1 + i];
        S.b2[i] = p[kB2 + i];
        if (i < 16) S.b3[i] = p[kB3 + i];
    }
}

// Forward pass of one 16-row tile held in S.x[wv]: leaves relu(h1), relu(h2)
// in LDS (FP16), pre-activations a1, a2 and logits z in D layout.
__device__ __forceinline__ void tile_forward(MlpLds &S, int wv, f4_t a1[4], f4_t a2[4], f4_t &z) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    // layer 1: [16 x 32] x [32 x 64]
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f4_t acc = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            half4_t a, b;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = S.x[wv][r * 32 + 16 * ks + 4 * q + i];
                b[i] = S.w[kH1 + (16 * ks + 4 * q + i) * 64 + 16 * j + r];
            }
            acc = mfma16(a, b, acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            acc[i] += S.b1[16 * j + r];
            S.h1[wv][(4 * q + i) * 64 + 16 * j + r] = (_Float16)fmaxf(acc[i], 0.0f);
        }
        a1[j] = acc;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // layer 2: [16 x 64] x [64 x 64]
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f4_t acc = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            half4_t a, b;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = S.h1[wv][r * 64 + 16 * ks + 4 * q + i];
                b[i] = S.w[kH2 + (16 * ks + 4 * q + i) * 64 + 16 * j + r];
            }
            acc = mfma16(a, b, acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            acc[i] += S.b2[16 * j + r];
            S.h2[wv][(4 * q + i) * 64 + 16 * j + r] = (_Float16)fmaxf(acc[i], 0.0f);
        }
        a2[j] = acc;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // layer 3: [16 x 64] x [64 x 16]
    f4_t acc = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        half4_t a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = S.h2[wv][r * 64 + 16 * ks + 4 * q + i];
            b[i] = S.w[kH3 + (16 * ks + 4 * q + i) * 16 + r];
        }
        acc = mfma16(a, b, acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += S.b3[r];
    z = acc;
}

__device__ __forceinline__ void load_x_tile(MlpLds &S, int wv, const _Float16 *x, uint32_t rows, uint32_t r0) {
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < 16 * 32; i += 64) {
        const uint32_t row = r0 + (uint32_t)(i >> 5);
        S.x[wv][i] = row < rows ? x[(size_t)row * 32 + (i & 31)] : (_Float16)0.0f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(256) k_mlp_fwd(const _Float16 *__restrict__ x, uint32_t rows,
                                                 const _Float16 *__restrict__ wh, const float *__restrict__ p,
                                                 float *__restrict__ z) {
    __shared__ MlpLds S;
    load_weights(S, wh, p);
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t ntiles = (rows + 15) / 16;
    for (uint32_t t = blockIdx.x * kWaves + wv; t < ntiles; t += gridDim.x * kWaves) {
        load_x_tile(S, wv, x, rows, t * 16);
        f4_t a1[4], a2[4], zz;
        tile_forward(S, wv, a1, a2, zz);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t row = t * 16 + 4 * (lane >> 4) + i;
            if (row < rows) z[(size_t)row * 16 + (lane & 15)] = zz[i];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Gradient partials.  Each wave writes kNP + kStat floats to part[wave].
__global__ void __launch_bounds__(256) k_mlp_grad(const _Float16 *__restrict__ x, const uint8_t *__restrict__ y,
                                                  const uint8_t *__restrict__ msk, uint32_t rows,
                                                  const _Float16 *__restrict__ wh, const float *__restrict__ p,
                                                  float *__restrict__ part) {
    __shared__ MlpLds S;
    load_weights(S, wh, p);
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    f4_t g1[2][4], g2[4][4], g3[4];
    float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gb3 = 0.0f, lsum = 0.0f, msum = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        g3[a] = f4_t{0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 4; ++b) g2[a][b] = f4_t{0, 0, 0, 0};
        if (a < 2)
#pragma unroll
            for (int b = 0; b < 4; ++b) g1[a][b] = f4_t{0, 0, 0, 0};
    }
    const uint32_t ntiles = (rows + 15) / 16;
    const int wave = blockIdx.x * kWaves + wv;
    for (uint32_t t = (uint32_t)wave; t < ntiles; t += gridDim.x * kWaves) {
        const uint32_t r0 = t * 16;
        load_x_tile(S, wv, x, rows, r0);
        f4_t a1[4], a2[4], z;
        tile_forward(S, wv, a1, a2, z);
        // dz = mask * (sigmoid(z) - y)   (loss scaled by the mask count)
        f4_t dz;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t row = r0 + 4 * q + i;
            float d = 0.0f;
            if (row < rows) {
                const float mk = (float)msk[(size_t)row * 16 + r];
                const float yy = (float)y[(size_t)row * 16 + r];
                const float zz = z[i];
                const float s = 1.0f / (1.0f + expf(-zz));
                d = mk * (s - yy);
                // softplus(z) - y z, stably
                lsum += mk * (fmaxf(zz, 0.0f) + log1pf(expf(-fabsf(zz))) - yy * zz);
                msum += mk;
            }
            dz[i] = d;
            S.t16[wv][(4 * q + i) * 16 + r] = (_Float16)d;
            gb3 += d;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // gW3 += h2^T dz : M = 64 units (4 tiles), N = 16, K = 16 rows
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            half4_t a, b;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = S.h2[wv][(4 * q + i) * 64 + 16 * mt + r];
                b[i] = S.t16[wv][(4 * q + i) * 16 + r];
            }
            g3[mt] = mfma16(a, b, g3[mt]);
        }
        // dh2 = dz W3^T : M = 16 rows, N = 64 units, K = 16 logits; da2 = dh2 * (a2 > 0)
        half4_t adz;
#pragma unroll
        for (int i = 0; i < 4; ++i) adz[i] = S.t16[wv][r * 16 + 4 * q + i];
        f4_t da2[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            half4_t b;
#pragma unroll
            for (int i = 0; i < 4; ++i) b[i] = S.w[kH3 + (16 * j + r) * 16 + 4 * q + i];
            f4_t acc = mfma16(adz, b, f4_t{0, 0, 0, 0});
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = a2[j][i] > 0.0f ? acc[i] : 0.0f;
            da2[j] = acc;
        }
        __builtin_amdgcn_wave_barrier();
        // da2 -> LDS (reuse t16 as [row][64])
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                S.t16[wv][(4 * q + i) * 64 + 16 * j + r] = (_Float16)da2[j][i];
                gb2[j] += da2[j][i];
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // gW2 += h1^T da2 : M = 64 (4 tiles), N = 64 (4 tiles), K = 16 rows
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            half4_t a;
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = S.h1[wv][(4 * q + i) * 64 + 16 * mt + r];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                half4_t b;
#pragma unroll
                for (int i = 0; i < 4; ++i) b[i] = S.t16[wv][(4 * q + i) * 64 + 16 * nt + r];
                g2[mt][nt] = mfma16(a, b, g2[mt][nt]);
            }
        }
        // dh1 = da2 W2^T : M = 16 rows, N = 64, K = 64; da1 = dh1 * (a1 > 0)
        f4_t da1[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f4_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                half4_t a, b;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    a[i] = S.t16[wv][r * 64 + 16 * ks + 4 * q + i];
                    b[i] = S.w[kH2 + (16 * j + r) * 64 + 16 * ks + 4 * q + i];
                }
                acc = mfma16(a, b, acc);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = a1[j][i] > 0.0f ? acc[i] : 0.0f;
            da1[j] = acc;
        }
        __builtin_amdgcn_wave_barrier();
        // da1 -> LDS (the h2 tile is no longer needed)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                S.h2[wv][(4 * q + i) * 64 + 16 * j + r] = (_Float16)da1[j][i];
                gb1[j] += da1[j][i];
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // gW1 += x^T da1 : M = 32 inputs (2 tiles), N = 64 (4 tiles), K = 16 rows
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            half4_t a;
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = S.x[wv][(4 * q + i) * 32 + 16 * mt + r];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                half4_t b;
#pragma unroll
                for (int i = 0; i < 4; ++i) b[i] = S.h2[wv][(4 * q + i) * 64 + 16 * nt + r];
                g1[mt][nt] = mfma16(a, b, g1[mt][nt]);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // write this wave's partials (D layout -> parameter layout)
    float *o = part + (size_t)wave * (kNP + kStat);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) o[kW1 + (16 * mt + 4 * q + i) * 64 + 16 * nt + r] = g1[mt][nt][i];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) o[kW2 + (16 * mt + 4 * q + i) * 64 + 16 * nt + r] = g2[mt][nt][i];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) o[kW3 + (16 * mt + 4 * q + i) * 16 + r] = g3[mt][i];
    // bias partials: reduce the four lane groups (q) of each column
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float v1 = gb1[j], v2 = gb2[j];
        v1 += __shfl_xor(v1, 16, 64);
        v1 += __shfl_xor(v1, 32, 64);
        v2 += __shfl_xor(v2, 16, 64);
        v2 += __shfl_xor(v2, 32, 64);
        if (q == 0) {
            o[kB1 + 16 * j + r] = v1;
            o[kB2 + 16 * j + r] = v2;
        }
    }
    float v3 = gb3;
    v3 += __shfl_xor(v3, 16, 64);
    v3 += __shfl_xor(v3, 32, 64);
    if (q == 0) o[kB3 + r] = v3;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lsum += __shfl_xor(lsum, off, 64);
        msum += __shfl_xor(msum, off, 64);
    }
    if (lane == 0) {
        o[kNP + 0] = lsum;
        o[kNP + 1] = msum;
    }
}

// Sum the partials in a fixed order (deterministic): a block takes 64
// parameters; each of its 16 waves sums every 16th partial of them
// (coalesced rows, independent loads), then a pairwise tree over the 16 wave
// sums in LDS.
constexpr int kRedGroups = 16;
__global__ void __launch_bounds__(64 * kRedGroups) k_mlp_reduce(const float *__restrict__ part, int nparts,
                                                               float *__restrict__ grad, float *__restrict__ stat) {
    __shared__ float sm[kRedGroups][64];
    const int p = threadIdx.x & 63, gi = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + p;
    float acc = 0.0f;
    if (k < kNP + kStat)
        for (int w = gi; w < nparts; w += kRedGroups) acc += part[(size_t)w * (kNP + kStat) + k];
    sm[gi][p] = acc;
    __syncthreads();
    for (int h = kRedGroups / 2; h >= 1; h >>= 1) {
        if (gi < h) sm[gi][p] += sm[gi + h][p];
        __syncthreads();
    }
    if (gi == 0 && k < kNP + kStat) {
        if (k < kNP) grad[k] = sm[0][p];
        else stat[k - kNP] = sm[0][p];
    }
}

__global__ void k_mlp_scale(float *__restrict__ grad, const float *__restrict__ stat) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const float n = fmaxf(stat[1], 1.0f);
    if (k < kNP) grad[k] /= n;
}

// Adam step on the FP32 master weights; refresh the FP16 copies.
__global__ void k_mlp_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ g, _Float16 *__restrict__ wh, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kNP) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float w = p[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    p[k] = w;
    if (k < kB1) wh[kH1 + k] = (_Float16)w;
    else if (k >= kW2 && k < kB2) wh[kH2 + (k - kW2)] = (_Float16)w;
    else if (k >= kW3 && k < kB3) wh[kH3 + (k - kW3)] = (_Float16)w;
}

__global__ void k_mlp_refresh(const float *__restrict__ p, _Float16 *__restrict__ wh) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kNP) return;
    const float w = p[k];
    if (k < kB1) wh[kH1 + k] = (_Float16)w;
    else if (k >= kW2 && k < kB2) wh[kH2 + (k - kW2)] = (_Float16)w;
    else if (k >= kW3 && k < kB3) wh[kH3 + (k - kW3)] = (_Float16)w;
}

}  // namespace ro

using namespace ro;

// Device layout of the parameter buffer (bytes): FP32 master [kNP], Adam m
// [kNP], Adam v [kNP], gradient [kNP], stats [kStat], FP16 copies [kNH];
// workspace: kPartials x (kNP + kStat) floats.
struct ro_mlp {
    float *p, *m, *v, *g, *stat;
    _Float16 *wh;
    float *part;
    uint32_t step;
};

static size_t mlp_param_bytes() { return (size_t)(4 * kNP + kStat) * 4 + (size_t)kNH * 2 + 256; }
static size_t mlp_work_bytes() { return (size_t)kPartials * (kNP + kStat) * 4; }

extern "C" ro_status ro_mlp_query(size_t *param_bytes, size_t *workspace_bytes) {
    RO_CHECK(param_bytes && workspace_bytes, RO_E_ARG, "null argument");
    *param_bytes = mlp_param_bytes();
    *workspace_bytes = mlp_work_bytes();
    return RO_OK;
}

extern "C" ro_status ro_mlp_create(void *params_dev, void *workspace_dev, ro_mlp **out) {
    RO_CHECK(params_dev && workspace_dev && out, RO_E_ARG, "null argument");
    RO_CHECK(((uintptr_t)params_dev & 255u) == 0 && ((uintptr_t)workspace_dev & 255u) == 0, RO_E_ARG,
             "device buffers must be 256-byte aligned");
    ro_mlp *n = new (std::nothrow) ro_mlp;
    RO_CHECK(n, RO_E_NOMEM, "out of host memory");
    float *f = (float *)params_dev;
    n->p = f;
    n->m = f + kNP;
    n->v = f + 2 * kNP;
    n->g = f + 3 * kNP;
    n->stat = f + 4 * kNP;
    n->wh = (_Float16 *)(f + 4 * kNP + kStat);
    n->part = (float *)workspace_dev;
    n->step = 0;
    *out = n;
    return RO_OK;
}

extern "C" void ro_mlp_destroy(ro_mlp *n) { delete n; }

// Host weight layout (unpadded): W1[24][64], b1[64], W2[64][64], b2[64],
// W3[64][9], b3[9].

extern "C" ro_status ro_mlp_set_weights(ro_mlp *n, const float *host, void *stream) {
    RO_CHECK(n && host, RO_E_ARG, "null argument");
    std::vector<float> buf(3 * (size_t)kNP, 0.0f);  // p, m = 0, v = 0
    const float *h = host;
    for (int i = 0; i < 24; ++i)
        for (int j = 0; j < 64; ++j) buf[kW1 + i * 64 + j] = *h++;
    for (int j = 0; j < 64; ++j) buf[kB1 + j] = *h++;
    for (int i = 0; i < 64; ++i)
        for (int j = 0; j < 64; ++j) buf[kW2 + i * 64 + j] = *h++;
    for (int j = 0; j < 64; ++j) buf[kB2 + j] = *h++;
    for (int i = 0; i < 64; ++i)
        for (int j = 0; j < 9; ++j) buf[kW3 + i * 16 + j] = *h++;
    for (int j = 0; j < 9; ++j) buf[kB3 + j] = *h++;
    hipStream_t s = (hipStream_t)stream;
    RO_HIP(hipMemcpyAsync(n->p, buf.data(), sizeof(float) * 3 * kNP, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_mlp_refresh, dim3((kNP + 255) / 256), dim3(256), 0, s, n->p, n->wh);
    RO_HIP(hipGetLastError());
    RO_HIP(hipStreamSynchronize(s));  // the host buffer dies here
    n->step = 0;
    return RO_OK;
}

extern "C" ro_status ro_mlp_get_weights(const ro_mlp *n, float *host, void *stream) {
    RO_CHECK(n && host, RO_E_ARG, "null argument");
    std::vector<float> buf(kNP);
    hipStream_t s = (hipStream_t)stream;
    RO_HIP(hipMemcpyAsync(buf.data(), n->p, sizeof(float) * kNP, hipMemcpyDeviceToHost, s));
    RO_HIP(hipStreamSynchronize(s));
    float *h = host;
    for (int i = 0; i < 24; ++i)
        for (int j = 0; j < 64; ++j) *h++ = buf[kW1 + i * 64 + j];
    for (int j = 0; j < 64; ++j) *h++ = buf[kB1 + j];
    for (int i = 0; i < 64; ++i)
        for (int j = 0; j < 64; ++j) *h++ = buf[kW2 + i * 64 + j];
    for (int j = 0; j < 64; ++j) *h++ = buf[kB2 + j];
    for (int i = 0; i < 64; ++i)
        for (int j = 0; j < 9; ++j) *h++ = buf[kW3 + i * 16 + j];
    for (int j = 0; j < 9; ++j) *h++ = buf[kB3 + j];
    return RO_OK;
}

extern "C" ro_status ro_mlp_forward(ro_mlp *n, const uint16_t *x, uint32_t rows, float *z, void *stream) {
    RO_CHECK(n && (rows == 0 || (x && z)), RO_E_ARG, "null argument");
    if (rows == 0) return RO_OK;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t tiles = (rows + 15) / 16;
    uint32_t blocks = (tiles + kWaves - 1) / kWaves;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks), dim3(64 * kWaves), 0, s, (const _Float16 *)x, rows, n->wh, n->p, z);
    RO_HIP(hipGetLastError());
    return RO_OK;
}

static ro_status mlp_grad(ro_mlp *n, const uint16_t *x, const uint8_t *y, const uint8_t *mask, uint32_t rows,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(kTrainBlocks), dim3(64 * kWaves), 0, s, (const _Float16 *)x, y, mask, rows,
                       n->wh, n->p, n->part);
    RO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNP + kStat + 63) / 64), dim3(64 * kRedGroups), 0, s, n->part, kPartials,
                       n->g, n->stat);
    RO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_scale, dim3((kNP + 255) / 256), dim3(256), 0, s, n->g, n->stat);
    RO_HIP(hipGetLastError());
    return RO_OK;
}

extern "C" ro_status ro_mlp_gradients(ro_mlp *n, const uint16_t *x, const uint8_t *y, const uint8_t *mask,
                                      uint32_t rows, float *grads_host, float *loss_host, void *stream) {
    RO_CHECK(n && x && y && mask && grads_host, RO_E_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    ro_status st = mlp_grad(n, x, y, mask, rows, s);
    if (st) return st;
    std::vector<float> g(kNP + kStat);
    RO_HIP(hipMemcpyAsync(g.data(), n->g, sizeof(float) * (kNP + kStat), hipMemcpyDeviceToHost, s));
    RO_HIP(hipStreamSynchronize(s));
    float *h = grads_host;
    for (int i = 0; i < 24; ++i)
        for (int j = 0; j < 64; ++j) *h++ = g[kW1 + i * 64 + j];
    for (int j = 0; j < 64; ++j) *h++ = g[kB1 + j];
    for (int i = 0; i < 64; ++i)
        for (int j = 0; j < 64; ++j) *h++ = g[kW2 + i * 64 + j];
    for (int j = 0; j < 64; ++j) *h++ = g[kB2 + j];
    for (int i = 0; i < 64; ++i)
        for (int j = 0; j < 9; ++j) *h++ = g[kW3 + i * 16 + j];
    for (int j = 0; j < 9; ++j) *h++ = g[kB3 + j];
    if (loss_host) *loss_host = g[kNP + 0] / (g[kNP + 1] > 0 ? g[kNP + 1] : 1.0f);
    return RO_OK;
}

extern "C" ro_status ro_mlp_train_step(ro_mlp *n, const uint16_t *x, const uint8_t *y, const uint8_t *mask,
                                       uint32_t rows, float lr, float *loss_host, void *stream) {
    RO_CHECK(n && x && y && mask, RO_E_ARG, "null argument");
    RO_CHECK(lr > 0.0f, RO_E_ARG, "lr must be > 0");
    hipStream_t s = (hipStream_t)stream;
    ro_status st = mlp_grad(n, x, y, mask, rows, s);
    if (st) return st;
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)n->step), c2 = 1.0f - powf(b2, (float)n->step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kNP + 255) / 256), dim3(256), 0, s, n->p, n->m, n->v, n->g, n->wh, lr, b1, b2,
                       eps, c1, c2);
    RO_HIP(hipGetLastError());
    if (loss_host) {
        float stat[kStat];
        RO_HIP(hipMemcpyAsync(stat, n->stat, sizeof(stat), hipMemcpyDeviceToHost, s));
        RO_HIP(hipStreamSynchronize(s));
        *loss_host = stat[0] / (stat[1] > 0 ? stat[1] : 1.0f);
    }
    return RO_OK;
}
