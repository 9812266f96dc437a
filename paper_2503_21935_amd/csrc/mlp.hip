// mlp.hip -- surrogate network kernels: BF16 matrix-core GEMMs with FP32
// accumulation and fused epilogues, loss, reductions, Adam; the C ABI of
// include/mlp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mlp.h"
#include "me_internal.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define MLP_KPAD 32  // first-layer inputs padded to one MFMA K step
#define MLP_DW_SPLITS 16  // batch splits of the weight-gradient GEMMs
#ifndef MLPF_TILE_ROWS
#define MLPF_TILE_ROWS 128  // rows per block of the fused inference kernel (64: 5 % slower)
#endif

// ---------------------------------------------------------------------------
// GEMM: C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m * a_sm + k * a_sk],
// B(k, n) = B[k * b_sk + n * b_sn], BF16 operands, FP32 accumulation on
// v_mfma_f32_16x16x32_bf16.  A 256-thread block computes a 64 x 64 tile, each
// wave 32 x 32 (2 x 2 MFMA tiles).  Fragment layouts (16x16x32): lane l holds
// A[l%16][8(l/16) .. +7], B[8(l/16) .. +7][l%16] and D[4(l/16) + v][l%16].
// Requirements: K % 32 == 0; rows/columns beyond M/N are computed on clamped
// operands and not stored.
// ---------------------------------------------------------------------------
enum { EPI_FWD_TRAIN = 0, EPI_FWD_INFER = 1, EPI_BWD_DH = 2, EPI_DW = 3 };

struct epi_args {
    const float* bias;  // FWD: [N]
    float* z;           // FWD_TRAIN: pre-activations [M][N]
    bf16* h;            // FWD: activations [M][ldh]
    int ldh;
    const float* zprev; // BWD_DH: pre-activations of the previous layer [M][N]
    bf16* dz;           // BWD_DH: output gradient w.r.t. those pre-activations [M][N]
    float* g;           // DW: gradient [M][N] row-major with leading dimension ldg
    int ldg;
    int64_t zstride;    // DW with split K: elements between the partial slabs of blockIdx.z
    int ncols_store;    // DW: columns actually stored (n_in for the first layer)
};

// Logistic function with the hardware reciprocal (v_rcp_f32, about 1 ulp):
// a correctly rounded division costs ten instructions per activation, and the
// value is rounded to BF16 (8 bits) or enters an FP32 gradient next.
__device__ __forceinline__ float sigmoidf_(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

template <bool AK1, bool BK1>
__device__ __forceinline__ void load_frags(const bf16* __restrict__ A, int64_t a_sm, int64_t a_sk,
                                           const bf16* __restrict__ B, int64_t b_sk, int64_t b_sn, int row0,
                                           int col0, int k0, int M, int N, int lane, bf16x8 (&a)[2],
                                           bf16x8 (&b)[2]) {
    const int kk = k0 + 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        int r = row0 + 16 * i + (lane & 15);
        r = r < M ? r : M - 1;
        const bf16* p = A + (int64_t)r * a_sm + (int64_t)kk * a_sk;
        if constexpr (AK1) {
            a[i] = *reinterpret_cast<const bf16x8*>(p);
        } else {
#pragma unroll
            for (int v = 0; v < 8; ++v) a[i][v] = p[(int64_t)v * a_sk];
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        int c = col0 + 16 * j + (lane & 15);
        c = c < N ? c : N - 1;
        const bf16* p = B + (int64_t)kk * b_sk + (int64_t)c * b_sn;
        if constexpr (BK1) {
            b[j] = *reinterpret_cast<const bf16x8*>(p);
        } else {
#pragma unroll
            for (int v = 0; v < 8; ++v) b[j][v] = p[(int64_t)v * b_sk];
        }
    }
}

// Split K: block z of gridDim.z handles k in [z kspan, (z + 1) kspan) (kspan a
// multiple of 32); only the DW epilogue supports it (one partial slab per z).
template <int EPI, bool AK1, bool BK1>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, int kspan, const bf16* __restrict__ A,
                                              int64_t a_sm, int64_t a_sk, const bf16* __restrict__ B,
                                              int64_t b_sk, int64_t b_sn, epi_args e) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int col0 = blockIdx.x * 64 + (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kb = blockIdx.z * kspan, ke = min(K, kb + kspan);
    for (int k0 = kb; k0 < ke; k0 += 32) {
        bf16x8 a[2], b[2];
        load_frags<AK1, BK1>(A, a_sm, a_sk, B, b_sk, b_sn, row0, col0, k0, M, N, lane, a, b);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = col0 + 16 * j + (lane & 15);
            if (c >= N) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = row0 + 16 * i + 4 * (lane >> 4) + v;
                if (r >= M) continue;
                const float x = acc[i][j][v];
                if constexpr (EPI == EPI_FWD_TRAIN || EPI == EPI_FWD_INFER) {
                    const float z = x + e.bias[c];
                    if constexpr (EPI == EPI_FWD_TRAIN) e.z[(int64_t)r * N + c] = z;
                    e.h[(int64_t)r * e.ldh + c] = (bf16)(z * sigmoidf_(z));
                } else if constexpr (EPI == EPI_BWD_DH) {
                    const float z = e.zprev[(int64_t)r * N + c];
                    const float s = sigmoidf_(z);
                    e.dz[(int64_t)r * N + c] = (bf16)(x * s * (1.f + z * (1.f - s)));
                } else {
                    if (c < e.ncols_store) e.g[(int64_t)blockIdx.z * e.zstride + (int64_t)r * e.ldg + c] = x;
                }
            }
        }
}

// ---------------------------------------------------------------------------
// Fused inference for width 256: a block of 256 threads (4 waves) carries a
// tile of 128 rows through every layer with the activations in LDS, so the
// only HBM traffic is the input, the output and (from L2) the weights.  Per
// layer, wave w computes output columns 64w..64w+63 for all 128 rows (8 x 4
// MFMA tiles of 16 x 16, K steps of 32); after a barrier the bias + SiLU
// epilogue writes the BF16 activations over the layer's input.  Numerics as
// in the layered path: BF16 inputs, weights and activations, FP32
// accumulation, FP32 bias, activation and output layer.
// ---------------------------------------------------------------------------
#define MLPF_W 256
#define MLPF_PITCH (MLPF_W + 8)  // bf16 per LDS row: rows 528 B apart, no bank conflicts
#define MLPF_MAXDEPTH 8

struct mlpf_args {
    const bf16* w[MLPF_MAXDEPTH];   // hidden layers, [256][K] (K = 32 for the first, padded)
    const float* b[MLPF_MAXDEPTH];  // their biases [256]
    const float* wout;              // output weights [256]
    const float* bout;              // output bias [1]
};

// ROWS rows per 256-thread block (a multiple of 16 dividing 256).
template <int ROWS>
__global__ __launch_bounds__(256, 8192 / (ROWS * 32)) void k_mlp_infer(const float* __restrict__ x, int64_t n,
                                                                        int n_in, int depth, mlpf_args a,
                                                                        float* __restrict__ y) {
    constexpr int RT = ROWS / 16;      // 16-row MFMA tiles
    constexpr int TPR = 256 / ROWS;    // threads per row in the output layer
    __shared__ __attribute__((aligned(16))) bf16 H[ROWS * MLPF_PITCH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * ROWS;
    for (int e = threadIdx.x; e < ROWS * MLP_KPAD; e += 256) {
        const int r = e / MLP_KPAD, k = e % MLP_KPAD;
        const int64_t gr = row0 + r;
        H[r * MLPF_PITCH + k] = (bf16)((gr < n && k < n_in) ? x[gr * n_in + k] : 0.f);
    }
    __syncthreads();
    const int li = lane & 15, lg = lane >> 4;
    int K = MLP_KPAD;
    for (int l = 0; l < depth; ++l) {
        f32x4 acc[RT][4];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[rt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        const bf16* W = a.w[l];
        for (int k0 = 0; k0 < K; k0 += 32) {
            bf16x8 b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                b[t] = *reinterpret_cast<const bf16x8*>(W + (int64_t)(64 * wave + 16 * t + li) * K + k0 + 8 * lg);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const bf16x8 av = *reinterpret_cast<const bf16x8*>(H + (16 * rt + li) * MLPF_PITCH + k0 + 8 * lg);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[rt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[t], acc[rt][t], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave has read the layer's input
        const float* bias = a.b[l];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = 64 * wave + 16 * t + li;
            const float bc = bias[c];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float z = acc[rt][t][v] + bc;
                    H[(16 * rt + 4 * lg + v) * MLPF_PITCH + c] = (bf16)(z * sigmoidf_(z));
                }
        }
        __syncthreads();
        K = MLPF_W;
    }
    // output layer: y = sum_k h[k] w[k] + b; TPR adjacent threads per row, each
    // over MLPF_W / TPR columns in 16-byte reads, then a butterfly
    {
        const int r = threadIdx.x / TPR, part = threadIdx.x % TPR;
        constexpr int CW = MLPF_W / TPR;
        const bf16x8* hr = reinterpret_cast<const bf16x8*>(H + r * MLPF_PITCH + part * CW);
        const float* wo = a.wout + part * CW;
        float s = 0.f;
#pragma unroll 4
        for (int k8 = 0; k8 < CW / 8; ++k8) {
            const bf16x8 v = hr[k8];
#pragma unroll
            for (int q = 0; q < 8; ++q) s = fmaf((float)v[q], wo[8 * k8 + q], s);
        }
#pragma unroll
        for (int o = 1; o < TPR; o <<= 1) s += __shfl_xor(s, o);
        const int64_t gr = row0 + r;
        if (part == 0 && gr < n) y[gr] = s + a.bout[0];
    }
}

// ---------------------------------------------------------------------------
// Element-wise and reduction kernels
// ---------------------------------------------------------------------------

// X[j][k] = bf16(x[src(j)][k]) for k < n_in, zero for n_in <= k < 32.
__global__ void k_prep_input(const float* __restrict__ x, const int32_t* __restrict__ idx, int64_t n, int n_in,
                             bf16* __restrict__ X) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t src = idx ? idx[j] : j;
    for (int k = 0; k < MLP_KPAD; ++k) X[j * MLP_KPAD + k] = (bf16)(k < n_in ? x[src * n_in + k] : 0.f);
}

// y[m] = sum_k H[m][k] w[k] + b (FP32 accumulation)
__global__ void k_last_fwd(const bf16* __restrict__ H, int64_t M, int width, const float* __restrict__ w,
                           const float* __restrict__ b, float* __restrict__ y) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const bf16x8* h = reinterpret_cast<const bf16x8*>(H + m * width);
    float s = 0.f;
    for (int k8 = 0; k8 < width / 8; ++k8) {
        const bf16x8 v = h[k8];
#pragma unroll
        for (int q = 0; q < 8; ++q) s = fmaf((float)v[q], w[8 * k8 + q], s);
    }
    y[m] = s + b[0];
}

// dy[m] = 2 (y[m] - t[src(m)]) / M; per-block partial sums of the squared residual.
__global__ void k_loss(const float* __restrict__ y, const float* __restrict__ t, const int32_t* __restrict__ idx,
                       int64_t M, float* __restrict__ dy, float* __restrict__ partial) {
    __shared__ float red[256];
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float r2 = 0.f;
    if (m < M) {
        const float r = y[m] - t[idx ? idx[m] : m];
        dy[m] = 2.f * r / (float)M;
        r2 = r * r;
    }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_loss_final(const float* __restrict__ partial, int nblocks, int64_t M, float* __restrict__ loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < nblocks; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (float)M;
}

// dZ[m][n] = bf16(dy[m] w[n] silu'(Z[m][n]))
__global__ void k_last_bwd(const float* __restrict__ dy, const float* __restrict__ w, const float* __restrict__ Z,
                           int64_t M, int width, bf16* __restrict__ dZ) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * width) return;
    const int64_t m = i / width;
    const int n = (int)(i % width);
    const float z = Z[i];
    const float s = sigmoidf_(z);
    dZ[i] = (bf16)(dy[m] * w[n] * s * (1.f + z * (1.f - s)));
}

// part[z][n] = sum over rows m of chunk z of coef(m) A[m][n] (coef = dy[m] or 1);
// block (x, z) covers 64 columns of row chunk z; k_sum_splits adds the chunks.
template <typename TA>
__global__ void k_colsum_part(const TA* __restrict__ A, const float* __restrict__ coef, int64_t M, int N,
                              int64_t rows, float* __restrict__ part) {
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const int rg = threadIdx.x >> 6;
    const int64_t m0 = (int64_t)blockIdx.y * rows, m1 = (m0 + rows < M) ? m0 + rows : M;
    float s = 0.f;
    if (c < N)
        for (int64_t m = m0 + rg; m < m1; m += 4) s = fmaf(coef ? coef[m] : 1.f, (float)A[m * N + c], s);
    red[rg][threadIdx.x & 63] = s;
    __syncthreads();
    if (rg == 0 && c < N)
        part[(int64_t)blockIdx.y * N + c] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// out[0] = sum_m dy[m]
__global__ void k_sum(const float* __restrict__ v, int64_t M, float* __restrict__ out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t m = threadIdx.x; m < M; m += 256) s += v[m];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

struct layer_map {
    int64_t w_off[16], b_off[16];
    int fan_in[16];
};

// Adam with bias correction on the flat FP32 parameters, then the BF16 copies
// of the weight matrices (first layer padded to 32 inputs).
// Offset of element (n, k) of a [rows][K] matrix (rows a multiple of 16, K of
// 32) stored in fragment order: for each 16-row tile and 32-column step the
// 64 lanes' 16-byte B fragments of v_mfma_f32_16x16x32_bf16 (lane n % 16 +
// 16 ((k % 32) / 8) holds columns 8 ((k % 32) / 8) .. + 7 of row n) lie
// contiguously, so one load instruction reads 1 KB in lane order.
__device__ __forceinline__ int64_t frag_off(int n, int k, int K) {
    return ((int64_t)((n >> 4) * (K >> 5) + (k >> 5)) * 64 + (n & 15) + 16 * ((k & 31) >> 3)) * 8 + (k & 7);
}

__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t np, float lr, float c1, float c2, layer_map L,
                       int depth, int width, bf16* const* __restrict__ wbf, bf16* const* __restrict__ wbft,
                       bf16* const* __restrict__ wfr, bf16* const* __restrict__ wtfr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    theta[i] = th;
    for (int l = 0; l < depth; ++l) {
        const int64_t o = L.w_off[l];
        const int fi = L.fan_in[l];
        if (i >= o && i < o + (int64_t)width * fi) {
            const int64_t r = (i - o) / fi, k = (i - o) % fi;
            const int ld = (l == 0) ? MLP_KPAD : fi;
            wbf[l][r * ld + k] = (bf16)th;
            if (l > 0) wbft[l][k * width + r] = (bf16)th;
            if (wfr) {
                wfr[l][frag_off((int)r, (int)k, ld)] = (bf16)th;
                if (l > 0) wtfr[l][frag_off((int)k, (int)r, width)] = (bf16)th;
            }
        }
    }
}

// Fragment-order copies (see frag_off) of W_l (pads k >= fan_in zero) or, with
// trans, of W_l^T, from the master parameters.
__global__ void k_to_bf16_frag(const float* __restrict__ theta, int64_t o, int rows, int fi, int ld, int trans,
                               bf16* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * ld) return;
    if (!trans) {
        const int r = (int)(i / ld), k = (int)(i % ld);
        out[frag_off(r, k, ld)] = (bf16)(k < fi ? theta[o + (int64_t)r * fi + k] : 0.f);
    } else {
        const int k = (int)(i / rows), r = (int)(i % rows);  // row k of W^T, [fi][rows]
        out[frag_off(k, r, rows)] = (bf16)theta[o + (int64_t)r * fi + k];
    }
}

// BF16 copies from the master parameters (after set_params / init)
__global__ void k_to_bf16(const float* __restrict__ theta, int64_t o, int rows, int fi, int ld, bf16* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * ld) return;
    const int64_t r = i / ld, k = i % ld;
    w[i] = (bf16)(k < fi ? theta[o + r * fi + k] : 0.f);
}

// transposed BF16 copy wt[k][r] = theta[o + r fi + k] of a hidden weight matrix
__global__ void k_to_bf16_t(const float* __restrict__ theta, int64_t o, int rows, int fi, bf16* __restrict__ wt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * fi) return;
    const int64_t k = i / rows, r = i % rows;
    wt[i] = (bf16)theta[o + r * fi + k];
}

// ---------------------------------------------------------------------------
// Fused training step for width 256 (one cooperative launch; one grid-wide
// barrier inside a step, one between steps).  The batch's rows are
// independent through the whole forward and backward chain, so phase 1 gives
// each block tiles of FT_R rows and carries them through every layer forward
// (activations and pre-activations in LDS), the output layer and loss, and
// every layer backward down to the first pre-activation gradient, reading the
// BF16 weights (and their transposes) in MFMA fragment order from L2, each
// layer's fragments loaded during the previous layer's epilogue.  Each tile's
// activations and gradients also go to global memory transposed
// ([feature][batch], fragment order, written from LDS), and its share of the
// output layer's gradient to a per-tile partial.  The only cross-row work is
// the weight and bias gradients, sums over the batch: after the barrier,
// phase 2 computes them as GEMMs dW_l = dZ_l^T H_{l-1} on 32 x 32 tiles, one
// per block, each wave over a quarter of the batch; the quarters are added in
// LDS in a fixed order (the result does not depend on the grid) and the block
// applies Adam to the tile's FP32 masters and refreshes their BF16 copies, so
// every parameter is updated by the block that formed its gradient.  Rounding
// points are those of the layered path.
// ---------------------------------------------------------------------------
#define FT_R 16        // rows per phase-1 tile
#define FT_S 4         // batch quarters of the weight-gradient sums, one per wave
#define FT_MAXDEPTH 4  // pre-activations of every layer stay in LDS

struct ft_args {
    const float* x;           // [*][n_in]
    const float* t;           // targets
    const int32_t* idx;       // batch rows (nullptr: the first M)
    int64_t M;                // batch size (multiple of FT_S * 32)
    int n_in, depth;
    bf16* wfr[FT_MAXDEPTH];   // W_l [256][ld] in fragment order (ld 32 for the first layer)
    bf16* wtfr[FT_MAXDEPTH];  // W_l^T [fan_in][256] in fragment order (layers >= 1)
    bf16* wbf[FT_MAXDEPTH];   // row-major BF16 copies (other kernels), written by the launch's last step
    bf16* wbft[FT_MAXDEPTH];
    float* theta;             // FP32 masters (flat layout)
    float *m, *v;             // Adam moments
    float* grad_out;          // gradient only (no update) when non-null
    layer_map L;
    int64_t wout_off, bout_off, np;
    bf16* XT;                 // [32][M], fragment order with K = M
    bf16* HT[FT_MAXDEPTH];    // [256][M], the same
    bf16* DZT[FT_MAXDEPTH];   // [256][M], the same
    float* opart;             // [257][M / FT_R]: output-layer gradient per tile (weights, then bias)
    float* lossp;             // [gridDim.x]
    unsigned* bar;            // grid barrier state (zeroed once at allocation)
    float* loss;              // [nsteps] or nullptr
    float lr, c1, c2;         // one step (lrs == nullptr): its rate and bias corrections
    const float* lrs;         // [nsteps] rates of the steps, or nullptr
    int64_t step0;            // Adam steps taken before this launch
    int nsteps;               // steps in this launch, batch st on rows idx[st M ..] (or st M ..)
};

__device__ __forceinline__ float silu_d(float z) {
    const float s = sigmoidf_(z);
    return s * (1.f + z * (1.f - s));
}

// B fragments of rows 64 wave + 16 t + 0..15 of the [256][K] matrix Wm kept in
// fragment order (K / 32 MFMA k-steps).
template <int K>
__device__ __forceinline__ void ft_load_w(const bf16* __restrict__ Wm, int wave, int lane, bf16x8 (&b)[8][4]) {
#pragma unroll
    for (int ks = 0; ks < K / 32; ++ks)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            b[ks][t] = *reinterpret_cast<const bf16x8*>(Wm + ((int64_t)((4 * wave + t) * (K / 32) + ks) * 64 + lane) * 8);
}

// acc[t] = (16-row LDS tile A, pitch MLPF_PITCH) x (the loaded rows)^T.
template <int K>
__device__ __forceinline__ void ft_mma(const bf16* A, const bf16x8 (&b)[8][4], int li, int lg, f32x4 acc[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < K / 32; ++ks) {
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(A + li * MLPF_PITCH + 32 * ks + 8 * lg);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[ks][t], acc[t], 0, 0, 0);
    }
}

// The weights of product k of a tile's chain after the first layer (k = 1 ..
// 2 (depth - 1)): W_k forward for k < depth, then W_l^T backward for l =
// depth - 1 .. 1; nullptr past the end.
__device__ __forceinline__ const bf16* ft_chain_w(const bf16* const* wfr, const bf16* const* wtfr, int depth, int k) {
    if (k <= depth - 1) return wfr[k];
    if (k <= 2 * (depth - 1)) return wtfr[2 * depth - 1 - k];
    return nullptr;
}

// Grid-wide barrier of a cooperative launch (every block resident).  Each
// thread waits for its own memory operations, then one thread per block
// publishes the block's writes (agent-scope release: the L2 write-back),
// arrives on bar[0] and waits for the generation in bar[32] to move; the last
// block to arrive resets the count and moves the generation.  One release
// and one acquire per block, where a fence in every wave would write the L2
// back once per wave.
__device__ __forceinline__ void ft_grid_sync(unsigned* bar) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned g = __hip_atomic_load(&bar[32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned prev = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[32], g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(&bar[32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g)
                __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Column c of the 16-row LDS tile S (batch rows m0 .. m0 + 15) to the
// [feature][batch] array dst in fragment order with K = M (two 16-byte stores).
__device__ __forceinline__ void ft_store_t(const bf16* S, int c, bf16* dst, int64_t M, int64_t m0) {
    bf16x8 v0, v1;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        v0[r] = S[r * MLPF_PITCH + c];
        v1[r] = S[(8 + r) * MLPF_PITCH + c];
    }
    const int64_t base = ((int64_t)(c >> 4) * (M >> 5) + (m0 >> 5)) * 512 + (c & 15) * 8;
    const int q = (int)(m0 & 31) >> 3;  // 0 or 2
    *reinterpret_cast<bf16x8*>(dst + base + 128 * q) = v0;
    *reinterpret_cast<bf16x8*>(dst + base + 128 * (q + 1)) = v1;
}

// Adam on parameter i (FP32 master, moments) with gradient g and the loaded
// old values; returns the new master value.
__device__ __forceinline__ float ft_adam(const ft_args& a, int64_t i, float g, float mo, float vo, float th, float lr,
                                         float c1, float c2) {
    const float mi = 0.9f * mo + 0.1f * g;
    const float vi = 0.999f * vo + 0.001f * g * g;
    a.m[i] = mi;
    a.v[i] = vi;
    const float t2 = th - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    a.theta[i] = t2;
    return t2;
}

// The update of a parameter without BF16 copies (biases, output layer), or
// its gradient only.
__device__ __forceinline__ void ft_update(const ft_args& a, int64_t i, float g, float lr, float c1, float c2) {
    if (a.grad_out) {
        a.grad_out[i] = g;
        return;
    }
    ft_adam(a, i, g, a.m[i], a.v[i], a.theta[i], lr, c1, c2);
}

// The 16 input rows (padded to MLP_KPAD features) and targets of the tile at
// batch row m0 of step st: loaded into registers (two elements per thread),
// then written to LDS, so that the loads of the next step's first tile can be
// in flight across the end of the current step.
struct ft_rows {
    float xv[2], tv[2];
};

__device__ __forceinline__ void ft_rows_load(const ft_args& a, int st, int64_t m0, int tid, ft_rows& g) {
    static_assert(FT_R * MLP_KPAD == 2 * 256, "two elements per thread");
    const int32_t* idx = a.idx ? a.idx + (int64_t)st * a.M : nullptr;
    const float* x = a.idx ? a.x : a.x + (int64_t)st * a.M * a.n_in;
    const float* tg = a.idx ? a.t : a.t + (int64_t)st * a.M;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = tid + 256 * q, r = e / MLP_KPAD, k = e % MLP_KPAD;
        const int64_t src = idx ? idx[m0 + r] : m0 + r;
        g.xv[q] = k < a.n_in ? x[src * a.n_in + k] : 0.f;
        g.tv[q] = k == 0 ? tg[src] : 0.f;
    }
}

__device__ __forceinline__ void ft_rows_store(const ft_rows& g, int tid, bf16* Hs, float* tgs) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = tid + 256 * q, r = e / MLP_KPAD, k = e % MLP_KPAD;
        Hs[r * MLPF_PITCH + k] = (bf16)g.xv[q];
        if (k == 0) tgs[r] = g.tv[q];
    }
}

__global__ __launch_bounds__(256, 1) void k_mlp_train_fused(ft_args a) {
    constexpr int W = MLPF_W, P = MLPF_PITCH;
    static_assert(FT_R == 16 && W == 256, "one 16-row MFMA tile per phase-1 step, one thread per feature");
    __shared__ __attribute__((aligned(16))) bf16 Hs[FT_R * P];   // layer input / output
    __shared__ __attribute__((aligned(16))) bf16 Gs[FT_R * P];   // pre-activation gradient
    __shared__ float Zs[FT_MAXDEPTH][FT_R][W];                  // pre-activations
    __shared__ float bs[FT_MAXDEPTH][W];                        // hidden biases of this step
    __shared__ float wos[W + 1];                                // output weights and bias
    __shared__ float dys[FT_R], tgs[FT_R];
    __shared__ float red[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t M = a.M;
    const int nrt = (int)(M / FT_R);
    // B fragments: bw0 the first layer's (one k-step); the products after it
    // alternate between bwa (odd) and bwb (even), and the weights of product
    // k + 2 are loaded into a buffer as soon as product k has used it, so
    // every load has a whole layer's work to arrive
    bf16x8 bw0[8][4], bwa[8][4], bwb[8][4];
    bool first_in_lds = false;   // the step's first tile is already in Hs / tgs
    for (int st = 0; st < a.nsteps; ++st) {
        float* loss = a.loss ? a.loss + st : nullptr;
        const float lr = a.lrs ? a.lrs[st] : a.lr;
        const float c1 = a.lrs ? 1.f - powf(0.9f, (float)(a.step0 + st + 1)) : a.c1;
        const float c2 = a.lrs ? 1.f - powf(0.999f, (float)(a.step0 + st + 1)) : a.c2;
        float loss_acc = 0.f;
        for (int l = 0; l < a.depth; ++l) bs[l][tid] = a.theta[a.L.b_off[l] + tid];
        wos[tid] = a.theta[a.wout_off + tid];
        if (tid == 0) wos[W] = a.theta[a.bout_off];

        // ---------------- phase 1: rows through forward and backward ----------------
        for (int rt = blockIdx.x; rt < nrt; rt += gridDim.x) {
            const int64_t m0 = (int64_t)rt * FT_R;
            const bf16* const* wfr = a.wfr;
            const bf16* const* wtfr = a.wtfr;
            ft_load_w<MLP_KPAD>(wfr[0], wave, lane, bw0);
            if (const bf16* w1 = ft_chain_w(wfr, wtfr, a.depth, 1)) ft_load_w<W>(w1, wave, lane, bwa);
            if (const bf16* w2 = ft_chain_w(wfr, wtfr, a.depth, 2)) ft_load_w<W>(w2, wave, lane, bwb);
            if (!(first_in_lds && rt == (int)blockIdx.x)) {
                ft_rows g;
                ft_rows_load(a, st, m0, tid, g);
                ft_rows_store(g, tid, Hs, tgs);
            }
            __syncthreads();
            if (tid < MLP_KPAD) ft_store_t(Hs, tid, a.XT, M, m0);
#pragma unroll
            for (int l = 0; l < FT_MAXDEPTH; ++l) {
                if (l >= a.depth) break;
                f32x4 acc[4];
                if (l == 0) {
                    ft_mma<MLP_KPAD>(Hs, bw0, li, lg, acc);
                } else if (l & 1) {  // product l
                    ft_mma<W>(Hs, bwa, li, lg, acc);
                    if (const bf16* wn = ft_chain_w(wfr, wtfr, a.depth, l + 2)) ft_load_w<W>(wn, wave, lane, bwa);
                } else {
                    ft_mma<W>(Hs, bwb, li, lg, acc);
                    if (const bf16* wn = ft_chain_w(wfr, wtfr, a.depth, l + 2)) ft_load_w<W>(wn, wave, lane, bwb);
                }
                __syncthreads();  // the layer input has been read by every wave
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = 64 * wave + 16 * t + li;
                    const float bc = bs[l][c];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 4 * lg + v;
                        const float z = acc[t][v] + bc;
                        Zs[l][r][c] = z;
                        Hs[r * P + c] = (bf16)(z * sigmoidf_(z));
                    }
                }
                __syncthreads();
                ft_store_t(Hs, tid, a.HT[l], M, m0);
            }
            // output layer, residual, loss (16 threads per row)
            {
                const int r = tid >> 4, part = tid & 15;
                const bf16x8* hr = reinterpret_cast<const bf16x8*>(Hs + r * P + part * 16);
                float s = 0.f;
#pragma unroll
                for (int k8 = 0; k8 < 2; ++k8) {
                    const bf16x8 hv = hr[k8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) s = fmaf((float)hv[q], wos[part * 16 + 8 * k8 + q], s);
                }
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) s += __shfl_xor(s, o);
                if (part == 0) {
                    const float res = s + wos[W] - tgs[r];
                    dys[r] = 2.f * res / (float)M;
                    loss_acc += res * res;
                }
            }
            __syncthreads();
            // this tile's share of the output layer's gradient, and dZ of the last hidden layer
            {
                const int l = a.depth - 1, c = tid;
                const float woc = wos[c];
                float gw = 0.f, gb = 0.f;
#pragma unroll
                for (int r = 0; r < FT_R; ++r) {
                    gw = fmaf(dys[r], (float)Hs[r * P + c], gw);
                    gb += dys[r];
                    Gs[r * P + c] = (bf16)(dys[r] * woc * silu_d(Zs[l][r][c]));
                }
                a.opart[(int64_t)c * nrt + rt] = gw;
                if (c == 0) a.opart[(int64_t)W * nrt + rt] = gb;
            }
            __syncthreads();
            ft_store_t(Gs, tid, a.DZT[a.depth - 1], M, m0);
            // backward through the hidden layers: dZ_{l-1} = (dZ_l W_l) silu'(Z_{l-1})
            // (product 2 depth - 1 - l: bwa when l is even)
#pragma unroll
            for (int l = FT_MAXDEPTH - 1; l >= 1; --l) {
                if (l >= a.depth) continue;
                f32x4 acc[4];
                const int k = 2 * a.depth - 1 - l;
                if ((l & 1) == 0) {
                    ft_mma<W>(Gs, bwa, li, lg, acc);
                    if (const bf16* wn = ft_chain_w(wfr, wtfr, a.depth, k + 2)) ft_load_w<W>(wn, wave, lane, bwa);
                } else {
                    ft_mma<W>(Gs, bwb, li, lg, acc);
                    if (const bf16* wn = ft_chain_w(wfr, wtfr, a.depth, k + 2)) ft_load_w<W>(wn, wave, lane, bwb);
                }
                __syncthreads();  // Gs has been read by every wave
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 64 * wave + 16 * t + li;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 4 * lg + v;
                        Gs[r * P + k] = (bf16)(acc[t][v] * silu_d(Zs[l - 1][r][k]));
                    }
                }
                __syncthreads();
                ft_store_t(Gs, tid, a.DZT[l - 1], M, m0);
            }
            __syncthreads();  // Hs and Gs are rewritten by the next tile
        }
        red[tid] = loss_acc;
        __syncthreads();
        if (tid == 0) {
            float s = 0.f;
            for (int i = 0; i < 256; ++i) s += red[i];
            a.lossp[blockIdx.x] = s;
        }
        ft_grid_sync(a.bar);

        // ---------------- phase 2: weight gradients and the update ----------------
        if (blockIdx.x == 0 && loss && tid == 0) {
            float s = 0.f;
            for (int i = 0; i < (int)gridDim.x; ++i) s += a.lossp[i];
            loss[0] = s / (float)M;
        }
        // the next step's first tile, loaded across this phase and the barrier
        ft_rows nxt;
        const bool pre = st + 1 < a.nsteps && (int)blockIdx.x < nrt;
        if (pre) ft_rows_load(a, st + 1, (int64_t)blockIdx.x * FT_R, tid, nxt);
        // items: per layer l, 8 x (padded fan-in / 32) tiles of 32 x 32 of dW_l
        // (n-tile major), then eight output-layer items
        int nw = 0;
        for (int l = 0; l < a.depth; ++l) nw += 8 * (((l == 0) ? MLP_KPAD : W) / 32);
        const int nitems = nw + 8;
        float* part = &Zs[0][0][0];  // [wave][32][32] partial tiles, then [wave][32] bias partials
        // Items that share operand rows are neighbours in this order; blocks go
        // round-robin over the 8 XCDs, so slot v of XCD x takes item x q + v:
        // each XCD's L2 then fetches about an eighth of the operands instead
        // of nearly all of them.
        const int q8 = (nitems + 7) / 8;
        for (int vb = blockIdx.x; vb < 8 * q8; vb += gridDim.x) {
            const int it = (vb % 8) * q8 + vb / 8;
            if (it >= nitems) continue;
            if (it >= nw) {
                // output layer, columns 32 oq .. 32 oq + 31 (the last item also takes
                // the bias): eight threads per column add the per-tile partials in a
                // fixed interleave, combine them by shuffles and update
                const int oq = it - nw;
                const int c = 32 * oq + (tid >> 3), q = tid & 7;
                const float* src = a.opart + (int64_t)c * nrt;
                float g = 0.f;
#pragma unroll 8
                for (int i = q; i < nrt; i += 8) g += src[i];
                g += __shfl_xor(g, 1);
                g += __shfl_xor(g, 2);
                g += __shfl_xor(g, 4);
                if (q == 0) ft_update(a, a.wout_off + c, g, lr, c1, c2);
                if (oq == 7 && wave == 0) {
                    const float* sb = a.opart + (int64_t)W * nrt;
                    float d = 0.f;
#pragma unroll 8
                    for (int i = lane & 7; i < nrt; i += 8) d += sb[i];
                    d += __shfl_xor(d, 1);
                    d += __shfl_xor(d, 2);
                    d += __shfl_xor(d, 4);
                    if (lane == 0) ft_update(a, a.bout_off, d, lr, c1, c2);
                }
                continue;
            }
            int l = 0, j = it;
            for (; l < a.depth; ++l) {
                const int nl = 8 * (((l == 0) ? MLP_KPAD : W) / 32);
                if (j < nl) break;
                j -= nl;
            }
            const int kt = ((l == 0) ? MLP_KPAD : W) / 32;
            const int nb = j / kt, kb = j % kt;
            const int fi = a.L.fan_in[l], ld = (l == 0) ? MLP_KPAD : fi;
            // operands in fragment order: the fragment of 16-row tile f at batch
            // step m / 32 starts at (f (M / 32) + m / 32) 512
            const bf16* A = a.DZT[l];                       // dZ_l^T [n][m]
            const bf16* B = (l == 0) ? a.XT : a.HT[l - 1];  // H_{l-1}^T [k][m]
            const bf16* Ar[2];
            const bf16* Br[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                Ar[i] = A + (int64_t)(2 * nb + i) * (M >> 5) * 512 + lane * 8;
                Br[i] = B + (int64_t)(2 * kb + i) * (M >> 5) * 512 + lane * 8;
            }
            f32x4 acc[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int k = 0; k < 2; ++k) acc[i][k] = f32x4{0.f, 0.f, 0.f, 0.f};
            float bsum[2] = {0.f, 0.f};
            auto mstep = [&](const bf16x8 (&av)[2], const bf16x8 (&bv)[2]) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) bsum[i] += (float)av[i][q];
#pragma unroll
                    for (int k = 0; k < 2; ++k)
                        acc[i][k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[k], acc[i][k], 0, 0, 0);
                }
            };
            // this wave's quarter of the batch
            const int64_t mq = M / FT_S, mb = (int64_t)wave * mq;
            constexpr int U = 8;  // batch steps whose loads are all in flight together
            int64_t m = mb;
            for (; m + 32 * U <= mb + mq; m += 32 * U) {
                bf16x8 av[U][2], bv[U][2];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        av[u][i] = *reinterpret_cast<const bf16x8*>(Ar[i] + 16 * (m + 32 * u));
                        bv[u][i] = *reinterpret_cast<const bf16x8*>(Br[i] + 16 * (m + 32 * u));
                    }
#pragma unroll
                for (int u = 0; u < U; ++u) mstep(av[u], bv[u]);
            }
            for (; m < mb + mq; m += 32) {
                bf16x8 av[2], bv[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    av[i] = *reinterpret_cast<const bf16x8*>(Ar[i] + 16 * m);
                    bv[i] = *reinterpret_cast<const bf16x8*>(Br[i] + 16 * m);
                }
                mstep(av, bv);
            }
            // the wave's partial tile: element (n, k) = acc[i][k'][v], n = 16 i + 4 lg + v, k = 16 k' + li
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int v = 0; v < 4; ++v) part[(wave * 32 + 16 * i + 4 * lg + v) * 32 + 16 * k + li] = acc[i][k][v];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                bsum[i] += __shfl_xor(bsum[i], 16);
                bsum[i] += __shfl_xor(bsum[i], 32);
                if (lg == 0) part[4096 + wave * 32 + 16 * i + li] = bsum[i];
            }
            __syncthreads();
            // the four quarters added in wave order, then four of the tile's 1024
            // weights per thread (every load first)
            float g[4], mo[4], vo[4], th[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = tid + 256 * r, n = e >> 5, k = e & 31;
                g[r] = ((part[n * 32 + k] + part[(32 + n) * 32 + k]) + part[(64 + n) * 32 + k]) + part[(96 + n) * 32 + k];
                mo[r] = vo[r] = th[r] = 0.f;
                const int64_t i = a.L.w_off[l] + (int64_t)(32 * nb + n) * fi + 32 * kb + k;
                if (32 * kb + k < fi && !a.grad_out) {
                    mo[r] = a.m[i];
                    vo[r] = a.v[i];
                    th[r] = a.theta[i];
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = tid + 256 * r, n = e >> 5, k = e & 31;
                const int rr = 32 * nb + n, kk = 32 * kb + k;
                if (kk >= fi) continue;
                const int64_t i = a.L.w_off[l] + (int64_t)rr * fi + kk;
                if (a.grad_out) {
                    a.grad_out[i] = g[r];
                    continue;
                }
                const float t2 = ft_adam(a, i, g[r], mo[r], vo[r], th[r], lr, c1, c2);
                // the fragment-order copies feed the next step; the row-major
                // ones only other kernels, so they are written by the last step
                const bool last = st + 1 == a.nsteps;
                a.wfr[l][frag_off(rr, kk, ld)] = (bf16)t2;
                if (last) a.wbf[l][rr * ld + kk] = (bf16)t2;
                if (l > 0) {
                    a.wtfr[l][frag_off(kk, rr, W)] = (bf16)t2;
                    if (last) a.wbft[l][kk * W + rr] = (bf16)t2;
                }
            }
            if (kb == 0 && tid < 32) {
                const float gb = ((part[4096 + tid] + part[4096 + 32 + tid]) + part[4096 + 64 + tid]) + part[4096 + 96 + tid];
                ft_update(a, a.L.b_off[l] + 32 * nb + tid, gb, lr, c1, c2);
            }
            __syncthreads();  // part is rewritten by the next item
        }
        if (pre) ft_rows_store(nxt, tid, Hs, tgs);
        first_in_lds = pre;
        if (st + 1 < a.nsteps) ft_grid_sync(a.bar);  // the next step reads the updated weights
    }
}

__global__ void k_features(const double* __restrict__ mom, int64_t n, int npart, float* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* p = mom + i * npart * 4;
    const double E = p[0] + p[4], px = p[1] + p[5], py = p[2] + p[6], pz = p[3] + p[7];
    const double inv = 1.0 / sqrt(E * E - px * px - py * py - pz * pz);
    for (int c = 0; c < 4 * npart; ++c) x[i * 4 * npart + c] = (float)(p[c] * inv);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct me_mlp {
    int n_in, width, depth;
    int64_t np;
    layer_map L;
    int64_t wout_off, bout_off;
    float *theta, *grad, *m, *v;
    float* dwpart;           // split-K partial slabs of one weight gradient [MLP_DW_SPLITS][width][fan_in]
    std::vector<bf16*> wbf;  // per hidden layer, [width][ld]
    bf16** d_wbf;            // device array of those pointers
    std::vector<bf16*> wbft; // transposed copies [fan_in][width] (layers >= 1; the backward pass)
    bf16** d_wbft;
    std::vector<bf16*> wfr;  // fragment-order copies of W_l and W_l^T for the one-kernel step
    std::vector<bf16*> wtfr; // (width 256 only; empty otherwise)
    bf16 **d_wfr, **d_wtfr;
    bool fused;              // training step as one cooperative kernel where it applies
    int fgrid;               // its grid: co-resident blocks
    int64_t fcap;            // batch capacity of its buffers
    bf16 *XT, *HTb, *DZTb;   // transposed input, activations and gradients [feature][batch]
    float *flossp, *fopart;
    unsigned* fbar;          // grid barrier state of the fused kernel
    int64_t cap;             // activation capacity (rows)
    bf16* X;
    std::vector<bf16*> H;
    std::vector<float*> Z;
    bf16 *dZa, *dZb;
    float *y, *dy, *partial, *loss_tmp;
    int64_t step;
};

#define HCHK(expr)                                                                                   \
    do {                                                                                             \
        hipError_t _e = (expr);                                                                      \
        if (_e != hipSuccess) return me_fail(ME_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
    } while (0)

static uint64_t splitmix(uint64_t& s) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void free_acts(me_mlp* p) {
    auto f = [](void* q) {
        if (q) (void)hipFree(q);
    };
    f(p->X);
    for (auto q : p->H) f(q);
    for (auto q : p->Z) f(q);
    f(p->dZa);
    f(p->dZb);
    f(p->y);
    f(p->dy);
    f(p->partial);
    p->X = nullptr;
    p->H.assign(p->depth, nullptr);
    p->Z.assign(p->depth, nullptr);
    p->dZa = p->dZb = nullptr;
    p->y = p->dy = p->partial = nullptr;
    p->cap = 0;
}

static int ensure_acts(me_mlp* p, int64_t rows) {
    if (rows <= p->cap) return ME_OK;
    HCHK(hipDeviceSynchronize());
    free_acts(p);
    const int64_t W = p->width;
    HCHK(hipMalloc(&p->X, rows * MLP_KPAD * sizeof(bf16)));
    for (int l = 0; l < p->depth; ++l) {
        HCHK(hipMalloc(&p->H[l], rows * W * sizeof(bf16)));
        HCHK(hipMalloc(&p->Z[l], rows * W * sizeof(float)));
    }
    HCHK(hipMalloc(&p->dZa, rows * W * sizeof(bf16)));
    HCHK(hipMalloc(&p->dZb, rows * W * sizeof(bf16)));
    HCHK(hipMalloc(&p->y, rows * sizeof(float)));
    HCHK(hipMalloc(&p->dy, rows * sizeof(float)));
    HCHK(hipMalloc(&p->partial, ((rows + 255) / 256 + 1) * sizeof(float)));
    p->cap = rows;
    return ME_OK;
}

static hipError_t refresh_bf16(me_mlp* p, hipStream_t s) {
    for (int l = 0; l < p->depth; ++l) {
        const int fi = p->L.fan_in[l], ld = (l == 0) ? MLP_KPAD : fi;
        const int64_t tot = (int64_t)p->width * ld;
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p->theta, p->L.w_off[l],
                           p->width, fi, ld, p->wbf[l]);
        if (l > 0) {
            const int64_t nt = (int64_t)p->width * fi;
            hipLaunchKernelGGL(k_to_bf16_t, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, p->theta,
                               p->L.w_off[l], p->width, fi, p->wbft[l]);
        }
        if (p->d_wfr) {
            hipLaunchKernelGGL(k_to_bf16_frag, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p->theta,
                               p->L.w_off[l], p->width, fi, ld, 0, p->wfr[l]);
            if (l > 0)
                hipLaunchKernelGGL(k_to_bf16_frag, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p->theta,
                                   p->L.w_off[l], p->width, fi, ld, 1, p->wtfr[l]);
        }
    }
    return hipGetLastError();
}

template <int EPI, bool AK1, bool BK1>
// Returns the number of K splits launched (partial slabs for EPI_DW).
static int gemm(hipStream_t s, int M, int N, int K, const bf16* A, int64_t a_sm, int64_t a_sk, const bf16* B,
                int64_t b_sk, int64_t b_sn, const epi_args& e, int splits = 1) {
    const int kspan = ((K + splits - 1) / splits + 31) / 32 * 32;
    splits = (K + kspan - 1) / kspan;
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)splits);
    hipLaunchKernelGGL((k_gemm<EPI, AK1, BK1>), grid, dim3(256), 0, s, M, N, K, kspan, A, a_sm, a_sk, B, b_sk, b_sn,
                       e);
    return splits;
}

// out[i] = sum over z < splits of part[z n + i] (fixed order: deterministic)
__global__ void k_sum_splits(const float* __restrict__ part, int splits, int64_t n, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float acc = 0.f;
    for (int z = 0; z < splits; ++z) acc += part[(int64_t)z * n + i];
    out[i] = acc;
}

// out[n] = sum_m coef(m) A[m][n] over all M rows, in row chunks (partials in
// p->dwpart, summed in a fixed order).
static void colsum(hipStream_t s, const bf16* A, const float* coef, int64_t M, int N, float* scratch, float* out) {
    const int64_t chunks = std::min<int64_t>(64, (M + 63) / 64);
    const int64_t rows = (M + chunks - 1) / chunks;
    hipLaunchKernelGGL((k_colsum_part<bf16>), dim3((unsigned)((N + 63) / 64), (unsigned)chunks), dim3(256), 0, s, A,
                       coef, M, N, rows, scratch);
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, scratch, (int)chunks,
                       (int64_t)N, out);
}

// Forward over rows [0, M) of p->X; training keeps Z and every H.
static void forward(me_mlp* p, int64_t M, bool train, hipStream_t s) {
    const int W = p->width;
    const bf16* in = p->X;
    int ld_in = MLP_KPAD, K = MLP_KPAD;
    for (int l = 0; l < p->depth; ++l) {
        epi_args e{};
        e.bias = p->theta + p->L.b_off[l];
        e.z = train ? p->Z[l] : nullptr;
        bf16* out = train ? p->H[l] : ((l & 1) ? p->dZb : p->dZa);  // inference ping-pongs
        e.h = out;
        e.ldh = W;
        // Z = in . W_l^T: A = in [M][K] (k contiguous), B(k, n) = W_l[n][k] (k contiguous)
        if (train)
            gemm<EPI_FWD_TRAIN, true, true>(s, (int)M, W, K, in, ld_in, 1, p->wbf[l], 1, K, e);
        else
            gemm<EPI_FWD_INFER, true, true>(s, (int)M, W, K, in, ld_in, 1, p->wbf[l], 1, K, e);
        in = out;
        ld_in = W;
        K = W;
    }
    hipLaunchKernelGGL(k_last_fwd, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, in, M, W,
                       p->theta + p->wout_off, p->theta + p->bout_off, p->y);
}

// Loss and gradients (into p->grad) for rows [0, M) with targets t[idx].
static void backward(me_mlp* p, const float* t, const int32_t* idx, int64_t M, float* loss, hipStream_t s) {
    const int W = p->width;
    const unsigned nb = (unsigned)((M + 255) / 256);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, p->y, t, idx, M, p->dy, p->partial);
    if (loss) hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, p->partial, (int)nb, M, loss);
    bf16* Hl = p->H[p->depth - 1];
    // output layer: dw_out = sum_m dy[m] H[m][:], db_out = sum dy
    colsum(s, Hl, p->dy, M, W, p->dwpart, p->grad + p->wout_off);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, p->dy, M, p->grad + p->bout_off);
    hipLaunchKernelGGL(k_last_bwd, dim3((unsigned)((M * W + 255) / 256)), dim3(256), 0, s, p->dy,
                       p->theta + p->wout_off, p->Z[p->depth - 1], M, W, p->dZa);
    bf16* dz = p->dZa;
    bf16* dz_next = p->dZb;
    for (int l = p->depth - 1; l >= 0; --l) {
        const bf16* hin = (l == 0) ? p->X : p->H[l - 1];
        const int fi = p->L.fan_in[l], ldin = (l == 0) ? MLP_KPAD : W;
        // dW_l[n][k] = sum_m dZ[m][n] hin[m][k]: A(n, m) = dZ[m][n], B(m, k) = hin[m][k]
        // split over the batch (K): 16 x 16 blocks instead of 16, partial slabs summed after
        const int splits = (int)std::min<int64_t>(MLP_DW_SPLITS, std::max<int64_t>(1, M / 256));
        epi_args e{};
        e.g = splits > 1 ? p->dwpart : p->grad + p->L.w_off[l];
        e.ldg = fi;
        e.ncols_store = fi;
        e.zstride = (int64_t)W * fi;
        const int used = gemm<EPI_DW, false, false>(s, W, ldin, (int)M, dz, 1, W, hin, ldin, 1, e, splits);
        if (splits > 1) {
            const int64_t nw = (int64_t)W * fi;
            hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, p->dwpart, used, nw,
                               p->grad + p->L.w_off[l]);
        }
        colsum(s, dz, nullptr, M, W, p->dwpart, p->grad + p->L.b_off[l]);
        if (l > 0) {
            // dH_{l-1}[m][k] = sum_n dZ[m][n] W_l[n][k]; fused silu'(Z_{l-1})
            epi_args e2{};
            e2.zprev = p->Z[l - 1];
            e2.dz = dz_next;
            gemm<EPI_BWD_DH, true, false>(s, (int)M, W, W, dz, W, 1, p->wbf[l], W, 1, e2);
            bf16* tmp = dz;
            dz = dz_next;
            dz_next = tmp;
        }
    }
}

extern "C" {

int mlp_create(int n_in, int width, int depth, uint64_t seed, me_mlp** out) {
    if (!out || n_in < 1 || n_in > MLP_KPAD || width < 64 || width % 64 || width > 1024 || depth < 1 || depth > 16)
        return me_fail(ME_EINVAL, "mlp_create: need 1 <= n_in <= 32, width a multiple of 64 up to 1024, depth 1..16");
    me_mlp* p = new (std::nothrow) me_mlp();
    if (!p) return me_fail(ME_ENOMEM, "host allocation");
    p->n_in = n_in;
    p->width = width;
    p->depth = depth;
    int64_t o = 0;
    int fi = n_in;
    for (int l = 0; l < depth; ++l) {
        p->L.w_off[l] = o;
        p->L.fan_in[l] = fi;
        o += (int64_t)width * fi;
        p->L.b_off[l] = o;
        o += width;
        fi = width;
    }
    p->wout_off = o;
    o += width;
    p->bout_off = o;
    o += 1;
    p->np = o;
    p->H.assign(depth, nullptr);
    p->Z.assign(depth, nullptr);
    p->wbf.assign(depth, nullptr);
    p->wbft.assign(depth, nullptr);
    p->wfr.assign(depth, nullptr);
    p->wtfr.assign(depth, nullptr);
    std::vector<float> h(o, 0.f);
    uint64_t st = seed;
    for (int l = 0; l < depth; ++l) {
        const double a = std::sqrt(6.0 / p->L.fan_in[l]);
        for (int64_t i = 0; i < (int64_t)width * p->L.fan_in[l]; ++i)
            h[p->L.w_off[l] + i] = (float)(a * (2.0 * ((splitmix(st) >> 11) * (1.0 / 9007199254740992.0)) - 1.0));
    }
    {
        const double a = std::sqrt(6.0 / width);
        for (int64_t i = 0; i < width; ++i)
            h[p->wout_off + i] = (float)(a * (2.0 * ((splitmix(st) >> 11) * (1.0 / 9007199254740992.0)) - 1.0));
    }
    auto bad = [&](hipError_t e) {
        if (e != hipSuccess) {
            mlp_free(p);
            return true;
        }
        return false;
    };
    if (bad(hipMalloc(&p->theta, o * sizeof(float))) || bad(hipMalloc(&p->grad, o * sizeof(float))) ||
        bad(hipMalloc(&p->m, o * sizeof(float))) || bad(hipMalloc(&p->v, o * sizeof(float))) ||
        bad(hipMalloc(&p->dwpart, (size_t)MLP_DW_SPLITS * width * width * sizeof(float))))
        return me_fail(ME_ENOMEM, "mlp_create: device allocation");
    for (int l = 0; l < depth; ++l) {
        const int ld = (l == 0) ? MLP_KPAD : p->L.fan_in[l];
        if (bad(hipMalloc(&p->wbf[l], (size_t)width * ld * sizeof(bf16))))
            return me_fail(ME_ENOMEM, "mlp_create: device allocation");
        if (l > 0 && bad(hipMalloc(&p->wbft[l], (size_t)width * p->L.fan_in[l] * sizeof(bf16))))
            return me_fail(ME_ENOMEM, "mlp_create: device allocation");
    }
    p->fused = (width == MLPF_W && depth <= FT_MAXDEPTH && n_in <= MLP_KPAD);
    p->fgrid = 0;
    if (p->fused) {
        for (int l = 0; l < depth; ++l) {
            const int ld = (l == 0) ? MLP_KPAD : p->L.fan_in[l];
            if (bad(hipMalloc(&p->wfr[l], (size_t)width * ld * sizeof(bf16))) ||
                (l > 0 && bad(hipMalloc(&p->wtfr[l], (size_t)width * ld * sizeof(bf16)))))
                return me_fail(ME_ENOMEM, "mlp_create: device allocation");
        }
        if (bad(hipMalloc(&p->d_wfr, depth * sizeof(bf16*))) ||
            bad(hipMemcpy(p->d_wfr, p->wfr.data(), depth * sizeof(bf16*), hipMemcpyHostToDevice)) ||
            bad(hipMalloc(&p->d_wtfr, depth * sizeof(bf16*))) ||
            bad(hipMemcpy(p->d_wtfr, p->wtfr.data(), depth * sizeof(bf16*), hipMemcpyHostToDevice)))
            return me_fail(ME_EDEVICE, "mlp_create: device allocation");
        int dev = 0, cus = 0, per = 0;
        if (bad(hipGetDevice(&dev)) || bad(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) ||
            bad(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_mlp_train_fused, 256, 0)))
            return me_fail(ME_EDEVICE, "mlp_create: occupancy query");
        p->fgrid = cus * per;
        if (p->fgrid < 1) p->fused = false;
    }
    if (bad(hipMalloc(&p->d_wbf, depth * sizeof(bf16*))) ||
        bad(hipMemcpy(p->d_wbf, p->wbf.data(), depth * sizeof(bf16*), hipMemcpyHostToDevice)) ||
        bad(hipMalloc(&p->d_wbft, depth * sizeof(bf16*))) ||
        bad(hipMemcpy(p->d_wbft, p->wbft.data(), depth * sizeof(bf16*), hipMemcpyHostToDevice)) ||
        bad(hipMemcpy(p->theta, h.data(), o * sizeof(float), hipMemcpyHostToDevice)) ||
        bad(hipMemset(p->m, 0, o * sizeof(float))) || bad(hipMemset(p->v, 0, o * sizeof(float))) ||
        bad(hipMemset(p->grad, 0, o * sizeof(float))) || bad(refresh_bf16(p, nullptr)) ||
        bad(hipDeviceSynchronize()))
        return me_fail(ME_EDEVICE, "mlp_create: initialisation");
    p->step = 0;
    *out = p;
    return ME_OK;
}

int mlp_n_params(const me_mlp* p, int64_t* n) {
    if (!p || !n) return me_fail(ME_EINVAL, "null argument");
    *n = p->np;
    return ME_OK;
}

int mlp_dims(const me_mlp* p, int* n_in, int* width, int* depth) {
    if (!p) return me_fail(ME_EINVAL, "null network");
    if (n_in) *n_in = p->n_in;
    if (width) *width = p->width;
    if (depth) *depth = p->depth;
    return ME_OK;
}

int mlp_get_params(me_mlp* p, float* host, int64_t n) {
    if (!p || !host || n != p->np) return me_fail(ME_EINVAL, "mlp_get_params: null or wrong size");
    HCHK(hipDeviceSynchronize());
    HCHK(hipMemcpy(host, p->theta, n * sizeof(float), hipMemcpyDeviceToHost));
    return ME_OK;
}

int mlp_set_params(me_mlp* p, const float* host, int64_t n) {
    if (!p || !host || n != p->np) return me_fail(ME_EINVAL, "mlp_set_params: null or wrong size");
    HCHK(hipDeviceSynchronize());
    HCHK(hipMemcpy(p->theta, host, n * sizeof(float), hipMemcpyHostToDevice));
    HCHK(refresh_bf16(p, nullptr));
    HCHK(hipDeviceSynchronize());
    return ME_OK;
}

int mlp_forward(me_mlp* p, const float* x, int64_t n, float* y, void* stream) {
    if (!p || n < 0) return me_fail(ME_EINVAL, "mlp_forward: null or negative n");
    if (n == 0) return ME_OK;
    if (!x || !y) return me_fail(ME_EINVAL, "mlp_forward: null buffer");
    hipStream_t s = (hipStream_t)stream;
    if (p->width == MLPF_W && p->n_in <= MLP_KPAD && p->depth <= MLPF_MAXDEPTH) {
        mlpf_args a{};
        for (int l = 0; l < p->depth; ++l) {
            a.w[l] = p->wbf[l];
            a.b[l] = p->theta + p->L.b_off[l];
        }
        a.wout = p->theta + p->wout_off;
        a.bout = p->theta + p->bout_off;
        constexpr int rows = MLPF_TILE_ROWS;
        hipLaunchKernelGGL(k_mlp_infer<rows>, dim3((unsigned)((n + rows - 1) / rows)), dim3(256), 0, s, x, n,
                           p->n_in, p->depth, a, y);
        HCHK(hipGetLastError());
        return ME_OK;
    }
    const int64_t chunk = 1 << 16;
    int rc = ensure_acts(p, std::min<int64_t>(n, chunk));
    if (rc != ME_OK) return rc;
    for (int64_t o = 0; o < n; o += chunk) {
        const int64_t m = std::min<int64_t>(chunk, n - o);
        hipLaunchKernelGGL(k_prep_input, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, x + o * p->n_in,
                           nullptr, m, p->n_in, p->X);
        forward(p, m, false, s);
        HCHK(hipMemcpyAsync(y + o, p->y, m * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    HCHK(hipGetLastError());
    return ME_OK;
}

// Batch buffers of the fused step (grow on the first call with a larger batch;
// that call synchronises the device).
static int ensure_fused(me_mlp* p, int64_t M) {
    if (M <= p->fcap) return ME_OK;
    HCHK(hipDeviceSynchronize());
    auto f = [](void* q) {
        if (q) (void)hipFree(q);
    };
    f(p->XT);
    f(p->HTb);
    f(p->DZTb);
    f(p->flossp);
    f(p->fopart);
    f(p->fbar);
    p->fbar = nullptr;
    p->XT = p->HTb = p->DZTb = nullptr;
    p->flossp = p->fopart = nullptr;
    p->fcap = 0;
    const int64_t W = p->width;
    HCHK(hipMalloc(&p->XT, MLP_KPAD * M * sizeof(bf16)));
    HCHK(hipMalloc(&p->HTb, p->depth * W * M * sizeof(bf16)));
    HCHK(hipMalloc(&p->DZTb, p->depth * W * M * sizeof(bf16)));
    HCHK(hipMalloc(&p->flossp, p->fgrid * sizeof(float)));
    HCHK(hipMalloc(&p->fopart, (W + 1) * (M / FT_R) * sizeof(float)));
    HCHK(hipMalloc(&p->fbar, 64 * sizeof(unsigned)));
    HCHK(hipMemset(p->fbar, 0, 64 * sizeof(unsigned)));
    p->fcap = M;
    return ME_OK;
}

static bool fused_applies(const me_mlp* p, int64_t n) {
    return p->fused && n >= FT_S * 32 && n % (FT_S * 32) == 0 && n <= (int64_t)1 << 24;
}

// nsteps training steps (grad_out == nullptr; rates lr_dev[nsteps] on the
// device, or lr for a single step) or the gradient only, as one launch of the
// fused cooperative kernel.
static int fused_step(me_mlp* p, const float* x, const float* t, const int32_t* idx, int64_t n, int64_t nsteps,
                      float lr, const float* lr_dev, float* loss, float* grad_out, hipStream_t s) {
    int rc = ensure_fused(p, n);
    if (rc != ME_OK) return rc;
    ft_args a{};
    a.x = x;
    a.t = t;
    a.idx = idx;
    a.M = n;
    a.n_in = p->n_in;
    a.depth = p->depth;
    for (int l = 0; l < p->depth; ++l) {
        a.wfr[l] = p->wfr[l];
        a.wtfr[l] = p->wtfr[l];
        a.wbf[l] = p->wbf[l];
        a.wbft[l] = p->wbft[l];
        a.HT[l] = p->HTb + (int64_t)l * p->width * n;
        a.DZT[l] = p->DZTb + (int64_t)l * p->width * n;
    }
    a.theta = p->theta;
    a.m = p->m;
    a.v = p->v;
    a.grad_out = grad_out;
    a.L = p->L;
    a.wout_off = p->wout_off;
    a.bout_off = p->bout_off;
    a.np = p->np;
    a.XT = p->XT;
    a.opart = p->fopart;
    a.lossp = p->flossp;
    a.bar = p->fbar;
    a.loss = loss;
    a.nsteps = (int)nsteps;
    a.step0 = p->step;
    a.lrs = lr_dev;
    a.lr = lr;
    if (!grad_out) {
        a.c1 = 1.f - std::pow(0.9f, (float)(p->step + 1));
        a.c2 = 1.f - std::pow(0.999f, (float)(p->step + 1));
        p->step += nsteps;
    } else {
        a.c1 = a.c2 = 1.f;
    }
    void* args[] = {&a};
    HCHK(hipLaunchCooperativeKernel((const void*)k_mlp_train_fused, dim3((unsigned)p->fgrid), dim3(256), args, 0, s));
    return ME_OK;
}

static int grad_common(me_mlp* p, const float* x, const float* t, const int32_t* idx, int64_t n, float* loss,
                       hipStream_t s) {
    if (!p || !x || !t || n <= 0 || n % 64) return me_fail(ME_EINVAL, "batch must be a positive multiple of 64");
    int rc = ensure_acts(p, n);
    if (rc != ME_OK) return rc;
    hipLaunchKernelGGL(k_prep_input, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, idx, n, p->n_in, p->X);
    forward(p, n, true, s);
    backward(p, t, idx, n, loss, s);
    HCHK(hipGetLastError());
    return ME_OK;
}

int mlp_set_fused_step(me_mlp* p, int on) {
    if (!p) return me_fail(ME_EINVAL, "null network");
    if (on && !(p->width == MLPF_W && p->depth <= FT_MAXDEPTH && p->n_in <= MLP_KPAD && p->fgrid > 0))
        return me_fail(ME_ESTATE, "the fused step needs width 256, depth <= 4 and n_in <= 32");
    p->fused = on != 0;
    return ME_OK;
}

int mlp_backward(me_mlp* p, const float* x, const float* t, const int32_t* idx, int64_t n, float* grad_dev,
                 float* loss_dev, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (p && x && t && grad_dev && fused_applies(p, n))
        return fused_step(p, x, t, idx, n, 1, 0.f, nullptr, loss_dev, grad_dev, s);
    int rc = grad_common(p, x, t, idx, n, loss_dev, s);
    if (rc != ME_OK) return rc;
    if (grad_dev) HCHK(hipMemcpyAsync(grad_dev, p->grad, p->np * sizeof(float), hipMemcpyDeviceToDevice, s));
    return ME_OK;
}

int mlp_train_step(me_mlp* p, const float* x, const float* t, const int32_t* idx, int64_t n, float lr,
                   float* loss_dev, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (p && x && t && fused_applies(p, n)) return fused_step(p, x, t, idx, n, 1, lr, nullptr, loss_dev, nullptr, s);
    int rc = grad_common(p, x, t, idx, n, loss_dev, s);
    if (rc != ME_OK) return rc;
    p->step += 1;
    const float c1 = 1.f - std::pow(0.9f, (float)p->step), c2 = 1.f - std::pow(0.999f, (float)p->step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((p->np + 255) / 256)), dim3(256), 0, s, p->theta, p->m, p->v, p->grad,
                       p->np, lr, c1, c2, p->L, p->depth, p->width, p->d_wbf, p->d_wbft, p->d_wfr, p->d_wtfr);
    HCHK(hipGetLastError());
    return ME_OK;
}

int mlp_train_steps(me_mlp* p, const float* x, const float* t, const int32_t* idx, int64_t n, int64_t nsteps,
                    const float* lr_dev, float* loss_dev, void* stream) {
    if (!p || !x || !t || !lr_dev || nsteps < 0 || nsteps > INT32_MAX)
        return me_fail(ME_EINVAL, "mlp_train_steps: null argument or bad step count");
    if (nsteps == 0) return ME_OK;
    hipStream_t s = (hipStream_t)stream;
    if (fused_applies(p, n)) return fused_step(p, x, t, idx, n, nsteps, 0.f, lr_dev, loss_dev, nullptr, s);
    // layered path: one step at a time, rates read back first
    std::vector<float> lr((size_t)nsteps);
    HCHK(hipStreamSynchronize(s));
    HCHK(hipMemcpy(lr.data(), lr_dev, nsteps * sizeof(float), hipMemcpyDeviceToHost));
    for (int64_t st = 0; st < nsteps; ++st) {
        const int32_t* ix = idx ? idx + st * n : nullptr;
        const float* xs = idx ? x : x + st * n * p->n_in;
        const float* ts = idx ? t : t + st * n;
        const int rc = mlp_train_step(p, xs, ts, ix, n, lr[st], loss_dev ? loss_dev + st : nullptr, stream);
        if (rc != ME_OK) return rc;
    }
    return ME_OK;
}

int mlp_free(me_mlp* p) {
    if (!p) return ME_OK;
    (void)hipDeviceSynchronize();
    free_acts(p);
    auto f = [](void* q) {
        if (q) (void)hipFree(q);
    };
    f(p->theta);
    f(p->grad);
    f(p->dwpart);
    f(p->m);
    f(p->v);
    for (auto q : p->wbf) f(q);
    for (auto q : p->wbft) f(q);
    f(p->d_wbf);
    f(p->d_wbft);
    for (auto q : p->wfr) f(q);
    for (auto q : p->wtfr) f(q);
    f(p->d_wfr);
    f(p->d_wtfr);
    f(p->XT);
    f(p->HTb);
    f(p->DZTb);
    f(p->flossp);
    f(p->fopart);
    f(p->fbar);
    delete p;
    return ME_OK;
}

int me_features(const double* momenta, int64_t n, int npart, float* x, void* stream) {
    if (n < 0 || npart < 2 || npart > 8) return me_fail(ME_EINVAL, "me_features: bad size");
    if (n == 0) return ME_OK;
    if (!momenta || !x) return me_fail(ME_EINVAL, "me_features: null buffer");
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, momenta, n,
                       npart, x);
    HCHK(hipGetLastError());
    return ME_OK;
}

}  // extern "C"

// helper for the unweighting driver in me_unweight.hip
int mlp_forward_internal(me_mlp* p, const float* x, int64_t n, float* y, hipStream_t s) {
    return mlp_forward(p, x, n, y, s);
}
int mlp_n_in(const me_mlp* p) { return p->n_in; }
