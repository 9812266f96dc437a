// me_mixed.h -- the mixed-precision form of the matrix-element kernel.
//
// Amplitudes and wavefunctions in float32 (momentum algebra and propagator
// denominators stay float64); the colour sum J^dag N J is a dense GEMM on the
// matrix cores, batched over the 64 events of a wave: Z = A N with
// A = [Re J; Im J] (128 rows = 64 events x {re, im}, K = colour flows) carried
// as float16 hi + lo parts, N the exact integer colour numerators (exact in
// float16), accumulation in float32; then Q = sum_k A_k Z_k per event.
//
// Each event also gets an a-posteriori estimate of its relative rounding
// error: the float32 amplitudes contribute ~u32 times the magnitude sums
// S_k = sum |contributions to J_k| (cancellation between diagrams), carried
// through the colour form with Z = N J as 2 sum_k S_k |Z_k|; the colour GEMM
// adds its own hi/lo and accumulation terms (see the kernel).  Events above
// the tolerance are compacted into an index list for a float64 rerun.
#pragma once
#include "me_kernels.h"

// Waves per SIMD the mixed kernel is compiled for (register budget 512 / this).
#ifndef ME_MIXED_WAVES
#define ME_MIXED_WAVES 1
#endif

typedef _Float16 me_half8 __attribute__((ext_vector_type(8)));
typedef float me_float4 __attribute__((ext_vector_type(4)));

// Row tiles of 16 rows; each tile's LDS slot holds hi[16][NCOL] and
// lo[16][NCOL] float16 parts of A, later overwritten by Z[16][NCOL] float32.
template <int NCOL>
struct mfma_colour {
    // The matrix-core path needs a multiple of 8 colour flows (whole K groups
    // per lane); smaller processes sum colours on the VALU in float32.
    static constexpr bool enabled = (NCOL % 8 == 0);
    static constexpr int KS = (NCOL + 31) / 32;  // K steps of 32
    static constexpr int NT = (NCOL + 15) / 16;  // column tiles of 16
    static constexpr int MT = 8;                 // 128 rows
    static constexpr int TILE_BYTES = 16 * NCOL * 4;
    static constexpr int LDS_BYTES = enabled ? MT * TILE_BYTES : 16;
};

// B fragment of v_mfma_f32_16x16x32_f16 for K step ks, column tile n: lane l
// holds N[32 ks + 8 (l/16) + v][16 n + l%16], v = 0..7 (zero outside N).
template <class P>
MEV me_half8 colour_bfrag(int ks, int n, int lane) {
    me_half8 b;
    const int col = 16 * n + (lane & 15);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int k = 32 * ks + 8 * (lane >> 4) + v;
        b[v] = (k < P::ncol && col < P::ncol) ? (_Float16)colour_table<P>::get(k, col) : (_Float16)0;
    }
    return b;
}

// J^dag N J for the wave's 64 events (one per lane), on the matrix cores, in
// numerator units.  Also returns, from Z = N J, the two sums of the error
// estimate: zs = sum_k S_k (|Re Z_k| + |Im Z_k|) and zj = sum_k (|Re J_k||Re Z_k|
// + |Im J_k||Im Z_k|).  All 64 lanes must call it together.
template <class P>
MEV float colour_sum_mfma(const cx<float>* J, const float* S, char* lds, int lane, float& zs, float& zj) {
    using G = mfma_colour<P::ncol>;
    constexpr int NC = P::ncol;
    // per-event power-of-two scale: max |J s| < 2^14 keeps float16 in range
    float mx = 0.f;
#pragma unroll
    for (int k = 0; k < NC; ++k) mx = fmaxf(mx, fmaxf(fabsf(J[k].r), fabsf(J[k].i)));
    int e = 0;
    frexpf(mx, &e);
    const float s = (mx > 0.f) ? ldexpf(1.f, 14 - e) : 1.f;
    // rows: re of event e -> row e, im -> row 64 + e
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const int row = lane + 64 * part;
        char* tile = lds + (row >> 4) * G::TILE_BYTES;
        _Float16* hi = reinterpret_cast<_Float16*>(tile) + (row & 15) * NC;
        _Float16* lo = hi + 16 * NC;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const float v = (part ? J[k].i : J[k].r) * s;
            const _Float16 h = (_Float16)v;
            hi[k] = h;
            lo[k] = (_Float16)(v - (float)h);
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int t = 0; t < G::MT; ++t) {
        char* tile = lds + t * G::TILE_BYTES;
        const _Float16* hi = reinterpret_cast<const _Float16*>(tile);
        const _Float16* lo = hi + 16 * NC;
        me_half8 ahi[G::KS], alo[G::KS];
#pragma unroll
        for (int ks = 0; ks < G::KS; ++ks) {
            const int k0 = 32 * ks + 8 * (lane >> 4);
            if (k0 < NC) {
                ahi[ks] = *reinterpret_cast<const me_half8*>(hi + (lane & 15) * NC + k0);
                alo[ks] = *reinterpret_cast<const me_half8*>(lo + (lane & 15) * NC + k0);
            } else {
                ahi[ks] = me_half8{0, 0, 0, 0, 0, 0, 0, 0};
                alo[ks] = ahi[ks];
            }
        }
        me_float4 d[G::NT];
#pragma unroll
        for (int n = 0; n < G::NT; ++n) {
            me_float4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < G::KS; ++ks) {
                const me_half8 b = colour_bfrag<P>(ks, n, lane);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi[ks], b, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(alo[ks], b, acc, 0, 0, 0);
            }
            d[n] = acc;
        }
        // Z tile over the A tile (its fragments are in registers now):
        // lane holds Z[4 (l/16) + v][16 n + l%16]
        float* z = reinterpret_cast<float*>(tile);
#pragma unroll
        for (int n = 0; n < G::NT; ++n) {
            const int col = 16 * n + (lane & 15);
            if (col < NC) {
#pragma unroll
                for (int v = 0; v < 4; ++v) z[(4 * (lane >> 4) + v) * NC + col] = d[n][v];
            }
        }
    }
    __syncthreads();
    float q = 0.f, a = 0.f, b = 0.f;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const int row = lane + 64 * part;
        const float* z = reinterpret_cast<const float*>(lds + (row >> 4) * G::TILE_BYTES) + (row & 15) * NC;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const float j = (part ? J[k].i : J[k].r) * s;
            q = fmaf(j, z[k], q);
            a = fmaf(S[k], fabsf(z[k]), a);
            b = fmaf(fabsf(j), fabsf(z[k]), b);
        }
    }
    __syncthreads();  // the LDS slot is rewritten by the next helicity
    zs = a / s;
    zj = b / (s * s);
    return q / (s * s);
}

// Mixed kernel: out = float32-form |M|^2 (as float64); events whose error
// estimate exceeds tol are appended to flag_idx (wave-aggregated atomics on
// *flag_count).  err_out / flag_out (optional) receive the estimate and the
// decision per event.
template <class P>
__global__ __launch_bounds__(ME_BLOCK, ME_MIXED_WAVES) void k_me_gg_mixed(const double* __restrict__ mom, int64_t nevt,
                                                          double* __restrict__ out, const int* __restrict__ hels,
                                                          int nh, me_params prm, float tol, float cest,
                                                          int* __restrict__ flag_count, int* __restrict__ flag_idx,
                                                          float* __restrict__ err_out,
                                                          unsigned char* __restrict__ flag_out) {
    static_assert(ME_BLOCK == 64, "one wave per block");
    __shared__ __attribute__((aligned(16))) char lds[mfma_colour<P::ncol>::LDS_BYTES];
    const int lane = threadIdx.x;
    int64_t ev = (int64_t)blockIdx.x * ME_BLOCK + lane;
    const bool valid = ev < nevt;
    if (!valid) ev = nevt - 1;  // every lane takes part in the wave-wide colour GEMM
    using T = float;
    constexpr int NG = P::ngluon;
    __shared__ double Qt[ME_MOM_ROW(NG + 2)];
    gg_ext<T, NG> x;
    gg_setup<P, T>(x, mom, ev, Qt, lane, prm);
    float acc = 0.f, dacc = 0.f;
#pragma unroll 1
    for (int ih = 0; ih < nh; ++ih) {
        const int h = hels[ih];
        gg_externals<P, T>(x, h);
        cx<T> J[P::ncol];
        T S[P::ncol];
#pragma unroll
        for (int k = 0; k < P::ncol; ++k) {
            J[k] = mk(T(0), T(0));
            S[k] = T(0);
        }
        P::template amps_f32<T, true>(x, J, S);
        float jn2 = 0.f, sn2 = 0.f;
#pragma unroll
        for (int k = 0; k < P::ncol; ++k) {
            jn2 = fmaf(J[k].r, J[k].r, fmaf(J[k].i, J[k].i, jn2));
            sn2 = fmaf(S[k], S[k], sn2);
        }
        constexpr float u32 = 5.9604645e-8f;  // 2^-24
        if constexpr (mfma_colour<P::ncol>::enabled) {
            // amplitude rounding: |dJ_k| ~ c u32 S_k, so |dQ| <= 2 c u32 sum_k S_k |Z_k|;
            // colour GEMM: float16 hi+lo carries J to 2^-22 per element, float32
            // accumulation adds ~sqrt(K) u32 |J|^T |N| |J|
            float zs, zj;
            acc += colour_sum_mfma<P>(J, S, lds, lane, zs, zj);
            dacc += 2.f * cest * u32 * zs + 2.f * 2.3841858e-7f * zj +
                    sqrtf(float(P::ncol)) * u32 * float(P::abs_lambda_max) * jn2;
        } else {
            acc += P::template colour_sum<T>(J);
            dacc += 2.f * cest * u32 * float(P::abs_lambda_max) * sqrtf(jn2 * sn2);
        }
    }
    const double me2 = double(acc) * (1.0 / (256.0 * P::identical * P::lcd));
    const float est = dacc / acc;
    const bool flag = valid && !(est <= tol);  // NaN estimates are flagged too
    if (valid) {
        out[ev] = me2;
        if (err_out) err_out[ev] = est;
        if (flag_out) flag_out[ev] = flag ? 1 : 0;
    }
    if (flag_idx) {
        const unsigned long long ballot = __ballot(flag);
        if (ballot) {
            const int nflag = __popcll(ballot);
            int base = 0;
            const int leader = __ffsll((long long)ballot) - 1;
            if (lane == leader) base = atomicAdd(flag_count, nflag);
            base = __shfl(base, leader);
            if (flag) {
                const unsigned long long below = ballot & ((1ull << lane) - 1ull);
                flag_idx[base + __popcll(below)] = (int)ev;
            }
        }
    }
}

static __global__ void k_zero_int(int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}
