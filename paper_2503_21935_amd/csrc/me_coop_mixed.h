// me_coop_mixed.h -- the mixed-precision form of the workgroup kernel
// (g g -> t tbar g g g).
//
// The tile of 64 events is shared by the four waves as in k_me_gg_coop, with
// the amplitude program in float32 (momentum algebra and propagator
// denominators in float64).  J is accumulated in LDS in float32, together with
// S_k = sum of |contributions to J_k| for the error estimate.  The colour sum
// of a helicity is one GEMM per wave on the matrix cores: wave w takes events
// 16w..16w+15 as two 16-row tiles (Re J and Im J), A carried as float16 hi + lo
// with a per-event power-of-two scale, B = the integer colour numerators
// (exact in float16), float32 accumulation; then Q = sum_k A_k Z_k per row.
// The per-event error estimate is the one of k_me_gg_mixed:
//   est = sum_h [2 c u32 sum_k S_k |Z_k| + 2 2^-22 sum_k |J_k||Z_k|
//                + sqrt(ncol) u32 lambda_max(|N|) |J|^2] / sum_h Q,
// and events above the tolerance are compacted for a float64 rerun.
#pragma once
#include "me_coop.h"
#include "me_mixed.h"

template <class P>
__global__ __launch_bounds__(ME_TILE * P::waves, 1) void k_me_gg_coop_mixed(
    const double* __restrict__ mom, int64_t nevt, double* __restrict__ out, const int* __restrict__ hels, int nh,
    me_params prm, float tol, float cest, int* __restrict__ flag_count, int* __restrict__ flag_idx,
    float* __restrict__ err_out, unsigned char* __restrict__ flag_out) {
    constexpr int NP = P::npart, NG = P::ngluon, NC = P::ncol;
    constexpr int KS = (NC + 31) / 32, NT = (NC + 15) / 16;
    static_assert(P::waves * 16 == ME_TILE, "each wave takes 16 events of the tile in the colour GEMM");
    __shared__ float Jt[NC * 2 * ME_TILE];
    __shared__ float St[NC * ME_TILE];
    __shared__ double Qt[(NG + 2) * 4 * ME_TILE];
    __shared__ float rowres[3 * 2 * ME_TILE];  // [q, zs, zj][re, im][event]
    __shared__ float jnorm[ME_TILE];
    const int lane = threadIdx.x % ME_TILE;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / ME_TILE);
    const int64_t first = (int64_t)blockIdx.x * ME_TILE;
    if (first >= nevt) return;  // whole block
    int64_t ev = first + lane;
    const bool valid = ev < nevt;
    if (!valid) ev = nevt - 1;  // idle lanes repeat an event so that every wave runs the full program
    if (wave == 0) {
        const double2* pe = reinterpret_cast<const double2*>(mom + ev * (NP * 4));
#pragma unroll
        for (int r = 0; r < NG + 2; ++r) {
            const int ip = (r < 2) ? r : (r < NG) ? r + 2 : r - NG + 2;
            const double sg = (r >= 2 && r < NG) ? -1.0 : 1.0;
            const double2 a = pe[2 * ip], b = pe[2 * ip + 1];
            Qt[(4 * r + 0) * ME_TILE + lane] = sg * a.x;
            Qt[(4 * r + 1) * ME_TILE + lane] = sg * a.y;
            Qt[(4 * r + 2) * ME_TILE + lane] = sg * b.x;
            Qt[(4 * r + 3) * ME_TILE + lane] = sg * b.y;
        }
    }
    __syncthreads();
    using T = float;
    coop_ext<T, NG> x;
    x.m = prm.mt;
    x.mw = prm.mt * prm.wt;
    x.g = prm.gs;
    x.mT = T(prm.mt);
    x.gT = T(prm.gs);
    x.Q = (lds_cdouble*)(Qt + lane);
#pragma unroll
    for (int j = 0; j < NG; ++j) x.qo[j] = 4 * ME_TILE * P::perm(wave, j);
    x.qo[NG] = 4 * ME_TILE * NG;
    x.qo[NG + 1] = 4 * ME_TILE * (NG + 1);
    static_assert(NC <= 2 * ME_TILE, "flow map held in two registers");
    const int* fm = coop_table<P>::fmap(wave);
    const int fm0 = fm[lane];
    const int fm1 = (lane + ME_TILE < NC) ? fm[lane + ME_TILE] : 0;
    int wsel = wave;
    asm volatile("" : "+v"(wsel));
    const uint4* bfrag = reinterpret_cast<const uint4*>(coop_table<P>::bfrag());
    constexpr float u32 = 5.9604645e-8f;  // 2^-24
    const int i16 = lane & 15, g4 = lane >> 4;
    float acc = 0.f, dacc = 0.f;  // per event, held by wave 0
#pragma unroll 1
    for (int ih = 0; ih < nh; ++ih) {
        const int h = hels[ih];
        for (int e = threadIdx.x; e < NC * 2 * ME_TILE; e += ME_TILE * P::waves) Jt[e] = 0.f;
        for (int e = threadIdx.x; e < NC * ME_TILE; e += ME_TILE * P::waves) St[e] = 0.f;
        __syncthreads();
        coop_externals<P, T>(x, h, wave);
        P::template amps_wave<T, true>(x, Jt + lane, St + lane, fm0, fm1, wsel);
        __syncthreads();
        // ---- colour GEMM of this wave's 16 events --------------------------------
        const int ea = 16 * wave + i16;  // event of this lane's A row
        float mx = 0.f, n2 = 0.f;
        for (int k = g4; k < NC; k += 4) {
            const float re = Jt[(2 * k) * ME_TILE + ea], im = Jt[(2 * k + 1) * ME_TILE + ea];
            mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
            n2 = fmaf(re, re, fmaf(im, im, n2));
        }
        mx = fmaxf(mx, __shfl_xor(mx, 16));
        mx = fmaxf(mx, __shfl_xor(mx, 32));
        n2 += __shfl_xor(n2, 16);
        n2 += __shfl_xor(n2, 32);
        int ex = 0;
        frexpf(mx, &ex);
        const float sc = (mx > 0.f) ? ldexpf(1.f, 14 - ex) : 1.f;  // max |J sc| < 2^14
        if (g4 == 0) jnorm[ea] = n2;
        me_float4 d[2][NT];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int t = 0; t < NT; ++t) d[rt][t] = me_float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            me_half8 ahi[2], alo[2];
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const int k = 32 * ks + 8 * g4 + v;
                    const float a = (k < NC) ? Jt[(2 * k + rt) * ME_TILE + ea] * sc : 0.f;
                    const _Float16 hi = (_Float16)a;
                    ahi[rt][v] = hi;
                    alo[rt][v] = (_Float16)(a - (float)hi);
                }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const uint4 bw = bfrag[(ks * NT + t) * 64 + lane];
                me_half8 b;
                __builtin_memcpy(&b, &bw, sizeof(b));
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) {
                    d[rt][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi[rt], b, d[rt][t], 0, 0, 0);
                    d[rt][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(alo[rt], b, d[rt][t], 0, 0, 0);
                }
            }
        }
        // lane holds Z[row 4 g4 + v][col 16 t + i16] (scaled by the row event's sc)
        float part[3][2][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ez = 16 * wave + 4 * g4 + v;           // event of row 4 g4 + v
            const float inv = 1.f / __shfl(sc, 4 * g4 + v);  // that event's scale, held by lane 4 g4 + v
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                float q = 0.f, zs = 0.f, zj = 0.f;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int k = 16 * t + i16;
                    if (k < NC) {
                        const float z = d[rt][t][v] * inv;  // numerator units
                        const float jv = Jt[(2 * k + rt) * ME_TILE + ez];
                        q = fmaf(jv, z, q);
                        zs = fmaf(St[k * ME_TILE + ez], fabsf(z), zs);
                        zj = fmaf(fabsf(jv), fabsf(z), zj);
                    }
                }
                part[0][rt][v] = q;
                part[1][rt][v] = zs;
                part[2][rt][v] = zj;
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float a = part[c][rt][v];
                    a += __shfl_xor(a, 1);
                    a += __shfl_xor(a, 2);
                    a += __shfl_xor(a, 4);
                    a += __shfl_xor(a, 8);
                    if (i16 == 0) rowres[(c * 2 + rt) * ME_TILE + 16 * wave + 4 * g4 + v] = a;
                }
        __syncthreads();
        if (wave == 0) {
            const float q = rowres[0 * ME_TILE + lane] + rowres[1 * ME_TILE + lane];
            const float zs = rowres[2 * ME_TILE + lane] + rowres[3 * ME_TILE + lane];
            const float zj = rowres[4 * ME_TILE + lane] + rowres[5 * ME_TILE + lane];
            acc += q;
            dacc += 2.f * cest * u32 * zs + 2.f * 2.3841858e-7f * zj +
                    sqrtf(float(NC)) * u32 * float(P::abs_lambda_max) * jnorm[lane];
        }
        __syncthreads();
    }
    if (wave != 0) return;  // uniform per wave; no barrier follows
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
