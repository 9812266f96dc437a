// ps_rambo.hip -- flat phase-space points on the GPU: counter-based random
// numbers and the RAMBO map, one event per lane (the first two of the
// generator's three per-event steps, random numbers -> momenta -> matrix
// element, paper Sec. 2; its outlook, Sec. 3, names data-parallel phase-space
// sampling as the next step to move to the GPU).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
// the 64-bit seed, counter = (event, block b, 0); block b yields uniforms 2b
// and 2b + 1, each from 64 bits as ((hi:lo) >> 11 + 1/2) 2^-53 in (0, 1).
// Momenta: RAMBO (Kleiss, Stirling, Ellis 1986): isotropic massless q_i with
// energy density q0 e^-q0, conformally mapped to total (sqrt s, 0); masses by
// rescaling the 3-momenta with the xi that restores the total energy, and the
// corresponding weight.  The lane's momenta are assembled in LDS and each
// block writes its events' [npart][4] rows back as one contiguous, coalesced
// range.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/ps.h"
#include "me_internal.h"

#define PS_BLOCK 128
#define PS_MAXF 8  // final-state particles per event

struct ps_masses {
    double m[PS_MAXF];
};

struct philox_out {
    uint32_t x[4];
};

// Philox4x32-10: ten rounds of two 32 x 32 -> 64 bit products and a word
// exchange, the key advanced by the golden-ratio Weyl increments between rounds.
__device__ __forceinline__ philox_out philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                    uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return philox_out{{c0, c1, c2, c3}};
}

__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo) {
    const uint64_t v = ((uint64_t(hi) << 32) | lo) >> 11;
    return (double(v) + 0.5) * (1.0 / 9007199254740992.0);
}

// Events first .. first + nevt - 1 of the stream; momenta [nevt][NF + 2][4].
template <int NF>
__global__ __launch_bounds__(PS_BLOCK) void k_ps_rambo(double roots, ps_masses ms, int massive, double w0,
                                                       uint64_t seed, int64_t first, int64_t nevt,
                                                       double* __restrict__ mom, double* __restrict__ wt) {
    constexpr int NP = NF + 2, ROW = NP * 4;
    __shared__ double tile[PS_BLOCK * ROW];
    const int64_t e0 = (int64_t)blockIdx.x * PS_BLOCK;
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const uint64_t ctr = (uint64_t)(first + e);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    double q[NF][4], Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const philox_out a = philox4x32_10((uint32_t)ctr, (uint32_t)(ctr >> 32), 2 * i, 0u, k0, k1);
        const philox_out b = philox4x32_10((uint32_t)ctr, (uint32_t)(ctr >> 32), 2 * i + 1, 0u, k0, k1);
        const double c = 2.0 * u53(a.x[0], a.x[1]) - 1.0;
        const double phi = 2.0 * M_PI * u53(a.x[2], a.x[3]);
        const double q0 = -log(u53(b.x[0], b.x[1]) * u53(b.x[2], b.x[3]));
        const double st = sqrt(1.0 - c * c);
        double sp, cp;
        sincos(phi, &sp, &cp);
        q[i][0] = q0;
        q[i][1] = q0 * st * cp;
        q[i][2] = q0 * st * sp;
        q[i][3] = q0 * c;
#pragma unroll
        for (int k = 0; k < 4; ++k) Q[k] += q[i][k];
    }
    const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
    const double b1 = -Q[1] / M, b2 = -Q[2] / M, b3 = -Q[3] / M;
    const double x = roots / M, gam = Q[0] / M, a = 1.0 / (1.0 + gam);
    double p[NF][4];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const double bq = b1 * q[i][1] + b2 * q[i][2] + b3 * q[i][3];
        p[i][0] = x * (gam * q[i][0] + bq);
        p[i][1] = x * (q[i][1] + b1 * q[i][0] + a * bq * b1);
        p[i][2] = x * (q[i][2] + b2 * q[i][0] + a * bq * b2);
        p[i][3] = x * (q[i][3] + b3 * q[i][0] + a * bq * b3);
    }
    double xi = 1.0, w = w0;
    if (massive) {
        // sum_i sqrt(m_i^2 + xi^2 P_i^2) = roots: increasing in xi, negative at 0,
        // non-negative at 1; Newton steps kept inside the bracket
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 200; ++it) {
            double f = -roots, df = 0.0;
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                const double en = sqrt(ms.m[i] * ms.m[i] + xi * xi * p[i][0] * p[i][0]);
                f += en;
                df += xi * p[i][0] * p[i][0] / en;
            }
            if (f > 0.0) hi = xi;
            else lo = xi;
            double nx = xi - f / df;
            if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
            const bool done = fabs(nx - xi) <= 1e-16 * xi;
            xi = nx;
            if (done) break;
        }
    }
    double sk = 0.0, pr = 1.0, sk2 = 0.0;
    double* row = tile + t * ROW;
    row[0] = 0.5 * roots, row[1] = 0.0, row[2] = 0.0, row[3] = 0.5 * roots;
    row[4] = 0.5 * roots, row[5] = 0.0, row[6] = 0.0, row[7] = -0.5 * roots;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const double kx = xi * p[i][1], ky = xi * p[i][2], kz = xi * p[i][3];
        const double kk = sqrt(kx * kx + ky * ky + kz * kz);
        const double en = sqrt(ms.m[i] * ms.m[i] + kk * kk);  // on shell by construction
        row[4 * (i + 2) + 0] = en;
        row[4 * (i + 2) + 1] = kx;
        row[4 * (i + 2) + 2] = ky;
        row[4 * (i + 2) + 3] = kz;
        sk += kk;
        pr *= kk / en;
        sk2 += kk * kk / en;
    }
    if (massive) w = w0 * pow(sk / roots, 2 * NF - 3) * pr * roots / sk2;
    if (wt && e < nevt) wt[e] = w;
    __syncthreads();
    // coalesced write-back of the block's rows (double2 granules)
    const int64_t nb = (nevt - e0 < PS_BLOCK) ? (nevt - e0) : PS_BLOCK;
    const int total2 = (int)(nb * ROW / 2);
    const double2* src = reinterpret_cast<const double2*>(tile);
    double2* dst = reinterpret_cast<double2*>(mom + e0 * ROW);
    for (int j = t; j < total2; j += PS_BLOCK) dst[j] = src[j];
}

// ---------------------------------------------------------------------------
// Multi-channel sampling for a final state with a lepton pair (a, b): channel
// 0 flat RAMBO over the NF particles; channel 1 the pair's M^2 from a
// Breit-Wigner of (MZ, WZ) on [mlo^2, mhi^2] (arctangent map), channel 2 from
// 1/M^2 on the same window (logarithmic map); for both, RAMBO over NF - 1
// bodies (the pair as one particle of mass M first, the others in order) and
// an isotropic decay of the pair in its rest frame.  dPhi_n = dPhi_{n-1}
// dQ^2/(2 pi) dPhi_2 gives each channel's density from the final momenta,
//   g_0 = 1/V_n,  g_c = 2 pi p_c(M^2) / (w_R(x') Phi_2),  Phi_2 = 1/(8 pi),
// w_R(x') the massive RAMBO weight of the (n-1)-body configuration, and each
// point carries 1 / sum_c alpha_c g_c.  Uniforms: 4 per RAMBO particle as in
// k_ps_rambo; block 16 picks the channel and maps M^2, block 17 the decay.
// ---------------------------------------------------------------------------
struct ps_mc_args {
    double roots, a2, b2, mz, wz, bw_lo, bw_hi;
    double alpha[3];
    double vn;      // massless n-body volume
    double w0m1;    // massless (n-1)-body volume (RAMBO weight before the mass factor)
    int ia, ib;
};

// RAMBO over the first nb of NB bodies from the event's Philox stream
// (particle i: blocks 2i, 2i + 1), mass m0 on body 0 (0: all massless);
// bodies nb .. NB - 1 are left zero.  One code path for every channel, so
// that lanes of one wave in different channels do not run two RAMBO stages.
template <int NB>
__device__ __forceinline__ void rambo_active(double roots, double m0, int nb, uint64_t ctr, uint32_t k0,
                                             uint32_t k1, double (&p)[NB][4]) {
    double q[NB][4], Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        q[i][0] = q[i][1] = q[i][2] = q[i][3] = 0.0;
        if (i < nb) {
            const philox_out a = philox4x32_10((uint32_t)ctr, (uint32_t)(ctr >> 32), 2 * i, 0u, k0, k1);
            const philox_out b = philox4x32_10((uint32_t)ctr, (uint32_t)(ctr >> 32), 2 * i + 1, 0u, k0, k1);
            const double c = 2.0 * u53(a.x[0], a.x[1]) - 1.0;
            const double phi = 2.0 * M_PI * u53(a.x[2], a.x[3]);
            const double q0 = -log(u53(b.x[0], b.x[1]) * u53(b.x[2], b.x[3]));
            const double st = sqrt(1.0 - c * c);
            double sp, cp;
            sincos(phi, &sp, &cp);
            q[i][0] = q0;
            q[i][1] = q0 * st * cp;
            q[i][2] = q0 * st * sp;
            q[i][3] = q0 * c;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) Q[k] += q[i][k];
    }
    const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
    const double b1 = -Q[1] / M, b2 = -Q[2] / M, b3 = -Q[3] / M;
    const double x = roots / M, gam = Q[0] / M, a = 1.0 / (1.0 + gam);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const double bq = b1 * q[i][1] + b2 * q[i][2] + b3 * q[i][3];
        p[i][0] = x * (gam * q[i][0] + bq);
        p[i][1] = x * (q[i][1] + b1 * q[i][0] + a * bq * b1);
        p[i][2] = x * (q[i][2] + b2 * q[i][0] + a * bq * b2);
        p[i][3] = x * (q[i][3] + b3 * q[i][0] + a * bq * b3);
    }
    double xi = 1.0;
    if (m0 > 0.0) {
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 200; ++it) {
            double f = -roots, df = 0.0;
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                if (i < nb) {
                    const double mi = (i == 0) ? m0 : 0.0;
                    const double en = sqrt(mi * mi + xi * xi * p[i][0] * p[i][0]);
                    f += en;
                    df += xi * p[i][0] * p[i][0] / en;
                }
            }
            if (f > 0.0) hi = xi;
            else lo = xi;
            double nx = xi - f / df;
            if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
            const bool done = fabs(nx - xi) <= 1e-16 * xi;
            xi = nx;
            if (done) break;
        }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const double mi = (i == 0) ? m0 : 0.0;
        p[i][1] *= xi;
        p[i][2] *= xi;
        p[i][3] *= xi;
        const double kk = sqrt(p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]);
        p[i][0] = (m0 > 0.0) ? sqrt(mi * mi + kk * kk) : kk;
    }
}

template <int NF>
__global__ __launch_bounds__(PS_BLOCK) void k_ps_mc(ps_mc_args g, uint64_t seed, int64_t first, int64_t nevt,
                                                    double* __restrict__ mom, double* __restrict__ wt,
                                                    int32_t* __restrict__ chan) {
    constexpr int NP = NF + 2, ROW = NP * 4;
    __shared__ double tile[PS_BLOCK * ROW];
    const int64_t e0 = (int64_t)blockIdx.x * PS_BLOCK;
    const int t = threadIdx.x;
    const int64_t e = e0 + t;
    const uint64_t ctr = (uint64_t)(first + e);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const philox_out x16 = philox4x32_10((uint32_t)ctr, (uint32_t)(ctr >> 32), 16u, 0u, k0, k1);
    const double uc = u53(x16.x[0], x16.x[1]), um = u53(x16.x[2], x16.x[3]);
    const int c = (uc < g.alpha[0]) ? 0 : (uc < g.alpha[0] + g.alpha[1]) ? 1 : 2;
    // channels 1, 2: the pair's mass from its map, RAMBO over NF - 1 bodies
    double M = 0.0;
    if (c != 0) {
        const double m2 = (c == 1) ? g.mz * g.mz + g.mz * g.wz * tan(g.bw_lo + um * (g.bw_hi - g.bw_lo))
                                   : g.a2 * pow(g.b2 / g.a2, um);
        M = sqrt(m2);
    }
    double p[NF][4];
    rambo_active<NF>(g.roots, M, (c == 0) ? NF : NF - 1, ctr, k0, k1, p);
    double f[NF][4];
    if (c == 0) {
#pragma unroll
        for (int i = 0; i < NF; ++i)
#pragma unroll
            for (int kx = 0; kx < 4; ++kx) f[i][kx] = p[i][kx];
    } else {
        // isotropic decay of the pair (body 0, mass M) in its rest frame
        const philox_out x17 = philox4x32_10((uint32_t)ctr, (uint32_t)(ctr >> 32), 17u, 0u, k0, k1);
        const double ct = 2.0 * u53(x17.x[0], x17.x[1]) - 1.0, ph = 2.0 * M_PI * u53(x17.x[2], x17.x[3]);
        const double st = sqrt(1.0 - ct * ct);
        double sp, cp;
        sincos(ph, &sp, &cp);
        const double es = 0.5 * M;
        const double ks1 = es * st * cp, ks2 = es * st * sp, ks3 = es * ct;
        const double pk = p[0][1] * ks1 + p[0][2] * ks2 + p[0][3] * ks3;
        const double ea = (p[0][0] * es + pk) / M;
        const double fac = (ea + es) / (p[0][0] + M);
        double pa[4] = {ea, ks1 + fac * p[0][1], ks2 + fac * p[0][2], ks3 + fac * p[0][3]};
        double pb[4] = {p[0][0] - pa[0], p[0][1] - pa[1], p[0][2] - pa[2], p[0][3] - pa[3]};
        // massless products: energies from the 3-momenta
        pa[0] = sqrt(pa[1] * pa[1] + pa[2] * pa[2] + pa[3] * pa[3]);
        pb[0] = sqrt(pb[1] * pb[1] + pb[2] * pb[2] + pb[3] * pb[3]);
        // the other finals keep their order: final i takes body j, counting
        // up from 1 over the finals that are not in the pair
        int j = 1;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
#pragma unroll
            for (int kx = 0; kx < 4; ++kx) {
                double v = 0.0;
#pragma unroll
                for (int jj = 1; jj < NF - 1; ++jj) v = (jj == j) ? p[jj][kx] : v;
                f[i][kx] = (i == g.ia) ? pa[kx] : (i == g.ib) ? pb[kx] : v;
            }
            if (i != g.ia && i != g.ib) ++j;
        }
    }
    // the multi-channel weight from the final momenta
    double gsum = g.alpha[0] / g.vn;
    double fa[4], fb[4];
#pragma unroll
    for (int kx = 0; kx < 4; ++kx) {
        fa[kx] = 0.0, fb[kx] = 0.0;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            fa[kx] = (i == g.ia) ? f[i][kx] : fa[kx];
            fb[kx] = (i == g.ib) ? f[i][kx] : fb[kx];
        }
    }
    const double P0 = fa[0] + fb[0], P1 = fa[1] + fb[1], P2 = fa[2] + fb[2], P3 = fa[3] + fb[3];
    const double m2 = P0 * P0 - P1 * P1 - P2 * P2 - P3 * P3;
    if (m2 >= g.a2 && m2 <= g.b2 && (g.alpha[1] > 0.0 || g.alpha[2] > 0.0)) {
        // massive RAMBO weight of (pair, others) from the momenta alone
        double kk = sqrt(P1 * P1 + P2 * P2 + P3 * P3);
        double sk = kk, pr = kk / P0, sk2 = kk * kk / P0;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            if (i == g.ia || i == g.ib) continue;
            const double ki = sqrt(f[i][1] * f[i][1] + f[i][2] * f[i][2] + f[i][3] * f[i][3]);
            sk += ki;
            pr *= ki / f[i][0];
            sk2 += ki * ki / f[i][0];
        }
        const double wr = g.w0m1 * pow(sk / g.roots, 2 * (NF - 1) - 3) * pr * g.roots / sk2;
        const double mw = g.mz * g.wz, d = m2 - g.mz * g.mz;
        const double p_bw = mw / (d * d + mw * mw) / (g.bw_hi - g.bw_lo);
        const double p_ph = 1.0 / (m2 * log(g.b2 / g.a2));
        // 2 pi p / (w_R Phi_2) with Phi_2 = 1/(8 pi)
        gsum += (g.alpha[1] * p_bw + g.alpha[2] * p_ph) * (16.0 * M_PI * M_PI) / wr;
    }
    if (e < nevt) {
        if (wt) wt[e] = 1.0 / gsum;
        if (chan) chan[e] = c;
    }
    double* row = tile + t * ROW;
    row[0] = 0.5 * g.roots, row[1] = 0.0, row[2] = 0.0, row[3] = 0.5 * g.roots;
    row[4] = 0.5 * g.roots, row[5] = 0.0, row[6] = 0.0, row[7] = -0.5 * g.roots;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int kx = 0; kx < 4; ++kx) row[4 * (i + 2) + kx] = f[i][kx];
    __syncthreads();
    const int64_t nb = (nevt - e0 < PS_BLOCK) ? (nevt - e0) : PS_BLOCK;
    const int total2 = (int)(nb * ROW / 2);
    const double2* src = reinterpret_cast<const double2*>(tile);
    double2* dst = reinterpret_cast<double2*>(mom + e0 * ROW);
    for (int j = t; j < total2; j += PS_BLOCK) dst[j] = src[j];
}

template <int NF>
static hipError_t launch(double roots, const ps_masses& ms, int massive, double w0, uint64_t seed, int64_t first,
                         int64_t nevt, double* mom, double* wt, hipStream_t s) {
    const dim3 grid((unsigned)((nevt + PS_BLOCK - 1) / PS_BLOCK));
    hipLaunchKernelGGL(k_ps_rambo<NF>, grid, dim3(PS_BLOCK), 0, s, roots, ms, massive, w0, seed, first, nevt, mom,
                       wt);
    return hipGetLastError();
}

extern "C" int ps_rambo(double roots, const double* masses, int nfinal, uint64_t seed, int64_t first_event,
                        int64_t nevt, double* momenta, double* weights, void* stream) {
    if (nfinal < 2 || nfinal > PS_MAXF) return me_fail(ME_EINVAL, "ps_rambo: nfinal must be 2..8");
    if (!(roots > 0) || nevt < 0 || first_event < 0) return me_fail(ME_EINVAL, "ps_rambo: bad roots or sizes");
    if (nevt == 0) return ME_OK;
    if (!momenta || !masses) return me_fail(ME_EINVAL, "ps_rambo: null buffer");
    if (reinterpret_cast<uintptr_t>(momenta) % 16) return me_fail(ME_EINVAL, "ps_rambo: momenta not 16-byte aligned");
    ps_masses ms{};
    double msum = 0.0;
    int massive = 0;
    for (int i = 0; i < nfinal; ++i) {
        if (!(masses[i] >= 0)) return me_fail(ME_EINVAL, "ps_rambo: negative mass");
        ms.m[i] = masses[i];
        msum += masses[i];
        massive |= masses[i] != 0.0;
    }
    if (!(msum < roots)) return me_fail(ME_EINVAL, "ps_rambo: masses above sqrt(s)");
    // flat n-body volume (2 pi)^(4 - 3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!)
    const int n = nfinal;
    double f1 = 1.0, f2 = 1.0;
    for (int i = 2; i <= n - 1; ++i) f1 *= i;
    for (int i = 2; i <= n - 2; ++i) f2 *= i;
    const double s = roots * roots;
    const double w0 = std::pow(2 * M_PI, 4 - 3 * n) * std::pow(M_PI / 2, n - 1) * std::pow(s, n - 2) / (f1 * f2);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    switch (nfinal) {
        case 2: e = launch<2>(roots, ms, massive, w0, seed, first_event, nevt, momenta, weights, st); break;
        case 3: e = launch<3>(roots, ms, massive, w0, seed, first_event, nevt, momenta, weights, st); break;
        case 4: e = launch<4>(roots, ms, massive, w0, seed, first_event, nevt, momenta, weights, st); break;
        case 5: e = launch<5>(roots, ms, massive, w0, seed, first_event, nevt, momenta, weights, st); break;
        case 6: e = launch<6>(roots, ms, massive, w0, seed, first_event, nevt, momenta, weights, st); break;
        case 7: e = launch<7>(roots, ms, massive, w0, seed, first_event, nevt, momenta, weights, st); break;
        default: e = launch<8>(roots, ms, massive, w0, seed, first_event, nevt, momenta, weights, st); break;
    }
    if (e != hipSuccess) return me_fail(ME_EDEVICE, std::string("ps_rambo launch: ") + hipGetErrorString(e));
    return ME_OK;
}

template <int NF>
static hipError_t launch_mc(const ps_mc_args& g, uint64_t seed, int64_t first, int64_t nevt, double* mom, double* wt,
                            int32_t* ch, hipStream_t s) {
    const dim3 grid((unsigned)((nevt + PS_BLOCK - 1) / PS_BLOCK));
    hipLaunchKernelGGL(k_ps_mc<NF>, grid, dim3(PS_BLOCK), 0, s, g, seed, first, nevt, mom, wt, ch);
    return hipGetLastError();
}

extern "C" int ps_multichannel(double roots, int nfinal, int pair_a, int pair_b, double mlo, double mhi, double mz,
                               double wz, const double* alpha, uint64_t seed, int64_t first_event, int64_t nevt,
                               double* momenta, double* weights, int32_t* channels, void* stream) {
    if (nfinal < 3 || nfinal > PS_MAXF) return me_fail(ME_EINVAL, "ps_multichannel: nfinal must be 3..8");
    if (pair_a < 0 || pair_b < 0 || pair_a >= nfinal || pair_b >= nfinal || pair_a == pair_b)
        return me_fail(ME_EINVAL, "ps_multichannel: bad pair");
    if (!(roots > 0) || nevt < 0 || first_event < 0) return me_fail(ME_EINVAL, "ps_multichannel: bad roots or sizes");
    if (!(mlo > 0) || !(mhi > mlo) || !(mhi <= roots) || !(mz > 0) || !(wz > 0))
        return me_fail(ME_EINVAL, "ps_multichannel: bad mass window or resonance");
    if (!alpha) return me_fail(ME_EINVAL, "ps_multichannel: null alpha");
    const double at = alpha[0] + alpha[1] + alpha[2];
    if (!(alpha[0] >= 0 && alpha[1] >= 0 && alpha[2] >= 0 && at > 0))
        return me_fail(ME_EINVAL, "ps_multichannel: channel weights must be >= 0 with a positive sum");
    if (nevt == 0) return ME_OK;
    if (!momenta) return me_fail(ME_EINVAL, "ps_multichannel: null buffer");
    if (reinterpret_cast<uintptr_t>(momenta) % 16)
        return me_fail(ME_EINVAL, "ps_multichannel: momenta not 16-byte aligned");
    ps_mc_args g{};
    g.roots = roots;
    g.a2 = mlo * mlo;
    g.b2 = mhi * mhi;
    g.mz = mz;
    g.wz = wz;
    g.bw_lo = std::atan((g.a2 - mz * mz) / (mz * wz));
    g.bw_hi = std::atan((g.b2 - mz * mz) / (mz * wz));
    for (int c = 0; c < 3; ++c) g.alpha[c] = alpha[c] / at;
    auto volume = [&](int n) {
        double f1 = 1.0, f2 = 1.0;
        for (int i = 2; i <= n - 1; ++i) f1 *= i;
        for (int i = 2; i <= n - 2; ++i) f2 *= i;
        const double s = roots * roots;
        return std::pow(2 * M_PI, 4 - 3 * n) * std::pow(M_PI / 2, n - 1) * std::pow(s, n - 2) / (f1 * f2);
    };
    g.vn = volume(nfinal);
    g.w0m1 = volume(nfinal - 1);
    g.ia = pair_a;
    g.ib = pair_b;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    switch (nfinal) {
        case 3: e = launch_mc<3>(g, seed, first_event, nevt, momenta, weights, channels, st); break;
        case 4: e = launch_mc<4>(g, seed, first_event, nevt, momenta, weights, channels, st); break;
        case 5: e = launch_mc<5>(g, seed, first_event, nevt, momenta, weights, channels, st); break;
        case 6: e = launch_mc<6>(g, seed, first_event, nevt, momenta, weights, channels, st); break;
        case 7: e = launch_mc<7>(g, seed, first_event, nevt, momenta, weights, channels, st); break;
        default: e = launch_mc<8>(g, seed, first_event, nevt, momenta, weights, channels, st); break;
    }
    if (e != hipSuccess) return me_fail(ME_EDEVICE, std::string("ps_multichannel launch: ") + hipGetErrorString(e));
    return ME_OK;
}
