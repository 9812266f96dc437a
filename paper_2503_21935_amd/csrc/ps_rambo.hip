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
