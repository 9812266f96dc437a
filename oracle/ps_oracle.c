/*
 * ps_oracle.c -- CPU oracle of the phase-space sampling step (test
 * infrastructure only; never linked into or called by the product library).
 *
 * The paper's generator draws random numbers, maps them to momenta and then
 * evaluates the matrix element (Sec. 2, overview of the architecture); its
 * outlook (Sec. 3) names data-parallel phase-space sampling as the next step
 * to move to the GPU.  This file is the plain reference of that step for flat
 * phase space:
 *
 *   random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed
 *     by the 64-bit seed (k0 = low word, k1 = high word), counter
 *     (event low word, event high word, block, 0); uniform v of a block pair
 *     (w0, w1) = ((w0 * 2^32 + w1) >> 11 + 1/2) * 2^-53, in (0, 1).  Block b of
 *     an event gives uniforms 2b and 2b + 1 from its words (x0, x1) and
 *     (x2, x3).
 *
 *   momenta: RAMBO (Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986)
 *     359).  For each of the n final particles, with its four uniforms
 *     u1..u4: cos(theta) = 2 u1 - 1, phi = 2 pi u2, q0 = -ln(u3 u4), and
 *     q = q0 (sin(theta) cos(phi), sin(theta) sin(phi), cos(theta)).  With
 *     Q = sum q, M = sqrt(Q^2), b = -Q/M, x = sqrt(s)/M, gamma = Q0/M,
 *     a = 1/(1 + gamma), the conformal transformation
 *     p0 = x (gamma q0 + b.q), p = x (q + b q0 + a (b.q) b) gives n massless
 *     momenta summing to (sqrt(s), 0, 0, 0) with the constant weight
 *     w0 = (2 pi)^(4 - 3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!).
 *     Masses: the 3-momenta are scaled by the xi that solves
 *     sum_i sqrt(m_i^2 + xi^2 |p_i|^2) = sqrt(s) (Newton from xi = 1 with
 *     bisection safeguards), k = xi p, k0 = sqrt(m^2 + |k|^2), and the weight
 *     becomes w0 (sum|k|/sqrt s)^(2n-3) (prod |k_i|/k0_i) sqrt(s) / sum(|k_i|^2/k0_i).
 *
 *   layout: momenta [nevt][n + 2][4] (E, px, py, pz); particles 0 and 1 are
 *     the incoming partons (sqrt(s)/2)(1, 0, 0, +-1); the finals follow.
 *     Event e uses Philox counter e + first.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* One Philox4x32 round: two 32 x 32 -> 64 bit products, then the words are
 * exchanged and mixed with the key. */
static void philox_round(uint32_t x[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * x[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x[1] ^ k[0];
    const uint32_t y2 = hi0 ^ x[3] ^ k[1];
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
}

/* Philox4x32 with `rounds` rounds; the key is bumped by the Weyl constants
 * between rounds. */
void oracle_philox4x32(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4]) {
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < rounds; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(x, k);
    }
    memcpy(out, x, sizeof(x));
}

static double to_uniform(uint32_t hi, uint32_t lo) {
    const uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
    return ((double)v + 0.5) * (1.0 / 9007199254740992.0);
}

/* The uniforms of one event: u[0 .. nu-1]. */
void oracle_event_uniforms(uint64_t seed, uint64_t event, int nu, double* u) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int b = 0; 2 * b < nu; ++b) {
        const uint32_t ctr[4] = {(uint32_t)event, (uint32_t)(event >> 32), (uint32_t)b, 0u};
        uint32_t w[4];
        oracle_philox4x32(ctr, key, 10, w);
        u[2 * b] = to_uniform(w[0], w[1]);
        if (2 * b + 1 < nu) u[2 * b + 1] = to_uniform(w[2], w[3]);
    }
}

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* RAMBO points for events first .. first + nevt - 1 of the stream `seed`;
 * n final particles with masses m[0..n-1] (n <= 16).  cond (may be NULL)
 * receives (Q0/M)^2 per event: the conformal map divides by M^2 = Q0^2 - |Q|^2,
 * so rounding in the generated q is enlarged by this factor in the momenta.
 * Returns 0, or -1 on bad arguments. */
int oracle_rambo(double roots, const double* m, int n, uint64_t seed, int64_t first, int64_t nevt, double* mom,
                 double* wt, double* cond) {
    if (n < 2 || n > 16 || nevt < 0 || roots <= 0) return -1;
    const double s = roots * roots;
    const double w0 = pow(2 * M_PI, 4 - 3 * n) * pow(M_PI / 2, n - 1) * pow(s, n - 2) /
                      (factorial(n - 1) * factorial(n - 2));
    double msum = 0.0;
    int massive = 0;
    for (int i = 0; i < n; ++i) {
        msum += m[i];
        massive |= (m[i] != 0.0);
    }
    if (msum >= roots) return -1;
    for (int64_t e = 0; e < nevt; ++e) {
        double u[64];
        oracle_event_uniforms(seed, (uint64_t)(first + e), 4 * n, u);
        double q[16][4], Q[4] = {0, 0, 0, 0};
        for (int i = 0; i < n; ++i) {
            const double c = 2 * u[4 * i] - 1, phi = 2 * M_PI * u[4 * i + 1];
            const double q0 = -log(u[4 * i + 2] * u[4 * i + 3]);
            const double st = sqrt(1 - c * c);
            q[i][0] = q0;
            q[i][1] = q0 * st * cos(phi);
            q[i][2] = q0 * st * sin(phi);
            q[i][3] = q0 * c;
            for (int k = 0; k < 4; ++k) Q[k] += q[i][k];
        }
        const double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
        if (cond) cond[e] = (Q[0] / M) * (Q[0] / M);
        const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
        const double x = roots / M, gam = Q[0] / M, a = 1 / (1 + gam);
        double p[16][4];
        for (int i = 0; i < n; ++i) {
            const double bq = b[0] * q[i][1] + b[1] * q[i][2] + b[2] * q[i][3];
            p[i][0] = x * (gam * q[i][0] + bq);
            for (int k = 0; k < 3; ++k) p[i][k + 1] = x * (q[i][k + 1] + b[k] * q[i][0] + a * bq * b[k]);
        }
        double w = w0;
        double* o = mom + e * (int64_t)(n + 2) * 4;
        o[0] = roots / 2, o[1] = 0, o[2] = 0, o[3] = roots / 2;
        o[4] = roots / 2, o[5] = 0, o[6] = 0, o[7] = -roots / 2;
        if (!massive) {
            for (int i = 0; i < n; ++i) {
                double* oi = o + 4 * (i + 2);
                for (int k = 1; k < 4; ++k) oi[k] = p[i][k];
                oi[0] = sqrt(oi[1] * oi[1] + oi[2] * oi[2] + oi[3] * oi[3]);
            }
        } else {
            /* f(xi) = sum sqrt(m^2 + xi^2 P^2) - roots is increasing on [0, 1],
             * f(0) = sum m - roots < 0, f(1) >= 0. */
            double lo = 0.0, hi = 1.0, xi = 1.0;
            for (int it = 0; it < 200; ++it) {
                double f = -roots, df = 0.0;
                for (int i = 0; i < n; ++i) {
                    const double en = sqrt(m[i] * m[i] + xi * xi * p[i][0] * p[i][0]);
                    f += en;
                    df += xi * p[i][0] * p[i][0] / en;
                }
                if (f > 0) hi = xi;
                else lo = xi;
                double nx = xi - f / df;
                if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
                if (fabs(nx - xi) <= 1e-16 * xi) {
                    xi = nx;
                    break;
                }
                xi = nx;
            }
            double sk = 0.0, pr = 1.0, sk2 = 0.0;
            for (int i = 0; i < n; ++i) {
                double* oi = o + 4 * (i + 2);
                for (int k = 1; k < 4; ++k) oi[k] = xi * p[i][k];
                const double kk = sqrt(oi[1] * oi[1] + oi[2] * oi[2] + oi[3] * oi[3]);
                oi[0] = sqrt(m[i] * m[i] + kk * kk);
                sk += kk;
                pr *= kk / oi[0];
                sk2 += kk * kk / oi[0];
            }
            w = w0 * pow(sk / roots, 2 * n - 3) * pr * roots / sk2;
        }
        if (wt) wt[e] = w;
    }
    return 0;
}
