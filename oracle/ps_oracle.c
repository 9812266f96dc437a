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

/* ------------------------------------------------------------------ */
/* Multi-channel sampling for a final state with a lepton pair          */
/* ------------------------------------------------------------------ */

/*
 * Three channels for n final particles of which two (a, b) come from a
 * photon or Z (all final particles massless, n >= 3):
 *   0: flat RAMBO over the n particles (density 1/V_n, V_n the massless
 *      volume above);
 *   1: the pair's invariant mass squared M^2 from a Breit-Wigner of (MZ, WZ)
 *      restricted to [mlo^2, mhi^2] (inverse CDF through the arctangent),
 *      RAMBO over n-1 bodies (the pair as one particle of mass M first, the
 *      other finals in order), and an isotropic decay of the pair in its rest
 *      frame (particle a along (cos t = 2u - 1, phi = 2 pi u'));
 *   2: the same with M^2 distributed as 1/M^2 on the window (the photon).
 * From the factorisation dPhi_n = dPhi_{n-1}(P; Q, ...) dQ^2/(2 pi)
 * dPhi_2(Q; a, b), a channel-c point has density
 *   g_c(x) = 2 pi p_c(M^2) / (w_R(x') Phi_2),   Phi_2 = 1/(8 pi),
 * with w_R(x') the massive RAMBO weight of the (n-1)-body configuration x'
 * = (p_a + p_b, the others), which depends on the momenta only.  The point's
 * weight is 1 / sum_c alpha_c g_c(x) (alpha normalised), whichever channel
 * made it; g_1 = g_2 = 0 outside the window.
 *
 * Random numbers of event e (Philox stream as above): particle i of the
 * RAMBO stage takes uniforms 4i .. 4i + 3; uniform 32 picks the channel,
 * 33 maps M^2, 34 and 35 give the decay angles.
 */
static double rambo_w0(int n, double s) {
    return pow(2 * M_PI, 4 - 3 * n) * pow(M_PI / 2, n - 1) * pow(s, n - 2) / (factorial(n - 1) * factorial(n - 2));
}

/* RAMBO from uniforms u (4 per particle): n momenta p[n][4] with masses m,
 * summing to (roots, 0, 0, 0); returns the weight. */
static double rambo_from(double roots, const double* m, int n, const double* u, double p[][4]) {
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
    const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
    const double x = roots / M, gam = Q[0] / M, a = 1 / (1 + gam);
    for (int i = 0; i < n; ++i) {
        const double bq = b[0] * q[i][1] + b[1] * q[i][2] + b[2] * q[i][3];
        p[i][0] = x * (gam * q[i][0] + bq);
        for (int k = 0; k < 3; ++k) p[i][k + 1] = x * (q[i][k + 1] + b[k] * q[i][0] + a * bq * b[k]);
    }
    int massive = 0;
    for (int i = 0; i < n; ++i) massive |= (m[i] != 0.0);
    const double w0 = rambo_w0(n, roots * roots);
    if (!massive) {
        for (int i = 0; i < n; ++i) p[i][0] = sqrt(p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]);
        return w0;
    }
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
        for (int k = 1; k < 4; ++k) p[i][k] *= xi;
        const double kk = sqrt(p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]);
        p[i][0] = sqrt(m[i] * m[i] + kk * kk);
        sk += kk;
        pr *= kk / p[i][0];
        sk2 += kk * kk / p[i][0];
    }
    return w0 * pow(sk / roots, 2 * n - 3) * pr * roots / sk2;
}

/* Massive RAMBO weight of final momenta k[n][4] (from the momenta alone). */
static double rambo_weight_of(double roots, int n, const double k[][4]) {
    double sk = 0.0, pr = 1.0, sk2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double kk = sqrt(k[i][1] * k[i][1] + k[i][2] * k[i][2] + k[i][3] * k[i][3]);
        sk += kk;
        pr *= kk / k[i][0];
        sk2 += kk * kk / k[i][0];
    }
    return rambo_w0(n, roots * roots) * pow(sk / roots, 2 * n - 3) * pr * roots / sk2;
}

typedef struct {
    double a2, b2, mz, wz, alpha[3];
    double bw_lo, bw_hi;  /* arctangent bounds of the Breit-Wigner map */
} mc_setup;

static double mc_pdf(const mc_setup* S, int c, double m2) {
    if (!(m2 >= S->a2 && m2 <= S->b2)) return 0.0;
    if (c == 1) {
        const double mw = S->mz * S->wz, d = m2 - S->mz * S->mz;
        return mw / (d * d + mw * mw) / (S->bw_hi - S->bw_lo);
    }
    return 1.0 / (m2 * log(S->b2 / S->a2));
}

/* 1 / sum_c alpha_c g_c(x) for final momenta f[n][4], pair (ia, ib). */
static double mc_weight_of(const mc_setup* S, double roots, int n, const double f[][4], int ia, int ib) {
    double g = S->alpha[0] / rambo_w0(n, roots * roots);
    double P[4];
    for (int k = 0; k < 4; ++k) P[k] = f[ia][k] + f[ib][k];
    const double m2 = P[0] * P[0] - P[1] * P[1] - P[2] * P[2] - P[3] * P[3];
    if (m2 >= S->a2 && m2 <= S->b2 && (S->alpha[1] > 0 || S->alpha[2] > 0)) {
        double k[16][4];
        int j = 0;
        memcpy(k[j++], P, sizeof(P));
        for (int i = 0; i < n; ++i)
            if (i != ia && i != ib) memcpy(k[j++], f[i], sizeof(P));
        const double wr = rambo_weight_of(roots, n - 1, (const double(*)[4])k);
        const double phi2 = 1.0 / (8 * M_PI);
        for (int c = 1; c < 3; ++c) g += S->alpha[c] * 2 * M_PI * mc_pdf(S, c, m2) / (wr * phi2);
    }
    return 1.0 / g;
}

/* Events first .. first + nevt - 1: momenta [nevt][n + 2][4] as ps_rambo,
 * weights [nevt], chan [nevt] (may be NULL), wc [nevt] (may be NULL): the
 * weight of the generating channel alone, 1/g_c, from its construction.
 * Returns 0, or -1 on bad arguments. */
int oracle_ps_mc(double roots, int n, int ia, int ib, double mlo, double mhi, double mz, double wz,
                 const double* alpha, uint64_t seed, int64_t first, int64_t nevt, double* mom, double* wt,
                 int32_t* chan, double* wc) {
    if (n < 3 || n > 15 || ia < 0 || ib < 0 || ia >= n || ib >= n || ia == ib || nevt < 0 || roots <= 0) return -1;
    if (!(mlo > 0 && mhi > mlo && mhi <= roots)) return -1;
    const double at = alpha[0] + alpha[1] + alpha[2];
    if (!(alpha[0] >= 0 && alpha[1] >= 0 && alpha[2] >= 0 && at > 0)) return -1;
    mc_setup S;
    S.a2 = mlo * mlo;
    S.b2 = mhi * mhi;
    S.mz = mz;
    S.wz = wz;
    for (int c = 0; c < 3; ++c) S.alpha[c] = alpha[c] / at;
    S.bw_lo = atan((S.a2 - mz * mz) / (mz * wz));
    S.bw_hi = atan((S.b2 - mz * mz) / (mz * wz));
    for (int64_t e = 0; e < nevt; ++e) {
        double u[36];
        oracle_event_uniforms(seed, (uint64_t)(first + e), 36, u);
        const int c = (u[32] < S.alpha[0]) ? 0 : (u[32] < S.alpha[0] + S.alpha[1]) ? 1 : 2;
        double f[16][4];
        double w_own;
        if (c == 0) {
            double m0[16] = {0};
            w_own = rambo_from(roots, m0, n, u, f);
        } else {
            double m2;
            if (c == 1) {
                const double t = S.bw_lo + u[33] * (S.bw_hi - S.bw_lo);
                m2 = mz * mz + mz * wz * tan(t);
            } else {
                m2 = S.a2 * pow(S.b2 / S.a2, u[33]);
            }
            const double M = sqrt(m2);
            double m1[16] = {0}, k[16][4];
            m1[0] = M;
            const double wr = rambo_from(roots, m1, n - 1, u, k);
            /* decay of the pair (k[0], mass M) in its rest frame */
            const double ct = 2 * u[34] - 1, ph = 2 * M_PI * u[35], st = sqrt(1 - ct * ct);
            const double es = 0.5 * M;
            const double ks[3] = {es * st * cos(ph), es * st * sin(ph), es * ct};
            const double pk = k[0][1] * ks[0] + k[0][2] * ks[1] + k[0][3] * ks[2];
            const double e0 = (k[0][0] * es + pk) / M;
            const double fac = (e0 + es) / (k[0][0] + M);
            f[ia][0] = e0;
            for (int j = 0; j < 3; ++j) f[ia][j + 1] = ks[j] + fac * k[0][j + 1];
            for (int j = 0; j < 4; ++j) f[ib][j] = k[0][j] - f[ia][j];
            int jj = 1;
            for (int i = 0; i < n; ++i)
                if (i != ia && i != ib) memcpy(f[i], k[jj++], sizeof(f[i]));
            /* massless products: energies from the 3-momenta */
            f[ia][0] = sqrt(f[ia][1] * f[ia][1] + f[ia][2] * f[ia][2] + f[ia][3] * f[ia][3]);
            f[ib][0] = sqrt(f[ib][1] * f[ib][1] + f[ib][2] * f[ib][2] + f[ib][3] * f[ib][3]);
            w_own = wr / (8 * M_PI) / (2 * M_PI * mc_pdf(&S, c, m2));
        }
        double* o = mom + e * (int64_t)(n + 2) * 4;
        o[0] = roots / 2, o[1] = 0, o[2] = 0, o[3] = roots / 2;
        o[4] = roots / 2, o[5] = 0, o[6] = 0, o[7] = -roots / 2;
        for (int i = 0; i < n; ++i) memcpy(o + 4 * (i + 2), f[i], sizeof(f[i]));
        if (wt) wt[e] = mc_weight_of(&S, roots, n, (const double(*)[4])f, ia, ib);
        if (chan) chan[e] = c;
        if (wc) wc[e] = w_own;
    }
    return 0;
}
