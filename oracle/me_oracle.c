/*
 * me_oracle.c -- plain CPU reference for the squared matrix element |M|^2.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the package smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header or table
 * with the HIP path.
 *
 * What is computed (the paper's matrix-element step, Sec. 2: for each event
 * the per-event |M|^2 of a fixed partonic process; the generated physics code
 * evaluates Feynman diagrams, then the colour-matrix quadratic form, Sec. 3):
 *
 *   me2(p) = 1/(N_spin N_col S) * sum_helicities sum_colours |M(p)|^2
 *
 * written out from textbook tree-level Feynman rules, because the paper gives
 * no formulas.  S = (n-2)! for the identical final gluons of g g -> t tbar +
 * (n-2) g is parity unpinned: the GPU path applies the same reading and no
 * closed form or limit checked here involves more than one final gluon.
 * Conventions (the readings are listed in the design notes):
 *   metric (+,-,-,-); Dirac representation of the gamma matrices; helicity
 *   spinors and polarisation vectors built from polar angles; quark-gluon
 *   vertex  i g gamma^mu T^a;  three-gluon vertex  g f^{abc} V^{mu nu rho}
 *   with all momenta incoming;  four-gluon vertex  -i g^2 [f f (g g - g g)
 *   x 3];  gluon propagator -i g_{mu nu}/k^2 (Feynman gauge);  top propagator
 *   i(pslash + m)/(p^2 - m^2 + i m Gamma) on every internal top line;
 *   T^a = lambda^a / 2.
 *
 * Routes:
 *   1. e+ e- -> mu+ mu- : the two s-channel diagrams (photon, Z) written
 *      with explicit 4x4 matrices and summed over the 16 helicities.
 *   2. g g -> t tbar + (n-2) g, colour-ordered: for each ordering sigma of
 *      the n gluons along the top line, the partial amplitude J_sigma (the
 *      coefficient of (T^{a_sigma1} ... T^{a_sigma n})_{i j}) by Berends-Giele
 *      recursion (Berends, Giele, Nucl. Phys. B306 (1988) 759), with the
 *      colour-ordered vertices obtained from the full rules through
 *      f^{abc} T^c = -i [T^a, T^b]; then me2 = norm * sum_h J^dag C J with
 *      the colour matrix C passed in by the caller.
 *   3. g g -> t tbar + (n-2) g, colour-dressed: the same Feynman rules with
 *      every colour index explicit (recursion over subsets of gluons with
 *      f^{abc} and Gell-Mann T^a), and |M|^2 summed over all external colour
 *      assignments by brute force.  Independent of route 2's colour algebra.
 *   4. single Feynman diagrams of g g -> t tbar + (n-2) g (three-point
 *      vertices only), for the multi-channel weights.
 *   5. a massless quark line with n gluons and one photon/Z insertion that
 *      decays to a lepton pair (g ubar -> tau+ tau- g g ubar, the paper's
 *      DY+3j subprocess, Sec. 3, and its smaller relatives): colour-ordered
 *      recursion as in route 2 with the colourless insertion placed at every
 *      point of the quark line.
 *
 * Compiled twice: plain double (liboracle.so) and, with -DORACLE_QUAD,
 * __float128 (liboracle_quad.so) to adjudicate differences near 1e-12.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_QUAD
#include <quadmath.h>
typedef __float128 real;
typedef __complex128 cplx;
#define RSQRT sqrtq
#define RCOS cosq
#define RSIN sinq
#define RATAN2 atan2q
#define RFABS fabsq
#define CCONJ conjq
#define CREAL crealq
#define CIMAG cimagq
#else
typedef double real;
typedef double _Complex cplx;
#define RSQRT sqrt
#define RCOS cos
#define RSIN sin
#define RATAN2 atan2
#define RFABS fabs
#define CCONJ conj
#define CREAL creal
#define CIMAG cimag
#endif

#define CI ((cplx)_Complex_I)

/* ------------------------------------------------------------------ */
/* Dirac algebra                                                        */
/* ------------------------------------------------------------------ */

/* Constant tables are filled once when the library is loaded (before any
 * OpenMP region), so threads only ever read them. */
static cplx G[4][4][4]; /* gamma^mu, Dirac representation */
static cplx G5[4][4];

static void gamma_init(void) {
    memset(G, 0, sizeof G);
    memset(G5, 0, sizeof G5);
    /* gamma^0 = diag(1, 1, -1, -1) */
    G[0][0][0] = 1; G[0][1][1] = 1; G[0][2][2] = -1; G[0][3][3] = -1;
    /* gamma^k = [[0, sigma^k], [-sigma^k, 0]] */
    cplx s[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -CI}, {CI, 0}},
        {{1, 0}, {0, -1}},
    };
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                G[k + 1][a][b + 2] = s[k][a][b];
                G[k + 1][a + 2][b] = -s[k][a][b];
            }
    /* gamma^5 = [[0, 1], [1, 0]] */
    G5[0][2] = 1; G5[1][3] = 1; G5[2][0] = 1; G5[3][1] = 1;
}

static const real METRIC[4] = {1, -1, -1, -1};

/* Minkowski product of complex 4-vectors (no conjugation). */
static cplx cdot(const cplx a[4], const cplx b[4]) {
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

static real rdot(const real a[4], const real b[4]) {
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* out = gamma^mu v_mu (v contravariant). */
static void slash_c(const cplx v[4], cplx out[4][4]) {
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx acc = 0;
            for (int mu = 0; mu < 4; ++mu) acc += METRIC[mu] * v[mu] * G[mu][i][j];
            out[i][j] = acc;
        }
}

static void slash_r(const real v[4], cplx out[4][4]) {
    cplx c[4] = {v[0], v[1], v[2], v[3]};
    slash_c(c, out);
}

static void row_mat(const cplx r[4], cplx M[4][4], cplx out[4]) {
    cplx t[4];
    for (int j = 0; j < 4; ++j) {
        cplx acc = 0;
        for (int i = 0; i < 4; ++i) acc += r[i] * M[i][j];
        t[j] = acc;
    }
    memcpy(out, t, sizeof t);
}

static void mat_col(cplx M[4][4], const cplx c[4], cplx out[4]) {
    cplx t[4];
    for (int i = 0; i < 4; ++i) {
        cplx acc = 0;
        for (int j = 0; j < 4; ++j) acc += M[i][j] * c[j];
        t[i] = acc;
    }
    memcpy(out, t, sizeof t);
}

static cplx row_col(const cplx r[4], const cplx c[4]) {
    cplx acc = 0;
    for (int i = 0; i < 4; ++i) acc += r[i] * c[i];
    return acc;
}

/* Fermion propagator i (pslash + m) / (p^2 - m^2 + i m w). */
static void fprop(const real p[4], real m, real w, cplx S[4][4]) {
    cplx ps[4][4];
    slash_r(p, ps);
    cplx den = (rdot(p, p) - m * m) + CI * (m * w);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) S[i][j] = CI * (ps[i][j] + (i == j ? m : 0)) / den;
}

/* ------------------------------------------------------------------ */
/* External wavefunctions                                               */
/* ------------------------------------------------------------------ */

/* Two-component helicity eigenstates chi_lam(p) of sigma.p/|p|, lam = +-1. */
static void chi(const real p[4], int lam, cplx out[2]) {
    real pp = RSQRT(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
    real th = (pp > 0) ? RATAN2(RSQRT(p[1] * p[1] + p[2] * p[2]), p[3]) : 0;
    real ph = RATAN2(p[2], p[1]);
    real c = RCOS(th / 2), s = RSIN(th / 2);
    cplx e = RCOS(ph) + CI * RSIN(ph);
    if (lam > 0) {
        out[0] = c;
        out[1] = e * s;
    } else {
        out[0] = -CCONJ(e) * s;
        out[1] = c;
    }
}

/* u(p, lam) = (sqrt(E+m) chi, lam sqrt(E-m) chi) in the Dirac representation. */
static void u_spinor(const real p[4], real m, int lam, cplx out[4]) {
    cplx x[2];
    chi(p, lam, x);
    real a = RSQRT(p[0] + m);
    real d = p[0] - m;
    real b = (d > 0) ? RSQRT(d) : 0;
    out[0] = a * x[0];
    out[1] = a * x[1];
    out[2] = lam * b * x[0];
    out[3] = lam * b * x[1];
}

/* v(p, lam) = i gamma^2 u(p, lam)^*, the charge conjugate of u. */
static void v_spinor(const real p[4], real m, int lam, cplx out[4]) {
    cplx u[4], uc[4];
    u_spinor(p, m, lam, u);
    for (int i = 0; i < 4; ++i) uc[i] = CCONJ(u[i]);
    cplx t[4];
    mat_col(G[2], uc, t);
    for (int i = 0; i < 4; ++i) out[i] = CI * t[i];
}

/* psibar = psi^dagger gamma^0 */
static void bar(const cplx psi[4], cplx out[4]) {
    out[0] = CCONJ(psi[0]);
    out[1] = CCONJ(psi[1]);
    out[2] = -CCONJ(psi[2]);
    out[3] = -CCONJ(psi[3]);
}

/* Transverse helicity vector eps(k, lam) = (-lam e1 - i e2)/sqrt(2). */
static void eps_vec(const real k[4], int lam, cplx out[4]) {
    real pt = RSQRT(k[1] * k[1] + k[2] * k[2]);
    real th = RATAN2(pt, k[3]);
    real ph = RATAN2(k[2], k[1]);
    real ct = RCOS(th), st = RSIN(th), cp = RCOS(ph), sp = RSIN(ph);
    real e1[4] = {0, ct * cp, ct * sp, -st};
    real e2[4] = {0, -sp, cp, 0};
    real r = 1 / RSQRT((real)2);
    for (int mu = 0; mu < 4; ++mu) out[mu] = r * (-lam * e1[mu] - CI * e2[mu]);
}

/* ------------------------------------------------------------------ */
/* Route 1: e+ e- -> mu+ mu-                                            */
/* ------------------------------------------------------------------ */

/*
 * Particles: e+(p1) e-(p2) -> mu+(p3) mu-(p4), all massless.
 * Photon vertex -i e Q gamma^mu (Q = -1); Z vertex -i gz gamma^mu (gl PL + gr PR)
 * with gz = e/(sw cw), gl = -1/2 + sw^2, gr = sw^2; photon propagator -i g/s,
 * Z propagator -i (g - k k / MZ^2)/(s - MZ^2 + i MZ WZ).  i M = product of
 * factors, so M = (eQ)^2 (Je.Jm)/s + gz^2 [Je'.Jm' - (Je'.k)(Jm'.k)/MZ^2]/D.
 * Spin average 1/4.
 */
static real ee_one(const real *mom, real e, real sw2, real mz, real wz, real *qhel) {
    const real *p1 = mom, *p2 = mom + 4, *p3 = mom + 8, *p4 = mom + 12;
    real cw2 = 1 - sw2;
    real gz = e / RSQRT(sw2 * cw2);
    real gl = (real)-0.5 + sw2, gr = sw2;
    real k[4];
    for (int mu = 0; mu < 4; ++mu) k[mu] = p1[mu] + p2[mu];
    real s = rdot(k, k);
    cplx dz = (s - mz * mz) + CI * (mz * wz);
    /* chiral couplings as matrices: gl PL + gr PR, PL = (1 - g5)/2 */
    cplx Cz[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            Cz[i][j] = gl * ((i == j ? 1 : 0) - G5[i][j]) / 2 + gr * ((i == j ? 1 : 0) + G5[i][j]) / 2;
    real total = 0;
    for (int h = 0; h < 16; ++h) {
        int l1 = (h & 8) ? 1 : -1, l2 = (h & 4) ? 1 : -1, l3 = (h & 2) ? 1 : -1, l4 = (h & 1) ? 1 : -1;
        cplx v1[4], vb1[4], u2[4], v3[4], u4[4], ub4[4];
        v_spinor(p1, 0, l1, v1);
        bar(v1, vb1);
        u_spinor(p2, 0, l2, u2);
        v_spinor(p3, 0, l3, v3);
        u_spinor(p4, 0, l4, u4);
        bar(u4, ub4);
        cplx je[4], jm[4], jez[4], jmz[4];
        for (int mu = 0; mu < 4; ++mu) {
            cplx t[4], tz[4], GC[4][4];
            row_mat(vb1, G[mu], t);
            je[mu] = row_col(t, u2);
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    cplx acc = 0;
                    for (int l = 0; l < 4; ++l) acc += G[mu][i][l] * Cz[l][j];
                    GC[i][j] = acc;
                }
            row_mat(vb1, GC, tz);
            jez[mu] = row_col(tz, u2);
            row_mat(ub4, G[mu], t);
            jm[mu] = row_col(t, v3);
            row_mat(ub4, GC, tz);
            jmz[mu] = row_col(tz, v3);
        }
        cplx kc[4] = {k[0], k[1], k[2], k[3]};
        real Q = -1;
        cplx amp = (e * Q) * (e * Q) * cdot(je, jm) / s +
                   gz * gz * (cdot(jez, jmz) - cdot(jez, kc) * cdot(jmz, kc) / (mz * mz)) / dz;
        real a2 = CREAL(amp * CCONJ(amp));
        if (qhel) qhel[h] = a2;
        total += a2;
    }
    return total / 4;
}

int oracle_ee_mumu(const double *mom, int64_t n, double e, double sw2, double mz, double wz, double *out,
                   double *qhel) {
    if (!mom || !out || n < 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        real m[16];
        for (int j = 0; j < 16; ++j) m[j] = mom[16 * i + j];
        real q[16];
        out[i] = (double)ee_one(m, e, sw2, mz, wz, q);
        if (qhel)
            for (int h = 0; h < 16; ++h) qhel[16 * i + h] = (double)q[h];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Shared set-up for g g -> t tbar + gluons                             */
/* ------------------------------------------------------------------ */

#define MAXG 5
#define MAXNP (MAXG + 2)

/*
 * Momentum layout per event: [g1, g2, t, tbar, g3, ..., gn] x (E, px, py, pz).
 * Gluon index a = 0..n-1 maps to particle 0, 1, 4, 5, ...  Incoming gluons carry
 * their polarisation eps(p); outgoing gluons eps(p)^*.  Gluon momenta below are
 * taken as flowing INTO the diagram: q = p (incoming) or -p (outgoing).
 * Helicity index h: bit (npart-1-i) of h set means helicity + for particle i.
 * gauge_gluon >= 0 replaces that gluon's polarisation by q/q^0.
 */
typedef struct {
    int n;          /* number of gluons */
    real q[MAXG][4];  /* incoming-flow gluon momenta */
    cplx eps[MAXG][4];
    real p3[4], p4[4];
    cplx ubar3[4], v4[4];
    real mt, wt, gs;
} ggx_ext;

static int gluon_particle(int a) { return a < 2 ? a : a + 2; }

static void ggx_setup(const real *mom, int n, int h, int gauge_gluon, real gs, real mt, real wt, ggx_ext *X) {
    int np = n + 2;
    X->n = n;
    X->mt = mt;
    X->wt = wt;
    X->gs = gs;
    for (int a = 0; a < n; ++a) {
        int ip = gluon_particle(a);
        const real *p = mom + 4 * ip;
        int lam = ((h >> (np - 1 - ip)) & 1) ? 1 : -1;
        int incoming = (ip < 2);
        for (int mu = 0; mu < 4; ++mu) X->q[a][mu] = incoming ? p[mu] : -p[mu];
        cplx e[4];
        eps_vec(p, lam, e);
        for (int mu = 0; mu < 4; ++mu) X->eps[a][mu] = incoming ? e[mu] : CCONJ(e[mu]);
        if (a == gauge_gluon)
            for (int mu = 0; mu < 4; ++mu) X->eps[a][mu] = X->q[a][mu] / X->q[a][0];
    }
    for (int mu = 0; mu < 4; ++mu) {
        X->p3[mu] = mom[8 + mu];
        X->p4[mu] = mom[12 + mu];
    }
    int l3 = ((h >> (np - 3)) & 1) ? 1 : -1;
    int l4 = ((h >> (np - 4)) & 1) ? 1 : -1;
    cplx u3[4];
    u_spinor(X->p3, mt, l3, u3);
    bar(u3, X->ubar3);
    v_spinor(X->p4, mt, l4, X->v4);
}

/* Three-gluon vertex contracted with currents X, Y (flowing in with QX, QY):
 * V(QX, QY, -QX-QY)_{mu nu rho} X^mu Y^nu, returned with the index raised. */
static void v3(const cplx X[4], const real QX[4], const cplx Y[4], const real QY[4], cplx out[4]) {
    cplx xy = cdot(X, Y);
    real a[4], b[4];
    for (int mu = 0; mu < 4; ++mu) {
        a[mu] = QX[mu] + 2 * QY[mu];
        b[mu] = 2 * QX[mu] + QY[mu];
    }
    cplx ca[4] = {a[0], a[1], a[2], a[3]}, cb[4] = {b[0], b[1], b[2], b[3]};
    cplx ax = cdot(ca, X), by = cdot(cb, Y);
    for (int mu = 0; mu < 4; ++mu) out[mu] = xy * (QX[mu] - QY[mu]) + Y[mu] * ax - X[mu] * by;
}

/* ------------------------------------------------------------------ */
/* Route 2: colour-ordered Berends-Giele                                */
/* ------------------------------------------------------------------ */

/*
 * Colour-ordered rules (coefficient of T^{a1} T^{a2} ... in the full rules):
 *   quark-gluon vertex      i g gamma^mu
 *   ordered 3-gluon vertex  -i g V(QX, QY, -QX-QY)          (X before Y)
 *   ordered 4-gluon vertex   i g^2 [2 g^{mu rho} g^{nu sig} - g^{mu nu} g^{rho sig}
 *                                   - g^{mu sig} g^{nu rho}] (X, Y, Z, root)
 * Gluon currents include the propagator -i/Q^2.
 */
static void bg_amp(const ggx_ext *X, const int *sigma, cplx *out_amp, int with4) {
    int n = X->n;
    real g = X->gs;
    cplx J[MAXG][MAXG][4];
    real Q[MAXG][MAXG][4];
    for (int i = 0; i < n; ++i) {
        for (int mu = 0; mu < 4; ++mu) {
            J[i][i][mu] = X->eps[sigma[i]][mu];
            Q[i][i][mu] = X->q[sigma[i]][mu];
        }
    }
    for (int len = 2; len <= n; ++len) {
        for (int i = 0; i + len - 1 < n; ++i) {
            int j = i + len - 1;
            for (int mu = 0; mu < 4; ++mu) Q[i][j][mu] = Q[i][i][mu] + Q[i + 1][j][mu];
            real Q2 = rdot(Q[i][j], Q[i][j]);
            cplx acc[4] = {0, 0, 0, 0};
            for (int k = i; k < j; ++k) {
                cplx t[4];
                v3(J[i][k], Q[i][k], J[k + 1][j], Q[k + 1][j], t);
                /* (-i/Q^2)(-i g) = -g/Q^2 */
                for (int mu = 0; mu < 4; ++mu) acc[mu] += (-g / Q2) * t[mu];
            }
            for (int k = i; k < j && with4; ++k)
                for (int l = k + 1; l < j; ++l) {
                    const cplx *A = J[i][k], *B = J[k + 1][l], *C = J[l + 1][j];
                    cplx ac = cdot(A, C), ab = cdot(A, B), bc = cdot(B, C);
                    /* (-i/Q^2)(i g^2) = g^2/Q^2 */
                    for (int mu = 0; mu < 4; ++mu)
                        acc[mu] += (g * g / Q2) * (2 * ac * B[mu] - ab * C[mu] - bc * A[mu]);
                }
            for (int mu = 0; mu < 4; ++mu) J[i][j][mu] = acc[mu];
        }
    }
    /* Quark line: U[m] = ubar(p3) after the first m gluons of sigma. */
    cplx U[MAXG + 1][4];
    memcpy(U[0], X->ubar3, sizeof(cplx) * 4);
    for (int m = 1; m <= n; ++m) {
        cplx acc[4] = {0, 0, 0, 0};
        if (m < n) {
            real P[4];
            for (int mu = 0; mu < 4; ++mu) P[mu] = X->p3[mu] - Q[0][m - 1][mu];
            cplx S[4][4];
            fprop(P, X->mt, X->wt, S);
            for (int l = 0; l < m; ++l) {
                cplx js[4][4], t[4];
                slash_c(J[l][m - 1], js);
                row_mat(U[l], js, t);
                for (int a = 0; a < 4; ++a) acc[a] += CI * g * t[a];
            }
            row_mat(acc, S, U[m]);
        }
    }
    cplx amp = 0;
    for (int l = 0; l < n; ++l) {
        cplx js[4][4], t[4];
        slash_c(J[l][n - 1], js);
        row_mat(U[l], js, t);
        amp += CI * g * row_col(t, X->v4);
    }
    *out_amp = amp;
}

static int next_perm(int *a, int n) {
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) --i;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) --j;
    int t = a[i];
    a[i] = a[j];
    a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; ++l, --r) {
        t = a[l];
        a[l] = a[r];
        a[r] = t;
    }
    return 1;
}

static int factorial(int n) { return n <= 1 ? 1 : n * factorial(n - 1); }

/* Partial amplitudes J[k] for all n! orderings (lexicographic order of
 * permutations of gluon indices 0..n-1) at one helicity. */
static void ordered_amps(const ggx_ext *X, cplx *J, int with4) {
    int n = X->n;
    int sigma[MAXG];
    for (int i = 0; i < n; ++i) sigma[i] = i;
    int k = 0;
    do {
        bg_amp(X, sigma, &J[k++], with4);
    } while (next_perm(sigma, n));
}

/* sum_kl conj(J_k) C_kl J_l */
static real colour_form(const cplx *J, const real *C, int ncol) {
    cplx acc = 0;
    for (int k = 0; k < ncol; ++k) {
        cplx row = 0;
        for (int l = 0; l < ncol; ++l) row += C[k * ncol + l] * J[l];
        acc += CCONJ(J[k]) * row;
    }
    return CREAL(acc);
}

static real ggx_norm(int n) {
    /* 1/(4 spins * 64 colours * (n-2)! identical final gluons) */
    return (real)1 / ((real)256 * factorial(n - 2));
}

static real ggx_one(const real *mom, int n, const real *C, real gs, real mt, real wt, real *qhel) {
    int np = n + 2, ncol = factorial(n);
    cplx *J = (cplx *)malloc(sizeof(cplx) * ncol);
    real total = 0;
    for (int h = 0; h < (1 << np); ++h) {
        ggx_ext X;
        ggx_setup(mom, n, h, -1, gs, mt, wt, &X);
        ordered_amps(&X, J, 1);
        real q = colour_form(J, C, ncol);
        if (qhel) qhel[h] = q;
        total += q;
    }
    free(J);
    return total * ggx_norm(n);
}

int oracle_ggx(const double *mom, int64_t nevt, int n, const double *colour, double gs, double mt, double wt,
               double *out, double *qhel) {
    if (!mom || !out || !colour || n < 2 || n > MAXG || nevt < 0) return -1;
    int np = n + 2, ncol = factorial(n);
    real *C = (real *)malloc(sizeof(real) * ncol * ncol);
    for (int i = 0; i < ncol * ncol; ++i) C[i] = colour[i];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < nevt; ++e) {
        real m[4 * MAXNP];
        for (int j = 0; j < 4 * np; ++j) m[j] = mom[4 * np * e + j];
        real q[1 << MAXNP];
        out[e] = (double)ggx_one(m, n, C, gs, mt, wt, qhel ? q : NULL);
        if (qhel)
            for (int h = 0; h < (1 << np); ++h) qhel[(int64_t)(1 << np) * e + h] = (double)q[h];
    }
    free(C);
    return 0;
}

/* Partial amplitudes of one event at one helicity, for gauge and MHV checks.
 * out: [n!][2] (re, im). */
int oracle_ggx_amps(const double *mom1, int n, int h, int gauge_gluon, double gs, double mt, double wt,
                    double *out, int with4) {
    if (!mom1 || !out || n < 2 || n > MAXG) return -1;
    int np = n + 2, ncol = factorial(n);
    real m[4 * MAXNP];
    for (int j = 0; j < 4 * np; ++j) m[j] = mom1[j];
    ggx_ext X;
    ggx_setup(m, n, h, gauge_gluon, gs, mt, wt, &X);
    cplx *J = (cplx *)malloc(sizeof(cplx) * ncol);
    ordered_amps(&X, J, with4);
    for (int k = 0; k < ncol; ++k) {
        out[2 * k] = (double)CREAL(J[k]);
        out[2 * k + 1] = (double)CIMAG(J[k]);
    }
    free(J);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Route 3: colour-dressed brute force                                  */
/* ------------------------------------------------------------------ */

static cplx TA[8][3][3]; /* T^a = lambda^a / 2 */
static real FABC[8][8][8];

static void colour_init(void) {
    memset(TA, 0, sizeof TA);
    cplx l[8][3][3];
    memset(l, 0, sizeof l);
    l[0][0][1] = 1; l[0][1][0] = 1;
    l[1][0][1] = -CI; l[1][1][0] = CI;
    l[2][0][0] = 1; l[2][1][1] = -1;
    l[3][0][2] = 1; l[3][2][0] = 1;
    l[4][0][2] = -CI; l[4][2][0] = CI;
    l[5][1][2] = 1; l[5][2][1] = 1;
    l[6][1][2] = -CI; l[6][2][1] = CI;
    real r3 = 1 / RSQRT((real)3);
    l[7][0][0] = r3; l[7][1][1] = r3; l[7][2][2] = -2 * r3;
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) TA[a][i][j] = l[a][i][j] / 2;
    /* f^{abc} = -2 i Tr([T^a, T^b] T^c) */
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            for (int c = 0; c < 8; ++c) {
                cplx tr = 0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k)
                            tr += (TA[a][i][j] * TA[b][j][k] - TA[b][i][j] * TA[a][j][k]) * TA[c][k][i];
                FABC[a][b][c] = CREAL(-2 * CI * tr);
            }
}

__attribute__((constructor)) static void tables_init(void) {
    gamma_init();
    colour_init();
}

/* Gluon currents with explicit adjoint index for every subset of gluons. */
typedef struct {
    cplx J[1 << MAXG][8][4];
    real Q[1 << MAXG][4];
} dressed_cur;

static void dressed_currents(const ggx_ext *X, const int *col, dressed_cur *D) {
    int n = X->n;
    real g = X->gs;
    int full = (1 << n) - 1;
    for (int S = 1; S <= full; ++S) {
        for (int mu = 0; mu < 4; ++mu) {
            real acc = 0;
            for (int a = 0; a < n; ++a)
                if (S & (1 << a)) acc += X->q[a][mu];
            D->Q[S][mu] = acc;
        }
        memset(D->J[S], 0, sizeof D->J[S]);
    }
    for (int a = 0; a < n; ++a)
        for (int mu = 0; mu < 4; ++mu) D->J[1 << a][col[a]][mu] = X->eps[a][mu];
    /* subsets in order of increasing size */
    for (int sz = 2; sz <= n; ++sz) {
        for (int S = 1; S <= full; ++S) {
            if (__builtin_popcount(S) != sz) continue;
            real Q2 = rdot(D->Q[S], D->Q[S]);
            int low = S & -S;
            /* unordered two-way splits {X, Y}: X holds the lowest gluon */
            for (int Xs = (S - 1) & S; Xs > 0; Xs = (Xs - 1) & S) {
                if (!(Xs & low)) continue;
                int Ys = S ^ Xs;
                for (int b = 0; b < 8; ++b)
                    for (int c = 0; c < 8; ++c) {
                        int nzb = 0, nzc = 0;
                        for (int mu = 0; mu < 4; ++mu) {
                            nzb |= (D->J[Xs][b][mu] != 0);
                            nzc |= (D->J[Ys][c][mu] != 0);
                        }
                        if (!nzb || !nzc) continue;
                        cplx t[4];
                        v3(D->J[Xs][b], D->Q[Xs], D->J[Ys][c], D->Q[Ys], t);
                        for (int a = 0; a < 8; ++a) {
                            real f = FABC[b][c][a];
                            if (f == 0) continue;
                            /* vertex g f^{b c a} V(QX, QY, -QS); propagator -i/Q^2 */
                            for (int mu = 0; mu < 4; ++mu) D->J[S][a][mu] += (-CI / Q2) * g * f * t[mu];
                        }
                    }
            }
            /* unordered three-way splits {X, Y, Z} */
            if (sz >= 3) {
                for (int Xs = (S - 1) & S; Xs > 0; Xs = (Xs - 1) & S) {
                    if (!(Xs & low)) continue;
                    int R = S ^ Xs;
                    int lowR = R & -R;
                    for (int Ys = (R - 1) & R; Ys > 0; Ys = (Ys - 1) & R) {
                        if (!(Ys & lowR)) continue;
                        int Zs = R ^ Ys;
                        for (int b = 0; b < 8; ++b)
                            for (int c = 0; c < 8; ++c)
                                for (int d = 0; d < 8; ++d) {
                                    const cplx *A = D->J[Xs][b], *B = D->J[Ys][c], *C = D->J[Zs][d];
                                    cplx ab = cdot(A, B), ac = cdot(A, C), bc = cdot(B, C);
                                    if (ab == 0 && ac == 0 && bc == 0) continue;
                                    for (int a = 0; a < 8; ++a) {
                                        /* -i g^2 [f^{bce} f^{dae} (g^{mr} g^{ns} - g^{ms} g^{nr})
                                         *        + f^{bde} f^{cae} (g^{mn} g^{rs} - g^{ms} g^{nr})
                                         *        + f^{bae} f^{cde} (g^{mn} g^{rs} - g^{mr} g^{ns})] */
                                        real c1 = 0, c2 = 0, c3 = 0;
                                        for (int e = 0; e < 8; ++e) {
                                            c1 += FABC[b][c][e] * FABC[d][a][e];
                                            c2 += FABC[b][d][e] * FABC[c][a][e];
                                            c3 += FABC[b][a][e] * FABC[c][d][e];
                                        }
                                        if (c1 == 0 && c2 == 0 && c3 == 0) continue;
                                        for (int mu = 0; mu < 4; ++mu) {
                                            cplx v = c1 * (ac * B[mu] - A[mu] * bc) + c2 * (ab * C[mu] - A[mu] * bc) +
                                                     c3 * (ab * C[mu] - ac * B[mu]);
                                            /* (-i/Q^2)(-i g^2) = -g^2/Q^2 */
                                            D->J[S][a][mu] += (-g * g / Q2) * v;
                                        }
                                    }
                                }
                    }
                }
            }
        }
    }
}

/* |M|^2 summed over top/antitop colours for fixed gluon colours.
 * U carries spinor x fundamental colour: U[S][i0][spin][colour]
 * where i0 is the top's colour at the ubar end. */
static real dressed_colour_sum(const ggx_ext *X, const dressed_cur *D) {
    int n = X->n;
    real g = X->gs;
    int full = (1 << n) - 1;
    static __thread cplx U[1 << MAXG][3][4][3];
    memset(U, 0, sizeof(cplx) * (size_t)(full + 1) * 3 * 4 * 3);
    for (int i0 = 0; i0 < 3; ++i0)
        for (int s = 0; s < 4; ++s) U[0][i0][s][i0] = X->ubar3[s];
    real total = 0;
    for (int sz = 1; sz <= n; ++sz) {
        for (int S = 1; S <= full; ++S) {
            if (__builtin_popcount(S) != sz) continue;
            /* V(S) = sum over last block B of U(S \ B) (i g gamma.J_a(B) T^a) */
            cplx V[3][4][3];
            memset(V, 0, sizeof V);
            for (int B = S; B > 0; B = (B - 1) & S) {
                int L = S ^ B;
                for (int a = 0; a < 8; ++a) {
                    int nz = 0;
                    for (int mu = 0; mu < 4; ++mu) nz |= (D->J[B][a][mu] != 0);
                    if (!nz) continue;
                    cplx js[4][4];
                    slash_c(D->J[B][a], js);
                    for (int i0 = 0; i0 < 3; ++i0)
                        for (int c = 0; c < 3; ++c) {
                            cplx row[4], t[4];
                            int nzr = 0;
                            for (int s = 0; s < 4; ++s) {
                                row[s] = U[L][i0][s][c];
                                nzr |= (row[s] != 0);
                            }
                            if (!nzr) continue;
                            row_mat(row, js, t);
                            for (int c2 = 0; c2 < 3; ++c2) {
                                cplx tc = TA[a][c][c2];
                                if (tc == 0) continue;
                                for (int s = 0; s < 4; ++s) V[i0][s][c2] += CI * g * t[s] * tc;
                            }
                        }
                }
            }
            if (S == full) {
                /* close with v(p4): M[i0][j] = V[i0][.][j] . v4 */
                for (int i0 = 0; i0 < 3; ++i0)
                    for (int j = 0; j < 3; ++j) {
                        cplx m = 0;
                        for (int s = 0; s < 4; ++s) m += V[i0][s][j] * X->v4[s];
                        total += CREAL(m * CCONJ(m));
                    }
            } else {
                real P[4];
                for (int mu = 0; mu < 4; ++mu) P[mu] = X->p3[mu] - D->Q[S][mu];
                cplx Sp[4][4];
                fprop(P, X->mt, X->wt, Sp);
                for (int i0 = 0; i0 < 3; ++i0)
                    for (int c = 0; c < 3; ++c) {
                        cplx row[4], t[4];
                        for (int s = 0; s < 4; ++s) row[s] = V[i0][s][c];
                        row_mat(row, Sp, t);
                        for (int s = 0; s < 4; ++s) U[S][i0][s][c] = t[s];
                    }
            }
        }
    }
    return total;
}

/* me2 of one event by the colour-dressed route (slow: 8^n colour sums per helicity). */
int oracle_ggx_dressed(const double *mom1, int n, double gs, double mt, double wt, double *out_me2,
                       double *qhel) {
    if (!mom1 || !out_me2 || n < 2 || n > 4) return -1;
    int np = n + 2;
    real m[4 * MAXNP];
    for (int j = 0; j < 4 * np; ++j) m[j] = mom1[j];
    int nh = 1 << np;
    int ncolass = 1;
    for (int a = 0; a < n; ++a) ncolass *= 8;
    real *qh = (real *)calloc(nh, sizeof(real));
#pragma omp parallel for schedule(dynamic, 1)
    for (int h = 0; h < nh; ++h) {
        ggx_ext X;
        ggx_setup(m, n, h, -1, gs, mt, wt, &X);
        dressed_cur *D = (dressed_cur *)malloc(sizeof(dressed_cur));
        real acc = 0;
        for (int ca = 0; ca < ncolass; ++ca) {
            int col[MAXG], t = ca;
            for (int a = 0; a < n; ++a) {
                col[a] = t % 8;
                t /= 8;
            }
            dressed_currents(&X, col, D);
            acc += dressed_colour_sum(&X, D);
        }
        free(D);
        qh[h] = acc;
    }
    real total = 0;
    for (int h = 0; h < nh; ++h) {
        total += qh[h];
        if (qhel) qhel[h] = (double)qh[h];
    }
    free(qh);
    *out_me2 = (double)(total * ggx_norm(n));
    return 0;
}

int oracle_is_quad(void) {
#ifdef ORACLE_QUAD
    return 1;
#else
    return 0;
#endif
}

/* ------------------------------------------------------------------ */
/* Route 4: single Feynman diagrams (three-point vertices only)          */
/* ------------------------------------------------------------------ */

/*
 * The multi-channel weights of the paper's Sec. 2 need the squared amplitude
 * of each single Feynman diagram, summed over helicities.  Here a diagram is
 * a sequence of gluon trees attached along the top line from ubar(p3) to
 * v(p4); each tree is built from three-gluon vertices only (diagrams with a
 * four-gluon vertex are not channels).  With the colour factors stripped so
 * that every colour-flow coefficient has unit modulus (f^{abc} T^c =
 * -i [T^a, T^b], the quark-gluon vertex T^a), the kinematic amplitude is
 *   A = ubar(p3) (i g Wslash_1) S(P_1) (i g Wslash_2) ... (i g Wslash_j) v(p4),
 *   P_i = p3 - (sum of the incoming-flow momenta of trees 1..i),
 * with the tree currents W = eps for a leaf and
 *   W(X, Y) = (-i / Q^2)(-i g) V(Q_X, Q_Y, -Q_X - Q_Y) . W_X W_Y
 * for a vertex joining subtrees X and Y (the order of X and Y only flips the
 * sign).  |A|^2 does not depend on spinor or polarisation phase conventions.
 *
 * A diagram is encoded as ints: [nblocks, root node of each block (MAXG
 * slots), nnodes, then per node (left, right, leaf)], leaf >= 0 for an
 * external gluon (left = right = -1), otherwise left/right are earlier nodes.
 */
#define DIAG_STRIDE (2 + MAXG + 3 * 2 * MAXG)

static cplx diagram_amp(const ggx_ext *X, const int *d) {
    const int nb = d[0];
    const int *root = d + 1;
    const int nn = d[1 + MAXG];
    const int *node = d + 2 + MAXG;
    real g = X->gs;
    cplx W[2 * MAXG][4];
    real Q[2 * MAXG][4];
    for (int i = 0; i < nn; ++i) {
        const int l = node[3 * i], r = node[3 * i + 1], leaf = node[3 * i + 2];
        if (leaf >= 0) {
            for (int mu = 0; mu < 4; ++mu) {
                W[i][mu] = X->eps[leaf][mu];
                Q[i][mu] = X->q[leaf][mu];
            }
            continue;
        }
        for (int mu = 0; mu < 4; ++mu) Q[i][mu] = Q[l][mu] + Q[r][mu];
        const real Q2 = rdot(Q[i], Q[i]);
        cplx t[4];
        v3(W[l], Q[l], W[r], Q[r], t);
        for (int mu = 0; mu < 4; ++mu) W[i][mu] = (-g / Q2) * t[mu];
    }
    cplx U[4];
    memcpy(U, X->ubar3, sizeof(U));
    real P[4];
    memcpy(P, X->p3, sizeof(P));
    for (int b = 0; b < nb; ++b) {
        const int k = root[b];
        cplx js[4][4], t[4];
        slash_c(W[k], js);
        row_mat(U, js, t);
        for (int a = 0; a < 4; ++a) U[a] = CI * g * t[a];
        if (b + 1 < nb) {
            for (int mu = 0; mu < 4; ++mu) P[mu] -= Q[k][mu];
            cplx S[4][4];
            fprop(P, X->mt, X->wt, S);
            row_mat(U, S, t);
            memcpy(U, t, sizeof(U));
        }
    }
    return row_col(U, X->v4);
}

/* out[e][k] = sum over all helicities of |A_k|^2 for the ndiag diagrams in
 * enc ([ndiag][DIAG_STRIDE]), and (optionally) me2-normalised: the same
 * average over initial spins and colours as me2 is not applied (these are
 * ratios). */
int oracle_ggx_diagrams(const double *mom, int64_t nevt, int n, int ndiag, const int *enc, double gs, double mt,
                        double wt, double *out) {
    if (n < 2 || n > MAXG || ndiag < 1) return -1;
    const int np = n + 2, nhel = 1 << np;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < nevt; ++e) {
        real p[4 * MAXNP];
        for (int i = 0; i < 4 * np; ++i) p[i] = mom[e * 4 * np + i];
        double *o = out + e * ndiag;
        for (int k = 0; k < ndiag; ++k) o[k] = 0.0;
        for (int h = 0; h < nhel; ++h) {
            ggx_ext X;
            ggx_setup(p, n, h, -1, gs, mt, wt, &X);
            for (int k = 0; k < ndiag; ++k) {
                const cplx a = diagram_amp(&X, enc + (int64_t)k * DIAG_STRIDE);
                o[k] += (double)(CREAL(a) * CREAL(a) + CIMAG(a) * CIMAG(a));
            }
        }
    }
    return bad;
}

/* The complex amplitudes A_d of the ndiag encoded diagrams for one event at
 * one helicity (for checks). */
int oracle_ggx_diagram_amps(const double *mom1, int n, int h, int ndiag, const int *enc, double gs, double mt,
                            double wt, double *out) {
    if (!mom1 || !out || n < 2 || n > MAXG) return -1;
    real m[4 * MAXNP];
    for (int j = 0; j < 4 * (n + 2); ++j) m[j] = mom1[j];
    ggx_ext X;
    ggx_setup(m, n, h, -1, gs, mt, wt, &X);
    for (int k = 0; k < ndiag; ++k) {
        const cplx a = diagram_amp(&X, enc + (int64_t)k * DIAG_STRIDE);
        out[2 * k] = (double)CREAL(a);
        out[2 * k + 1] = (double)CIMAG(a);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Route 5: a massless quark line with gluons and one gamma/Z insertion */
/* ------------------------------------------------------------------ */

/*
 * Processes with one massless quark line, n gluons and a lepton pair from
 * gamma/Z, e.g. g ubar -> tau+ tau- g g ubar (the paper's DY+3j subprocess).
 * Descriptor desc[] (ints): n, npart, row particle, row kind (0 outgoing quark
 * ubar(p), 1 incoming antiquark vbar(p)), column particle, column kind (0
 * outgoing antiquark v(p), 1 incoming quark u(p)), l- particle, l+ particle,
 * then MAXG gluon particle indices and MAXG incoming flags.  Couplings cpl[]:
 * e, sin^2 theta_W, M_Z, Gamma_Z, g_s, Q and T3 of the quark, Q and T3 of the
 * lepton.  All fermions massless.
 *
 * Rules: quark-gluon i g_s gamma^mu T^a (colour-ordered: i g_s gamma^mu);
 * photon -i e Q gamma^mu; Z -i g_Z gamma^mu (gL PL + gR PR) with g_Z =
 * e/(s_W c_W), gL = T3 - Q s_W^2, gR = -Q s_W^2; photon propagator -i g/k^2;
 * Z propagator -i g/(k^2 - M_Z^2 + i M_Z Gamma_Z) (the k k / M_Z^2 term drops
 * against the conserved massless lepton current); quark propagator
 * i pslash / p^2.  The boson and lepton pair fold into one insertion on the
 * quark line, gamma^mu (EL_mu PL + ER_mu PR) with
 *   EX = i e^2 Qq Ql Jg / k^2 + i g_Z^2 gX(q) JZ / (k^2 - M_Z^2 + i M_Z Gamma_Z),
 *   Jg^mu = ubar(l-) gamma^mu v(l+),  JZ^mu = ubar(l-) gamma^mu (gL(l) PL + gR(l) PR) v(l+),
 * k = p(l-) + p(l+).  The insertion is a colour singlet, so the colour
 * decomposition is that of the quark line with n gluons.
 */
#define QEW_DESC (8 + 2 * MAXG)

typedef struct {
    int n;
    real q[MAXG][4];   /* incoming-flow gluon momenta */
    cplx eps[MAXG][4];
    real prow[4];      /* momentum along the fermion flow leaving the row end */
    cplx row[4], col[4];
    cplx GE[4][4];     /* the gamma/Z insertion as a Dirac matrix */
    real qE[4];        /* momentum flowing into the line at the insertion */
    real gs;
} qew_ext;

static void qew_setup(const real *mom, const int *d, const double *cpl, int h, int gauge_gluon, int gauge_ew,
                      qew_ext *X) {
    const int n = d[0], np = d[1];
    const int *gp = d + 8, *gin = d + 8 + MAXG;
    X->n = n;
    X->gs = cpl[4];
#define HEL(i) ((((h) >> (np - 1 - (i))) & 1) ? 1 : -1)
    for (int a = 0; a < n; ++a) {
        const real *p = mom + 4 * gp[a];
        const int incoming = gin[a];
        cplx e[4];
        eps_vec(p, HEL(gp[a]), e);
        for (int mu = 0; mu < 4; ++mu) {
            X->q[a][mu] = incoming ? p[mu] : -p[mu];
            X->eps[a][mu] = incoming ? e[mu] : CCONJ(e[mu]);
        }
        if (a == gauge_gluon)
            for (int mu = 0; mu < 4; ++mu) X->eps[a][mu] = X->q[a][mu] / X->q[a][0];
    }
    /* quark line ends */
    {
        const real *p = mom + 4 * d[2];
        cplx s[4];
        if (d[3] == 0) {
            u_spinor(p, 0, HEL(d[2]), s);
            for (int mu = 0; mu < 4; ++mu) X->prow[mu] = p[mu];
        } else {
            v_spinor(p, 0, HEL(d[2]), s);
            for (int mu = 0; mu < 4; ++mu) X->prow[mu] = -p[mu];
        }
        bar(s, X->row);
        const real *pc = mom + 4 * d[4];
        if (d[5] == 0)
            v_spinor(pc, 0, HEL(d[4]), X->col);
        else
            u_spinor(pc, 0, HEL(d[4]), X->col);
    }
    /* lepton pair and the gamma/Z insertion */
    const real *pm = mom + 4 * d[6], *pp = mom + 4 * d[7];
    cplx um[4], ubm[4], vp[4];
    u_spinor(pm, 0, HEL(d[6]), um);
    bar(um, ubm);
    v_spinor(pp, 0, HEL(d[7]), vp);
#undef HEL
    const real e = cpl[0], sw2 = cpl[1], mz = cpl[2], wz = cpl[3];
    const real Qq = cpl[5], T3q = cpl[6], Ql = cpl[7], T3l = cpl[8];
    const real gz = e / RSQRT(sw2 * (1 - sw2));
    const real gLq = T3q - Qq * sw2, gRq = -Qq * sw2, gLl = T3l - Ql * sw2, gRl = -Ql * sw2;
    real k[4];
    for (int mu = 0; mu < 4; ++mu) {
        k[mu] = pm[mu] + pp[mu];
        X->qE[mu] = -k[mu];
    }
    const real k2 = rdot(k, k);
    const cplx dz = (k2 - mz * mz) + CI * (mz * wz);
    cplx Jg[4], JZ[4];
    for (int mu = 0; mu < 4; ++mu) {
        cplx Cl[4][4], t[4];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cplx acc = 0;
                for (int l = 0; l < 4; ++l) {
                    const cplx pl = ((l == j ? 1 : 0) - G5[l][j]) / 2, pr = ((l == j ? 1 : 0) + G5[l][j]) / 2;
                    acc += G[mu][i][l] * (gLl * pl + gRl * pr);
                }
                Cl[i][j] = acc;
            }
        row_mat(ubm, G[mu], t);
        Jg[mu] = row_col(t, vp);
        row_mat(ubm, Cl, t);
        JZ[mu] = row_col(t, vp);
    }
    cplx EL[4], ER[4];
    for (int mu = 0; mu < 4; ++mu) {
        const cplx ga = CI * e * e * Qq * Ql * Jg[mu] / k2;
        EL[mu] = ga + CI * gz * gz * gLq * JZ[mu] / dz;
        ER[mu] = ga + CI * gz * gz * gRq * JZ[mu] / dz;
        if (gauge_ew) EL[mu] = ER[mu] = X->qE[mu];
    }
    cplx SL[4][4], SR[4][4];
    slash_c(EL, SL);
    slash_c(ER, SR);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx acc = 0;
            for (int l = 0; l < 4; ++l) {
                const cplx pl = ((l == j ? 1 : 0) - G5[l][j]) / 2, pr = ((l == j ? 1 : 0) + G5[l][j]) / 2;
                acc += SL[i][l] * pl + SR[i][l] * pr;
            }
            X->GE[i][j] = acc;
        }
}

/* Colour-ordered amplitude for gluon order sigma: gluon currents over
 * contiguous ranges of sigma (three- and four-gluon vertices, as in route 2),
 * then the quark line from the row end, absorbing the gluon ranges in order
 * and the colourless insertion at any point: U[m][e] is the row spinor after
 * the first m gluons of sigma and e insertions, propagator included. */
static cplx qew_amp(const qew_ext *X, const int *sigma) {
    const int n = X->n;
    const real g = X->gs;
    cplx J[MAXG][MAXG][4];
    real Q[MAXG][MAXG][4];
    for (int i = 0; i < n; ++i)
        for (int mu = 0; mu < 4; ++mu) {
            J[i][i][mu] = X->eps[sigma[i]][mu];
            Q[i][i][mu] = X->q[sigma[i]][mu];
        }
    for (int len = 2; len <= n; ++len)
        for (int i = 0; i + len - 1 < n; ++i) {
            const int j = i + len - 1;
            for (int mu = 0; mu < 4; ++mu) Q[i][j][mu] = Q[i][i][mu] + Q[i + 1][j][mu];
            const real Q2 = rdot(Q[i][j], Q[i][j]);
            cplx acc[4] = {0, 0, 0, 0};
            for (int k = i; k < j; ++k) {
                cplx t[4];
                v3(J[i][k], Q[i][k], J[k + 1][j], Q[k + 1][j], t);
                for (int mu = 0; mu < 4; ++mu) acc[mu] += (-g / Q2) * t[mu];
            }
            for (int k = i; k < j; ++k)
                for (int l = k + 1; l < j; ++l) {
                    const cplx *A = J[i][k], *B = J[k + 1][l], *C = J[l + 1][j];
                    const cplx ac = cdot(A, C), ab = cdot(A, B), bc = cdot(B, C);
                    for (int mu = 0; mu < 4; ++mu) acc[mu] += (g * g / Q2) * (2 * ac * B[mu] - ab * C[mu] - bc * A[mu]);
                }
            for (int mu = 0; mu < 4; ++mu) J[i][j][mu] = acc[mu];
        }
    cplx U[MAXG + 1][2][4];
    memcpy(U[0][0], X->row, sizeof(cplx) * 4);
    cplx amp = 0;
    for (int m = 0; m <= n; ++m)
        for (int e = 0; e < 2; ++e) {
            if (m == 0 && e == 0) continue;
            cplx acc[4] = {0, 0, 0, 0};
            for (int l = 0; l < m; ++l) {
                cplx js[4][4], t[4];
                slash_c(J[l][m - 1], js);
                row_mat(U[l][e], js, t);
                for (int a = 0; a < 4; ++a) acc[a] += CI * g * t[a];
            }
            if (e == 1) {
                cplx t[4];
                row_mat(U[m][0], (cplx(*)[4])X->GE, t);
                for (int a = 0; a < 4; ++a) acc[a] += t[a];
            }
            if (m == n && e == 1) {
                amp = row_col(acc, X->col);
                break;
            }
            real P[4];
            for (int mu = 0; mu < 4; ++mu) P[mu] = X->prow[mu] - (m > 0 ? Q[0][m - 1][mu] : 0) - e * X->qE[mu];
            cplx S[4][4];
            fprop(P, 0, 0, S);
            row_mat(acc, S, U[m][e]);
        }
    return amp;
}

static void qew_ordered(const qew_ext *X, cplx *out) {
    int sigma[MAXG];
    for (int i = 0; i < X->n; ++i) sigma[i] = i;
    int k = 0;
    do {
        out[k++] = qew_amp(X, sigma);
    } while (next_perm(sigma, X->n));
}

/* |M|^2 per event: norm x sum over helicities of J^dagger C J, C the colour
 * matrix of the quark line with n gluons ([n!][n!]). */
int oracle_qew(const double *mom, int64_t nevt, const int *desc, const double *cpl, const double *colour,
               double norm, double *out, double *qhel) {
    if (!mom || !desc || !cpl || !colour || !out || nevt < 0) return -1;
    const int n = desc[0], np = desc[1];
    if (n < 0 || n > MAXG - 1 || np > MAXNP) return -1;
    const int ncol = factorial(n), nh = 1 << np;
    real *C = (real *)malloc(sizeof(real) * ncol * ncol);
    for (int i = 0; i < ncol * ncol; ++i) C[i] = colour[i];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ev = 0; ev < nevt; ++ev) {
        real m[4 * MAXNP];
        for (int j = 0; j < 4 * np; ++j) m[j] = mom[4 * np * ev + j];
        cplx J[120];
        real total = 0;
        for (int h = 0; h < nh; ++h) {
            qew_ext X;
            qew_setup(m, desc, cpl, h, -1, 0, &X);
            qew_ordered(&X, J);
            const real qh = colour_form(J, C, ncol);
            if (qhel) qhel[(int64_t)nh * ev + h] = (double)qh;
            total += qh;
        }
        out[ev] = (double)(total * norm);
    }
    free(C);
    return 0;
}

/* Partial amplitudes (n! of them, lexicographic orders) of one event at one
 * helicity; gauge_gluon >= 0 replaces that gluon's polarisation by q/q^0,
 * gauge_ew replaces the insertion's vectors by its momentum.  out: [n!][2]. */
int oracle_qew_amps(const double *mom1, const int *desc, const double *cpl, int h, int gauge_gluon, int gauge_ew,
                    double *out) {
    if (!mom1 || !desc || !cpl || !out) return -1;
    const int n = desc[0], np = desc[1];
    if (n < 0 || n > MAXG - 1 || np > MAXNP) return -1;
    real m[4 * MAXNP];
    for (int j = 0; j < 4 * np; ++j) m[j] = mom1[j];
    qew_ext X;
    qew_setup(m, desc, cpl, h, gauge_gluon, gauge_ew, &X);
    cplx J[120];
    qew_ordered(&X, J);
    for (int k = 0; k < factorial(n); ++k) {
        out[2 * k] = (double)CREAL(J[k]);
        out[2 * k + 1] = (double)CIMAG(J[k]);
    }
    return 0;
}

/* The external pieces of one event at one helicity, for checks against the
 * gluon recursion: gluon q and eps, the row spinor and its momentum, the
 * column spinor, the insertion's momentum and its vector (for a vector-like
 * quark coupling, EL = ER).  out (doubles): q[n][4], eps[n][4][2],
 * prow[4], row[4][2], col[4][2], qE[4], EL[4][2], ER[4][2]. */
static void qew_vectors(const real *mom, const int *d, const double *cpl, int h, cplx EL[4], cplx ER[4]) {
    /* recompute the insertion vectors (the setup keeps only their matrix) */
    const real *pm = mom + 4 * d[6], *pp = mom + 4 * d[7];
    const int np = d[1];
    const int lm = ((h >> (np - 1 - d[6])) & 1) ? 1 : -1, lp = ((h >> (np - 1 - d[7])) & 1) ? 1 : -1;
    cplx um[4], ubm[4], vp[4];
    u_spinor(pm, 0, lm, um);
    bar(um, ubm);
    v_spinor(pp, 0, lp, vp);
    const real e = cpl[0], sw2 = cpl[1], mz = cpl[2], wz = cpl[3];
    const real Qq = cpl[5], T3q = cpl[6], Ql = cpl[7], T3l = cpl[8];
    const real gz = e / RSQRT(sw2 * (1 - sw2));
    const real gLq = T3q - Qq * sw2, gRq = -Qq * sw2, gLl = T3l - Ql * sw2, gRl = -Ql * sw2;
    real k[4];
    for (int mu = 0; mu < 4; ++mu) k[mu] = pm[mu] + pp[mu];
    const real k2 = rdot(k, k);
    const cplx dz = (k2 - mz * mz) + CI * (mz * wz);
    for (int mu = 0; mu < 4; ++mu) {
        cplx t[4], tl[4], tr[4];
        row_mat(ubm, G[mu], t);
        const cplx jg = row_col(t, vp);
        cplx PL[4][4], PR[4][4], GL[4][4], GR[4][4];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                PL[i][j] = ((i == j ? 1 : 0) - G5[i][j]) / 2;
                PR[i][j] = ((i == j ? 1 : 0) + G5[i][j]) / 2;
            }
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cplx a = 0, b = 0;
                for (int l = 0; l < 4; ++l) {
                    a += G[mu][i][l] * PL[l][j];
                    b += G[mu][i][l] * PR[l][j];
                }
                GL[i][j] = a;
                GR[i][j] = b;
            }
        row_mat(ubm, GL, tl);
        row_mat(ubm, GR, tr);
        const cplx jz = gLl * row_col(tl, vp) + gRl * row_col(tr, vp);
        const cplx ga = CI * e * e * Qq * Ql * jg / k2;
        EL[mu] = ga + CI * gz * gz * gLq * jz / dz;
        ER[mu] = ga + CI * gz * gz * gRq * jz / dz;
    }
}

int oracle_qew_externals(const double *mom1, const int *desc, const double *cpl, int h, double *out) {
    if (!mom1 || !desc || !cpl || !out) return -1;
    const int n = desc[0], np = desc[1];
    if (n < 0 || n > MAXG - 1 || np > MAXNP) return -1;
    real m[4 * MAXNP];
    for (int j = 0; j < 4 * np; ++j) m[j] = mom1[j];
    qew_ext X;
    qew_setup(m, desc, cpl, h, -1, 0, &X);
    cplx EL[4], ER[4];
    qew_vectors(m, desc, cpl, h, EL, ER);
    double *o = out;
    for (int a = 0; a < n; ++a)
        for (int mu = 0; mu < 4; ++mu) *o++ = (double)X.q[a][mu];
    for (int a = 0; a < n; ++a)
        for (int mu = 0; mu < 4; ++mu) {
            *o++ = (double)CREAL(X.eps[a][mu]);
            *o++ = (double)CIMAG(X.eps[a][mu]);
        }
    for (int mu = 0; mu < 4; ++mu) *o++ = (double)X.prow[mu];
    for (int i = 0; i < 4; ++i) {
        *o++ = (double)CREAL(X.row[i]);
        *o++ = (double)CIMAG(X.row[i]);
    }
    for (int i = 0; i < 4; ++i) {
        *o++ = (double)CREAL(X.col[i]);
        *o++ = (double)CIMAG(X.col[i]);
    }
    for (int mu = 0; mu < 4; ++mu) *o++ = (double)X.qE[mu];
    for (int mu = 0; mu < 4; ++mu) {
        *o++ = (double)CREAL(EL[mu]);
        *o++ = (double)CIMAG(EL[mu]);
    }
    for (int mu = 0; mu < 4; ++mu) {
        *o++ = (double)CREAL(ER[mu]);
        *o++ = (double)CIMAG(ER[mu]);
    }
    return 0;
}

/* Route 2's colour-ordered amplitude for explicit externals: n gluon-like
 * legs (incoming-flow momenta q[n][4], vectors eps[n][4][2]), row spinor and
 * its momentum, column spinor, line mass and width, coupling g; one order. */
int oracle_bg_custom(int n, const double *q, const double *eps, const double *prow, const double *row,
                     const double *col, double m, double w, double g, const int *sigma, int with4, double *out) {
    if (n < 1 || n > MAXG || !q || !eps || !prow || !row || !col || !sigma || !out) return -1;
    ggx_ext X;
    X.n = n;
    X.mt = m;
    X.wt = w;
    X.gs = g;
    for (int a = 0; a < n; ++a)
        for (int mu = 0; mu < 4; ++mu) {
            X.q[a][mu] = q[4 * a + mu];
            X.eps[a][mu] = eps[8 * a + 2 * mu] + CI * eps[8 * a + 2 * mu + 1];
        }
    for (int mu = 0; mu < 4; ++mu) {
        X.p3[mu] = prow[mu];
        X.ubar3[mu] = row[2 * mu] + CI * row[2 * mu + 1];
        X.v4[mu] = col[2 * mu] + CI * col[2 * mu + 1];
    }
    cplx a;
    bg_amp(&X, sigma, &a, with4);
    out[0] = (double)CREAL(a);
    out[1] = (double)CIMAG(a);
    return 0;
}
