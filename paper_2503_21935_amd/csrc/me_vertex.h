// me_vertex.h -- wavefunctions and vertex functions for one event per lane.
//
// The matrix-element step evaluates Feynman diagrams from external and
// internal wavefunctions and vertex functions (paper Sec. 2-3; the formulas are
// textbook tree-level rules, written here in the chiral representation):
//
//   gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]],  sigma = (1, s), sigmabar = (1, -s)
//   spinor components 0,1 = left-handed, 2,3 = right-handed; metric (+,-,-,-).
//
// Every function is templated on the real type (double for the exact path,
// float for the mixed path) and works on registers only.  Vectors are
// contravariant; "row" spinors are already barred (psi^dagger gamma^0).
#pragma once
#include <hip/hip_runtime.h>

#define MEV __device__ __forceinline__

template <typename T>
struct cx {
    T r, i;
};

template <typename T> MEV cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> MEV cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T> MEV cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T> MEV cx<T> operator-(cx<T> a) { return {-a.r, -a.i}; }
template <typename T> MEV cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T> MEV cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <typename T> MEV cx<T> operator*(cx<T> a, T s) { return {s * a.r, s * a.i}; }
template <typename T> MEV cx<T>& operator+=(cx<T>& a, cx<T> b) { a.r += b.r; a.i += b.i; return a; }
template <typename T> MEV cx<T>& operator-=(cx<T>& a, cx<T> b) { a.r -= b.r; a.i -= b.i; return a; }
template <typename T> MEV cx<T> conj(cx<T> a) { return {a.r, -a.i}; }
template <typename T> MEV cx<T> times_i(cx<T> a) { return {-a.i, a.r}; }
template <typename T> MEV cx<T> times_mi(cx<T> a) { return {a.i, -a.r}; }
// a + s * b with real s (one fma per component)
template <typename T> MEV cx<T> axpy(T s, cx<T> b, cx<T> a) { return {fma(s, b.r, a.r), fma(s, b.i, a.i)}; }
// a + b * c
template <typename T> MEV cx<T> cfma(cx<T> b, cx<T> c, cx<T> a) {
    return {fma(b.r, c.r, fma(-b.i, c.i, a.r)), fma(b.r, c.i, fma(b.i, c.r, a.i))};
}

template <typename T>
struct vec4 {  // complex 4-vector
    cx<T> v[4];
};
template <typename T>
struct spinor {  // Dirac spinor, chiral components
    cx<T> s[4];
};
template <typename T>
struct mom4 {  // real 4-vector
    T e, x, y, z;
};

template <typename T> MEV mom4<T> operator+(mom4<T> a, mom4<T> b) { return {a.e + b.e, a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T> MEV mom4<T> operator-(mom4<T> a, mom4<T> b) { return {a.e - b.e, a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T> MEV mom4<T> operator-(mom4<T> a) { return {-a.e, -a.x, -a.y, -a.z}; }
// Opaque copy: the optimiser may not assume the outputs equal the inputs.
template <typename T>
MEV void fence1(mom4<T>& q) {
    asm volatile("" : "+v"(q.e), "+v"(q.x), "+v"(q.y), "+v"(q.z));
}
template <typename... M>
MEV void fence(M&... m) {
    (fence1(m), ...);
    __builtin_amdgcn_sched_barrier(0);  // keep the emitted node order
}

// Opaque copies of wavefunctions: each use sees a fresh value, so the
// optimiser cannot merge subexpressions of one wavefunction across its uses
// (which would keep those subexpressions alive between the uses).
template <typename T>
MEV vec4<T> opq(vec4<T> a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(a.v[k].r), "+v"(a.v[k].i));
    return a;
}
template <typename T>
MEV spinor<T> opq(spinor<T> a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(a.s[k].r), "+v"(a.s[k].i));
    return a;
}

// Conversions from the float64 momentum algebra to the amplitude type.
template <typename T> MEV mom4<T> to_t(const mom4<double>& p) { return {T(p.e), T(p.x), T(p.y), T(p.z)}; }
template <typename T> MEV cx<T> to_t(const cx<double>& c) { return {T(c.r), T(c.i)}; }

template <typename T> MEV T msq(mom4<T> p) { return p.e * p.e - p.x * p.x - p.y * p.y - p.z * p.z; }

// Minkowski product of complex 4-vectors
template <typename T> MEV cx<T> dot(const vec4<T>& a, const vec4<T>& b) {
    cx<T> r = a.v[0] * b.v[0];
    r = cfma(-a.v[1], b.v[1], r);
    r = cfma(-a.v[2], b.v[2], r);
    r = cfma(-a.v[3], b.v[3], r);
    return r;
}
// Minkowski product of a real and a complex 4-vector
template <typename T> MEV cx<T> dot(mom4<T> q, const vec4<T>& b) {
    cx<T> r = q.e * b.v[0];
    r = axpy(-q.x, b.v[1], r);
    r = axpy(-q.y, b.v[2], r);
    r = axpy(-q.z, b.v[3], r);
    return r;
}

// --------------------------------------------------------------------------
// External wavefunctions
// --------------------------------------------------------------------------

// Transverse helicity vector eps(k, lam) = (-lam e1 - i e2)/sqrt2 with
// e1 = (cos th cos ph, cos th sin ph, -sin th), e2 = (-sin ph, cos ph, 0), time
// component zero in the frame of the given momenta.  Outgoing gluons take the
// complex conjugate.
template <typename T>
MEV vec4<T> gluon_eps(mom4<T> k, int lam, bool outgoing) {
    T kt2 = k.x * k.x + k.y * k.y;
    T kk = sqrt(kt2 + k.z * k.z);
    T kt = sqrt(kt2);
    // Along the z axis (the beams) the azimuth is taken as 0.  Both cases are
    // computed and selected without a branch: the off-axis values are the
    // same operations as in a branch, and a branch here makes the compiler
    // spill around it in every helicity.
    const bool axis = !(kt > T(0));
    const T ikt = T(1) / kt, ikk = T(1) / kk;
    const T c = k.z * ikk;
    const T e1x = axis ? ((k.z >= T(0)) ? T(1) : T(-1)) : c * k.x * ikt;
    const T e1y = axis ? T(0) : c * k.y * ikt;
    const T e1z = axis ? T(0) : -kt * ikk;
    const T e2x = axis ? T(0) : -k.y * ikt;
    const T e2y = axis ? T(1) : k.x * ikt;
    const T r2 = T(0.70710678118654752440);
    T s = -T(lam) * r2;
    T ims = outgoing ? r2 : -r2;  // imaginary part coefficient of e2
    vec4<T> e;
    e.v[0] = mk(T(0), T(0));
    e.v[1] = mk(s * e1x, ims * e2x);
    e.v[2] = mk(s * e1y, ims * e2y);
    e.v[3] = mk(s * e1z, T(0));
    return e;
}

// Two-component helicity eigenstates of s.p/|p| for lam = +-1:
//   chi_+ = (cos th/2, e^{i ph} sin th/2),  chi_- = (-e^{-i ph} sin th/2, cos th/2),
// evaluated from components; |p| + p_z is taken as pT^2/(|p| - p_z) when p_z < 0.
template <typename T>
MEV void helicity_chi(mom4<T> p, T pabs, int lam, cx<T>& c0, cx<T>& c1) {
    T pt2 = p.x * p.x + p.y * p.y;
    // pT^2 / (|p| - p_z) is |p| + p_z without cancellation when p_z < 0;
    // both forms are computed and one selected (no branch, as in gluon_eps)
    const T ppz = (p.z >= T(0)) ? pabs + p.z : pt2 / (pabs - p.z);
    const bool minus_z = !(pt2 > T(0) || p.z > T(0));  // along -z: theta = pi, azimuth 0
    const T n = T(1) / sqrt(T(2) * pabs * ppz);
    const T c = ppz * n;  // cos(th/2)
    const cx<T> se = mk(p.x * n, p.y * n);  // e^{i ph} sin(th/2)
    if (lam > 0) {
        c0 = minus_z ? mk(T(0), T(0)) : mk(c, T(0));
        c1 = minus_z ? mk(T(1), T(0)) : se;
    } else {
        const cx<T> mse = -conj(se);
        c0 = minus_z ? mk(T(-1), T(0)) : mse;
        c1 = minus_z ? mk(T(0), T(0)) : mk(c, T(0));
    }
}

// sqrt(E - |p|) and sqrt(E + |p|); E - |p| = m^2/(E + |p|) avoids cancellation.
template <typename T>
MEV void spinor_weights(mom4<T> p, T m, T& pabs, T& wminus, T& wplus) {
    pabs = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
    T ep = p.e + pabs;
    wplus = sqrt(ep);
    wminus = (m > T(0)) ? m / wplus : T(0);
}

// u(p, lam) = (sqrt(E - lam|p|) chi_lam, sqrt(E + lam|p|) chi_lam)
template <typename T>
MEV spinor<T> u_spinor(mom4<T> p, T m, int lam) {
    T pabs, wm, wp;
    spinor_weights(p, m, pabs, wm, wp);
    cx<T> c0, c1;
    helicity_chi(p, pabs, lam, c0, c1);
    T a = (lam > 0) ? wm : wp, b = (lam > 0) ? wp : wm;
    spinor<T> u;
    u.s[0] = a * c0;
    u.s[1] = a * c1;
    u.s[2] = b * c0;
    u.s[3] = b * c1;
    return u;
}

// v(p, lam) = (sqrt(E + lam|p|) chi_-lam, -sqrt(E - lam|p|) chi_-lam)
template <typename T>
MEV spinor<T> v_spinor(mom4<T> p, T m, int lam) {
    T pabs, wm, wp;
    spinor_weights(p, m, pabs, wm, wp);
    cx<T> c0, c1;
    helicity_chi(p, pabs, -lam, c0, c1);
    T a = (lam > 0) ? wp : wm, b = (lam > 0) ? -wm : -wp;
    spinor<T> v;
    v.s[0] = a * c0;
    v.s[1] = a * c1;
    v.s[2] = b * c0;
    v.s[3] = b * c1;
    return v;
}

// psibar = psi^dagger gamma^0: swap chiral halves and conjugate.
template <typename T>
MEV spinor<T> bar(const spinor<T>& u) {
    spinor<T> r;
    r.s[0] = conj(u.s[2]);
    r.s[1] = conj(u.s[3]);
    r.s[2] = conj(u.s[0]);
    r.s[3] = conj(u.s[1]);
    return r;
}

// --------------------------------------------------------------------------
// Fermion-line algebra
// --------------------------------------------------------------------------

// row * (gamma.W)
template <typename T>
MEV spinor<T> row_slash(const spinor<T>& f, const vec4<T>& W) {
    cx<T> a = W.v[0] + W.v[3], b = W.v[0] - W.v[3];
    cx<T> c = W.v[1] + times_i(W.v[2]), d = W.v[1] - times_i(W.v[2]);
    spinor<T> o;
    o.s[0] = cfma(f.s[2], a, f.s[3] * c);
    o.s[1] = cfma(f.s[2], d, f.s[3] * b);
    o.s[2] = cfma(f.s[0], b, -(f.s[1] * c));
    o.s[3] = cfma(f.s[1], a, -(f.s[0] * d));
    return o;
}

// row * (gamma.EL P_L + gamma.ER P_R): a vector insertion with different
// left- and right-handed couplings (P_L keeps the first two components of the
// column it acts on), as row_slash with EL in the first half of the result
// and ER in the second.
template <typename T>
MEV spinor<T> row_ew(const spinor<T>& f, const vec4<T>& EL, const vec4<T>& ER) {
    const cx<T> a = EL.v[0] + EL.v[3], b = EL.v[0] - EL.v[3];
    const cx<T> c = EL.v[1] + times_i(EL.v[2]), d = EL.v[1] - times_i(EL.v[2]);
    const cx<T> A = ER.v[0] + ER.v[3], B = ER.v[0] - ER.v[3];
    const cx<T> C = ER.v[1] + times_i(ER.v[2]), D = ER.v[1] - times_i(ER.v[2]);
    spinor<T> o;
    o.s[0] = cfma(f.s[2], a, f.s[3] * c);
    o.s[1] = cfma(f.s[2], d, f.s[3] * b);
    o.s[2] = cfma(f.s[0], B, -(f.s[1] * C));
    o.s[3] = cfma(f.s[1], A, -(f.s[0] * D));
    return o;
}

// (gamma.EL P_L + gamma.ER P_R) * column
template <typename T>
MEV spinor<T> ew_col(const vec4<T>& EL, const vec4<T>& ER, const spinor<T>& p) {
    const cx<T> a = EL.v[0] + EL.v[3], b = EL.v[0] - EL.v[3];
    const cx<T> c = EL.v[1] + times_i(EL.v[2]), d = EL.v[1] - times_i(EL.v[2]);
    const cx<T> A = ER.v[0] + ER.v[3], B = ER.v[0] - ER.v[3];
    const cx<T> C = ER.v[1] + times_i(ER.v[2]), D = ER.v[1] - times_i(ER.v[2]);
    spinor<T> o;
    o.s[0] = cfma(B, p.s[2], -(D * p.s[3]));
    o.s[1] = cfma(A, p.s[3], -(C * p.s[2]));
    o.s[2] = cfma(a, p.s[0], d * p.s[1]);
    o.s[3] = cfma(c, p.s[0], b * p.s[1]);
    return o;
}

// (gamma.W) * column
template <typename T>
MEV spinor<T> slash_col(const vec4<T>& W, const spinor<T>& p) {
    cx<T> a = W.v[0] + W.v[3], b = W.v[0] - W.v[3];
    cx<T> c = W.v[1] + times_i(W.v[2]), d = W.v[1] - times_i(W.v[2]);
    spinor<T> o;
    o.s[0] = cfma(b, p.s[2], -(d * p.s[3]));
    o.s[1] = cfma(a, p.s[3], -(c * p.s[2]));
    o.s[2] = cfma(a, p.s[0], d * p.s[1]);
    o.s[3] = cfma(c, p.s[0], b * p.s[1]);
    return o;
}

// row * (pslash + m), real P
template <typename T>
MEV spinor<T> row_prop(const spinor<T>& f, mom4<T> P, T m) {
    T a = P.e + P.z, b = P.e - P.z;
    cx<T> c = mk(P.x, P.y), d = mk(P.x, -P.y);
    spinor<T> o;
    o.s[0] = axpy(a, f.s[2], axpy(m, f.s[0], f.s[3] * c));
    o.s[1] = axpy(b, f.s[3], axpy(m, f.s[1], f.s[2] * d));
    o.s[2] = axpy(b, f.s[0], axpy(m, f.s[2], -(f.s[1] * c)));
    o.s[3] = axpy(a, f.s[1], axpy(m, f.s[3], -(f.s[0] * d)));
    return o;
}

// (pslash + m) * column, real P
template <typename T>
MEV spinor<T> prop_col(mom4<T> P, T m, const spinor<T>& p) {
    T a = P.e + P.z, b = P.e - P.z;
    cx<T> c = mk(P.x, P.y), d = mk(P.x, -P.y);
    spinor<T> o;
    o.s[0] = axpy(b, p.s[2], axpy(m, p.s[0], -(d * p.s[3])));
    o.s[1] = axpy(a, p.s[3], axpy(m, p.s[1], -(c * p.s[2])));
    o.s[2] = axpy(a, p.s[0], axpy(m, p.s[2], d * p.s[1]));
    o.s[3] = axpy(b, p.s[1], axpy(m, p.s[3], c * p.s[0]));
    return o;
}

template <typename T>
MEV spinor<T> scale(cx<T> s, const spinor<T>& f) {
    spinor<T> o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o.s[k] = s * f.s[k];
    return o;
}

template <typename T>
MEV cx<T> row_col(const spinor<T>& f, const spinor<T>& p) {
    cx<T> r = f.s[0] * p.s[0];
    r = cfma(f.s[1], p.s[1], r);
    r = cfma(f.s[2], p.s[2], r);
    r = cfma(f.s[3], p.s[3], r);
    return r;
}

// Vector current fbar gamma^mu psi, split into the parts through P_L and P_R:
//   left  = (f2, f3) sigmabar^mu (p0, p1),  right = (f0, f1) sigma^mu (p2, p3)
template <typename T>
MEV void fbar_gamma_f_lr(const spinor<T>& f, const spinor<T>& p, vec4<T>& L, vec4<T>& R) {
    cx<T> f0p2 = f.s[0] * p.s[2], f1p3 = f.s[1] * p.s[3], f0p3 = f.s[0] * p.s[3], f1p2 = f.s[1] * p.s[2];
    cx<T> f2p0 = f.s[2] * p.s[0], f3p1 = f.s[3] * p.s[1], f2p1 = f.s[2] * p.s[1], f3p0 = f.s[3] * p.s[0];
    R.v[0] = f0p2 + f1p3;
    R.v[1] = f0p3 + f1p2;
    R.v[2] = times_i(f1p2 - f0p3);
    R.v[3] = f0p2 - f1p3;
    L.v[0] = f2p0 + f3p1;
    L.v[1] = -(f2p1 + f3p0);
    L.v[2] = times_i(f2p1 - f3p0);
    L.v[3] = f3p1 - f2p0;
}

template <typename T>
MEV vec4<T> fbar_gamma_f(const spinor<T>& f, const spinor<T>& p) {
    vec4<T> L, R, o;
    fbar_gamma_f_lr(f, p, L, R);
#pragma unroll
    for (int k = 0; k < 4; ++k) o.v[k] = L.v[k] + R.v[k];
    return o;
}

// --------------------------------------------------------------------------
// Gluon self-interactions
// --------------------------------------------------------------------------

// V(QX, QY, -QX-QY)_{mu nu rho} X^mu Y^nu with the free index raised:
//   (X.Y)(QX - QY) + Y ((QX + 2 QY).X) - X ((2 QX + QY).Y)
template <typename T>
MEV vec4<T> vvv(const vec4<T>& X, mom4<T> QX, const vec4<T>& Y, mom4<T> QY) {
    cx<T> xy = dot(X, Y);
    mom4<T> a = {QX.e + T(2) * QY.e, QX.x + T(2) * QY.x, QX.y + T(2) * QY.y, QX.z + T(2) * QY.z};
    mom4<T> b = {T(2) * QX.e + QY.e, T(2) * QX.x + QY.x, T(2) * QX.y + QY.y, T(2) * QX.z + QY.z};
    cx<T> ax = dot(a, X), by = dot(b, Y);
    T d[4] = {QX.e - QY.e, QX.x - QY.x, QX.y - QY.y, QX.z - QY.z};
    vec4<T> o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o.v[k] = cfma(Y.v[k], ax, axpy(d[k], xy, -(X.v[k] * by)));
    return o;
}

// Four-gluon colour channels contracted with X, Y, Z (free index raised):
//   ch 0: (X.Z) Y - (Y.Z) X    ch 1: (X.Y) Z - (Y.Z) X    ch 2: (X.Y) Z - (X.Z) Y
template <typename T>
MEV vec4<T> vvvv(const vec4<T>& X, const vec4<T>& Y, const vec4<T>& Z, int ch) {
    vec4<T> o;
    if (ch == 0) {
        cx<T> xz = dot(X, Z), yz = dot(Y, Z);
#pragma unroll
        for (int k = 0; k < 4; ++k) o.v[k] = cfma(xz, Y.v[k], -(yz * X.v[k]));
    } else if (ch == 1) {
        cx<T> xy = dot(X, Y), yz = dot(Y, Z);
#pragma unroll
        for (int k = 0; k < 4; ++k) o.v[k] = cfma(xy, Z.v[k], -(yz * X.v[k]));
    } else {
        cx<T> xy = dot(X, Y), xz = dot(X, Z);
#pragma unroll
        for (int k = 0; k < 4; ++k) o.v[k] = cfma(xy, Z.v[k], -(xz * Y.v[k]));
    }
    return o;
}

template <typename T>
MEV vec4<T> vscale(cx<T> s, const vec4<T>& a) {
    vec4<T> o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o.v[k] = s * a.v[k];
    return o;
}

template <typename T>
MEV vec4<T> vscale(T s, const vec4<T>& a) {
    vec4<T> o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o.v[k] = s * a.v[k];
    return o;
}

template <typename T>
MEV void vacc(vec4<T>& acc, cx<T> c, const vec4<T>& a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.v[k] = cfma(c, a.v[k], acc.v[k]);
}

template <typename T>
MEV void vadd(vec4<T>& acc, const vec4<T>& a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.v[k] += a.v[k];
}

template <typename T>
MEV void vsub(vec4<T>& acc, const vec4<T>& a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.v[k] -= a.v[k];
}

template <typename T>
MEV void vadd_i(vec4<T>& acc, const vec4<T>& a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.v[k] += times_i(a.v[k]);
}

template <typename T>
MEV void vsub_i(vec4<T>& acc, const vec4<T>& a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.v[k] -= times_i(a.v[k]);
}

// 1 / (re + i im)
template <typename T>
MEV cx<T> crecip(T re, T im) {
    T d = T(1) / (re * re + im * im);
    return mk(re * d, -im * d);
}
