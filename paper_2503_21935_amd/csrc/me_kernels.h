// me_kernels.h -- the per-event |M|^2 kernels (one event per lane).
//
// For each event the kernel loads its momenta, loops over the helicity
// combinations handed in, builds the external wavefunctions, runs the
// process's generated diagram program into the colour-flow amplitudes J,
// takes the colour sum J^dag C J and accumulates over helicities (the
// matrix-element step of the paper, Sec. 2-3).  The result is averaged over
// initial spins and colours and divided by the identical-particle factor.
#pragma once
#include "me_launch.h"

template <int NPART>
MEV int helicity_of(int h, int i) {
    return ((h >> (NPART - 1 - i)) & 1) ? 1 : -1;
}

template <typename T>
MEV void opaque_mom(mom4<T>& q) {
    asm volatile("" : "+v"(q.e), "+v"(q.x), "+v"(q.y), "+v"(q.z));
}

template <typename T>
MEV void opaque(mom4<T>* p, int n) {
#pragma unroll
    for (int i = 0; i < n; ++i) opaque_mom(p[i]);
}

template <typename T, int NP>
MEV void load_event(const double* __restrict__ mom, int64_t ev, mom4<T>* p) {
    const double2* pe = reinterpret_cast<const double2*>(mom + ev * (NP * 4));
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const double2 a = pe[2 * i], b = pe[2 * i + 1];
        p[i] = mom4<T>{T(a.x), T(a.y), T(b.x), T(b.y)};
    }
}

// Wavefunctions of one helicity in the amplitude type T (built in float64
// from the momenta in LDS: incoming gluons p = q, outgoing p = -q).
template <class P, typename T>
MEV void gg_externals(gg_ext<T, P::ngluon>& x, int h) {
    constexpr int NP = P::npart, NG = P::ngluon;
#pragma unroll
    for (int a = 0; a < NG; ++a) {
        const int ip = (a < 2) ? a : a + 2;
        const mom4<double> q = mom_ld(x, a);
        const vec4<double> e = gluon_eps((a < 2) ? q : -q, helicity_of<NP>(h, ip), a >= 2);
#pragma unroll
        for (int c = 0; c < 4; ++c) x.eps[a].v[c] = to_t<T>(e.v[c]);
    }
    const spinor<double> u = bar(u_spinor(mom_ld(x, NG), x.m, helicity_of<NP>(h, 2)));
    const spinor<double> v = v_spinor(mom_ld(x, NG + 1), x.m, helicity_of<NP>(h, 3));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        x.ubar3.s[c] = to_t<T>(u.s[c]);
        x.v4.s[c] = to_t<T>(v.s[c]);
    }
}

// Writes this lane's event into its column of the block's momentum tile Qt
// (slots as described at gg_ext) and points x at it.  Each lane reads back
// only its own column, which the same wave wrote before: no barrier needed.
template <class P, typename T>
MEV void gg_setup(gg_ext<T, P::ngluon>& x, const double* __restrict__ mom, int64_t ev, double* Qt, int lane,
                  const me_params& prm) {
    constexpr int NP = P::npart, NG = P::ngluon;
    const double2* pe = reinterpret_cast<const double2*>(mom + ev * (NP * 4));
#pragma unroll
    for (int r = 0; r < NG + 2; ++r) {
        const int ip = (r < 2) ? r : (r < NG) ? r + 2 : r - NG + 2;
        const double sg = (r >= 2 && r < NG) ? -1.0 : 1.0;
        const double2 a = pe[2 * ip], b = pe[2 * ip + 1];
        Qt[ME_MOM_ROW(r) + 0 * 64 + lane] = sg * a.x;
        Qt[ME_MOM_ROW(r) + 1 * 64 + lane] = sg * a.y;
        Qt[ME_MOM_ROW(r) + 2 * 64 + lane] = sg * b.x;
        Qt[ME_MOM_ROW(r) + 3 * 64 + lane] = sg * b.y;
    }
    x.Q = (lds_cdouble*)(Qt + lane);
    x.m = prm.mt;
    x.mw = prm.mt * prm.wt;
    x.g = prm.gs;
    x.mT = T(prm.mt);
    x.gT = T(prm.gs);
}

// qhel (optional): per-helicity J^dag C J, [nevt][P::nhel], for the helicity
// filter and for tests; entries of helicities not in the list are untouched.
// idx (optional): evaluate only events idx[0..*count) (the float64 rerun of
// events flagged by the mixed-precision kernel); out is indexed the same way.
template <class P>
__global__ __launch_bounds__(ME_BLOCK) void k_me_gg(const double* __restrict__ mom, int64_t nevt,
                                                    double* __restrict__ out, const int* __restrict__ hels,
                                                    int nh, me_params prm, double* __restrict__ qhel,
                                                    const int* __restrict__ idx, const int* __restrict__ count) {
    int64_t ev = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (count) {
        if (ev >= *count) return;
        ev = idx[ev];
    } else if (ev >= nevt) {
        return;
    }
    using T = double;
    constexpr int NG = P::ngluon;
    static_assert(ME_BLOCK == 64, "one wave per block");
    __shared__ double Qt[ME_MOM_ROW(NG + 2)];
    gg_ext<T, NG> x;
    gg_setup<P, T>(x, mom, ev, Qt, threadIdx.x, prm);
    T acc = T(0);
#pragma unroll 1
    for (int ih = 0; ih < nh; ++ih) {
        const int h = hels[ih];
        // The momenta are read from LDS where they are used: the
        // helicity-independent subexpressions are recomputed per helicity
        // instead of being hoisted out of the loop into registers.
        gg_externals<P, T>(x, h);
        cx<T> J[P::ncol];
#pragma unroll
        for (int k = 0; k < P::ncol; ++k) J[k] = mk(T(0), T(0));
        P::template amps<T>(x, J);
        const T q = P::template colour_sum<T>(J);
        if (qhel) qhel[ev * P::nhel + h] = double(q) / P::lcd;
        acc += q;
    }
    out[ev] = double(acc) * (1.0 / (256.0 * P::identical * P::lcd));
}

template <class P>
__global__ __launch_bounds__(ME_BLOCK) void k_me_ee(const double* __restrict__ mom, int64_t nevt,
                                                    double* __restrict__ out, const int* __restrict__ hels,
                                                    int nh, me_params prm, double* __restrict__ qhel,
                                                    const int* __restrict__ idx, const int* __restrict__ count) {
    int64_t ev = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (count) {
        if (ev >= *count) return;
        ev = idx[ev];
    } else if (ev >= nevt) {
        return;
    }
    using T = double;
    mom4<T> p[P::npart];
    load_event<T, P::npart>(mom, ev, p);
    T acc = T(0);
    for (int ih = 0; ih < nh; ++ih) {
        const int h = hels[ih];
        const T q = P::template me_hel<T>(p, h, prm);
        if (qhel) qhel[ev * P::nhel + h] = double(q);
        acc += q;
    }
    out[ev] = double(acc) * 0.25;
}
