// me_qew.h -- the per-event |M|^2 kernel of the quark-line + lepton-pair
// processes (a massless quark line with gluons and one photon/Z insertion
// decaying to a lepton pair; g ubar -> tau+ tau- g g ubar is the DY+3j
// subprocess of the paper's Sec. 3).  One event per lane, helicities looped
// (or spread over 2^lg lanes), as the gluon-process kernel: externals, the
// generated diagram program into the colour-flow amplitudes J, the colour sum.
#pragma once
#include "me_kernels.h"

// Momentum slots of the LDS tile: gluons 0..NG-1 flowing into the diagram,
// NG the fermion-flow momentum leaving the row end, NG+1 the one leaving the
// column end, NG+2 the insertion's inflowing momentum -(p(l-) + p(l+)), NG+3
// and NG+4 the lepton momenta.
template <class P>
MEV void qew_setup(qew_ext<double, P::ngluon>& x, const double* __restrict__ mom, int64_t ev, double* Qt, int lane,
                   const me_params& prm) {
    constexpr int NG = P::ngluon;
    const double* pe = mom + ev * (P::npart * 4);
    auto put = [&](int slot, double sg, const double* p) {
#pragma unroll
        for (int c = 0; c < 4; ++c) Qt[ME_MOM_ROW(slot) + c * 64 + lane] = sg * p[c];
    };
#pragma unroll
    for (int a = 0; a < NG; ++a) put(a, P::gluon_in[a] ? 1.0 : -1.0, pe + 4 * P::gluon_part[a]);
    put(NG, P::row_in ? -1.0 : 1.0, pe + 4 * P::row_part);
    put(NG + 1, P::col_in ? -1.0 : 1.0, pe + 4 * P::col_part);
    const double* pm = pe + 4 * P::lm_part;
    const double* pp = pe + 4 * P::lp_part;
    const double qE[4] = {-(pm[0] + pp[0]), -(pm[1] + pp[1]), -(pm[2] + pp[2]), -(pm[3] + pp[3])};
    put(NG + 2, 1.0, qE);
    put(NG + 3, 1.0, pm);
    put(NG + 4, 1.0, pp);
    x.Q = (lds_cdouble*)(Qt + lane);
    x.m = 0.0;
    x.mw = 0.0;
    x.g = prm.gs;
    x.mT = 0.0;
    x.gT = prm.gs;
}

// External wavefunctions of one helicity: gluon polarisations, the quark
// line's end spinors, and the insertion
//   EX = i e^2 Qq Ql Jg / k^2 + i gZ^2 gX(q) JZ / (k^2 - MZ^2 + i MZ WZ),  X = L, R,
// with Jg = ubar(l-) gamma v(l+), JZ = gL(l) JL + gR(l) JR its chiral parts
// weighted with the lepton's Z charges, gL = T3 - Q sin^2, gR = -Q sin^2,
// k = p(l-) + p(l+): the photon and Z vertices and propagators of both lines
// (the k k / MZ^2 part of the Z propagator vanishes on the massless lepton
// current).
template <class P>
MEV void qew_externals(qew_ext<double, P::ngluon>& x, int h, const me_params& prm) {
    constexpr int NP = P::npart, NG = P::ngluon;
#pragma unroll
    for (int a = 0; a < NG; ++a) {
        const mom4<double> q = mom_ld(x, a);
        x.eps[a] = gluon_eps(P::gluon_in[a] ? q : -q, helicity_of<NP>(h, P::gluon_part[a]), !P::gluon_in[a]);
    }
    {
        const mom4<double> q = mom_ld(x, NG);
        const mom4<double> p = P::row_in ? -q : q;
        const int l = helicity_of<NP>(h, P::row_part);
        x.ubar3 = bar(P::row_in ? v_spinor(p, 0.0, l) : u_spinor(p, 0.0, l));
    }
    {
        const mom4<double> q = mom_ld(x, NG + 1);
        const mom4<double> p = P::col_in ? -q : q;
        const int l = helicity_of<NP>(h, P::col_part);
        x.v4 = P::col_in ? u_spinor(p, 0.0, l) : v_spinor(p, 0.0, l);
    }
    const mom4<double> pm = mom_ld(x, NG + 3), pp = mom_ld(x, NG + 4);
    const spinor<double> ub = bar(u_spinor(pm, 0.0, helicity_of<NP>(h, P::lm_part)));
    const spinor<double> v = v_spinor(pp, 0.0, helicity_of<NP>(h, P::lp_part));
    vec4<double> jl, jr;
    fbar_gamma_f_lr(ub, v, jl, jr);
    const double k2 = msq(pm + pp);
    const double sw2 = prm.sw2, gz2 = prm.gz * prm.gz;
    const double gl_q = P::q_t3 - P::q_charge * sw2, gr_q = -P::q_charge * sw2;
    const double gl_l = P::l_t3 - P::l_charge * sw2, gr_l = -P::l_charge * sw2;
    const cx<double> iz = times_i(crecip(k2 - prm.mz * prm.mz, prm.mz * prm.wz));  // i / D_Z
    const double ga = prm.e * prm.e * P::q_charge * P::l_charge / k2;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const cx<double> jg = jl.v[c] + jr.v[c];
        const cx<double> jz = gl_l * jl.v[c] + gr_l * jr.v[c];
        const cx<double> a = times_i(ga * jg);
        const cx<double> zz = iz * jz;
        x.EL.v[c] = a + (gz2 * gl_q) * zz;
        x.ER.v[c] = a + (gz2 * gr_q) * zz;
    }
}

// qhel, idx, count and lg as for k_me_gg.
template <class P>
__global__ __launch_bounds__(ME_BLOCK) void k_me_qew(const double* __restrict__ mom, int64_t nevt,
                                                     double* __restrict__ out, const int* __restrict__ hels,
                                                     int nh, me_params prm, double* __restrict__ qhel,
                                                     const int* __restrict__ idx, const int* __restrict__ count,
                                                     int lg) {
    const int grp = threadIdx.x & ((1 << lg) - 1);
    int64_t ev = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lg;
    if (count) {
        if (ev >= *count) return;
        ev = idx[ev];
    } else if (ev >= nevt) {
        return;
    }
    using T = double;
    constexpr int NG = P::ngluon;
    static_assert(ME_BLOCK == 64, "one wave per block");
    __shared__ double Qt[ME_MOM_ROW(NG + 5)];
    qew_ext<T, NG> x;
    qew_setup<P>(x, mom, ev, Qt, threadIdx.x, prm);
    T acc = T(0);
#pragma unroll 1
    for (int ih = grp; ih < nh; ih += 1 << lg) {
        const int h = hels[ih];
        qew_externals<P>(x, h, prm);
        cx<T> J[P::ncol];
#pragma unroll
        for (int k = 0; k < P::ncol; ++k) J[k] = mk(T(0), T(0));
        P::template amps<T>(x, J);
        const T q = P::template colour_sum<T>(J);
        if (qhel) qhel[ev * P::nhel + h] = double(q) / P::lcd;
        acc += q;
    }
    const double tot = group_sum(double(acc), lg);
    if (grp == 0) out[ev] = tot * (1.0 / (P::avg * P::lcd));
}
