// me_kernels.h -- the per-event |M|^2 kernels (one event per lane).
//
// For each event the kernel loads its momenta, loops over the helicity
// combinations handed in, builds the external wavefunctions, runs the
// process's generated diagram program into the colour-flow amplitudes J,
// takes the colour sum J^dag C J and accumulates over helicities (the
// matrix-element step of the paper, Sec. 2-3).  The result is averaged over
// initial spins and colours and divided by the identical-particle factor.
#pragma once
#include "me_colour_mfma.h"
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

// Sum of v over the 2^lg adjacent lanes that share an event (lanes
// e 2^lg .. e 2^lg + 2^lg - 1); every lane of the group receives the sum.
MEV double group_sum(double v, int lg) {
#pragma unroll 1
    for (int off = (1 << lg) >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// qhel (optional): per-helicity J^dag C J, [nevt][P::nhel], for the helicity
// filter and for tests; entries of helicities not in the list are untouched.
// idx (optional): evaluate only events idx[0..*count) (the float64 rerun of
// events flagged by the mixed-precision kernel); out is indexed the same way.
// lg: helicity parallelism, 2^lg lanes per event (0 <= lg <= 6): lane
// g = lane % 2^lg of an event takes the helicities ih = g, g + 2^lg, ... of
// the list, and the group's partial sums are added across its lanes at the
// end, so a block of 64 lanes holds 64 / 2^lg events (the paper's
// helicity-level parallelism, Sec. 2: fewer events in flight fill the GPU).
template <class P>
__global__ __launch_bounds__(ME_BLOCK) void k_me_gg(const double* __restrict__ mom, int64_t nevt,
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
    __shared__ double Qt[ME_MOM_ROW(NG + 2)];
    gg_ext<T, NG> x;
    gg_setup<P, T>(x, mom, ev, Qt, threadIdx.x, prm);
    T acc = T(0);
#pragma unroll 1
    for (int ih = grp; ih < nh; ih += 1 << lg) {
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
    // the lanes of one event are all valid or all returned above
    const double tot = group_sum(double(acc), lg);
    if (grp == 0) out[ev] = tot * (1.0 / (256.0 * P::identical * P::lcd));
}

// The same evaluation with the colour sum on the matrix cores: after each
// helicity's program the wave stages its 64 lanes' J in LDS as
// [flow][re, im][lane] and the four 16-lane column blocks go through
// colour_mfma16 (float64 MFMA GEMM, me_colour_mfma.h).  The MFMA needs all 64
// lanes, so lanes past the end repeat the last event (no store) and every
// lane makes the same number of helicity passes.
template <class P>
__global__ __launch_bounds__(ME_BLOCK) void k_me_gg_cm(const double* __restrict__ mom, int64_t nevt,
                                                       double* __restrict__ out, const int* __restrict__ hels,
                                                       int nh, me_params prm, double* __restrict__ qhel,
                                                       const int* __restrict__ idx, const int* __restrict__ count,
                                                       int lg) {
    const int lane = threadIdx.x;
    const int grp = lane & ((1 << lg) - 1);
    const int64_t n = count ? (int64_t)*count : nevt;
    const int64_t first = ((int64_t)blockIdx.x * ME_BLOCK) >> lg;
    if (first >= n) return;  // the whole block
    int64_t i = first + (lane >> lg);
    const bool valid = i < n;
    if (!valid) i = n - 1;
    const int64_t ev = count ? (int64_t)idx[i] : i;
    using T = double;
    constexpr int NG = P::ngluon;
    static_assert(ME_BLOCK == 64, "one wave per block");
    __shared__ double Qt[ME_MOM_ROW(NG + 2)];
    __shared__ double Jt[P::ncol * 2 * ME_BLOCK];
    const double* frag = colour_table<P>::mfma_frag();
    gg_ext<T, NG> x;
    gg_setup<P, T>(x, mom, ev, Qt, lane, prm);
    T acc = T(0);
    const int passes = (nh + (1 << lg) - 1) >> lg;
#pragma unroll 1
    for (int it = 0; it < passes; ++it) {
        const int ih = grp + (it << lg);
        const bool used = ih < nh;
        const int h = hels[used ? ih : nh - 1];
        gg_externals<P, T>(x, h);
        cx<T> J[P::ncol];
#pragma unroll
        for (int k = 0; k < P::ncol; ++k) J[k] = mk(T(0), T(0));
        P::template amps<T>(x, J);
        __syncthreads();  // the previous pass's reads of Jt are done
#pragma unroll
        for (int k = 0; k < P::ncol; ++k) {
            Jt[(2 * k) * ME_BLOCK + lane] = J[k].r;
            Jt[(2 * k + 1) * ME_BLOCK + lane] = J[k].i;
        }
        __syncthreads();
        T q = T(0);
#pragma unroll
        for (int eb = 0; eb < 4; ++eb) {
            const double p = colour_mfma_group_sum(colour_mfma16<P::ncol>(Jt, 16 * eb, frag, lane));
            if (eb == (lane >> 4)) q = p;  // this lane's own column
        }
        if (qhel && valid && used) qhel[ev * P::nhel + h] = double(q) / P::lcd;
        acc += used ? q : T(0);
    }
    const double tot = group_sum(double(acc), lg);
    if (valid && grp == 0) out[ev] = tot * (1.0 / (256.0 * P::identical * P::lcd));
}

// Multi-channel form: the program of P (the unmerged plan: one amplitude per
// Feynman diagram) also sums, over the helicities, |A_d|^2 over the channel
// diagrams d (those with three-point vertices only) and |A_c|^2 for the
// event's channel c = chan[ev]; alpha[ev] = sum_h |A_c|^2 / sum_h sum_d |A_d|^2
// is the single-diagram-enhancement weight of the paper's multi-channel
// integration (Sec. 2: events of different channels in one kernel), 0 for a
// channel id outside 0 .. P::nchan - 1.  out[ev] is |M|^2 as from k_me_gg.
// The channel only selects which |A_d|^2 enters the numerator (a select, no
// branch), so events of different channels share a wave at no cost.
template <class P>
__global__ __launch_bounds__(ME_BLOCK) void k_me_gg_mc(const double* __restrict__ mom, int64_t nevt,
                                                       double* __restrict__ out, const int* __restrict__ hels,
                                                       int nh, me_params prm, const int* __restrict__ chan,
                                                       double* __restrict__ alpha) {
    const int64_t ev = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ev >= nevt) return;
    using T = double;
    constexpr int NG = P::ngluon;
    static_assert(ME_BLOCK == 64, "one wave per block");
    __shared__ double Qt[ME_MOM_ROW(NG + 2)];
    gg_ext<T, NG> x;
    gg_setup<P, T>(x, mom, ev, Qt, threadIdx.x, prm);
    const int ch = chan[ev];
    T acc = T(0), num = T(0), den = T(0);
#pragma unroll 1
    for (int ih = 0; ih < nh; ++ih) {
        gg_externals<P, T>(x, hels[ih]);
        cx<T> J[P::ncol];
#pragma unroll
        for (int k = 0; k < P::ncol; ++k) J[k] = mk(T(0), T(0));
        P::template amps<T>(x, J, ch, num, den);
        acc += P::template colour_sum<T>(J);
    }
    out[ev] = double(acc) * (1.0 / (256.0 * P::identical * P::lcd));
    alpha[ev] = num / den;
}

template <class P>
__global__ __launch_bounds__(ME_BLOCK) void k_me_ee(const double* __restrict__ mom, int64_t nevt,
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
    mom4<T> p[P::npart];
    load_event<T, P::npart>(mom, ev, p);
    T acc = T(0);
    for (int ih = grp; ih < nh; ih += 1 << lg) {
        const int h = hels[ih];
        const T q = P::template me_hel<T>(p, h, prm);
        if (qhel) qhel[ev * P::nhel + h] = double(q);
        acc += q;
    }
    const double tot = group_sum(double(acc), lg);
    if (grp == 0) out[ev] = tot * 0.25;
}
