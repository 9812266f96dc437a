// me_lds.h -- access to a tile's colour-flow amplitudes held in LDS.
//
// The tile holds J for 64 events as [flow k][re, im][lane]: J_k of one lane
// at Jl[2k*64] and Jl[(2k+1)*64] with Jl pointing at the lane's column, so a
// wave touches 64 consecutive elements per access (no bank conflicts).
#pragma once
#include "me_process.h"

// J_k += v (atomic: several waves add into the same J_k).  On MI355X the
// float64 form (ds_add_f64) is fast; the float32 one (ds_add_f32) was
// measured about 20 times slower per wave instruction.
template <typename T>
MEV void lds_acc(T* __restrict__ Jl, int k, const cx<T>& v) {
    atomicAdd(Jl + (2 * k) * 64, v.r);
    atomicAdd(Jl + (2 * k + 1) * 64, v.i);
}

// S_k += v (magnitude sums of the float32 form, [k][lane])
template <typename T>
MEV void lds_acc_s(T* __restrict__ Sl, int k, T v) {
    atomicAdd(Sl + k * 64, v);
}

template <typename T>
MEV cx<T> lds_get(const T* __restrict__ Jl, int k) {
    return mk(Jl[(2 * k) * 64], Jl[(2 * k + 1) * 64]);
}

// Entry K of a 128-entry table held one entry per lane in two registers
// (entries 0..63 in t0, 64..127 in t1): a lane read, no memory access.
template <int K>
MEV int fmap_at(int t0, int t1) {
    if constexpr (K < 64)
        return __builtin_amdgcn_readlane(t0, K);
    else
        return __builtin_amdgcn_readlane(t1, K - 64);
}

// New values of a and b as far as the compiler can tell (no instruction is
// emitted): lane reads of them after this point cannot be merged with reads
// before it.
MEV void opaque_int(int& a, int& b) { asm volatile("" : "+v"(a), "+v"(b)); }

// External wavefunctions and constants of the workgroup program.  The
// momenta are not held here: the tile keeps them in LDS as
// [slot][component][lane] (slots: the NG gluons in incoming-flow sign, then
// p3, p4), read afresh by every node through mom_ld; qo[j] is the LDS row of
// the gluon this wave holds in slot j.
template <typename T, int NG>
struct coop_ext {
    vec4<T> eps[NG];
    spinor<T> ubar3, v4;
    double m, mw, g;
    T mT, gT;
    lds_cdouble* Q;   // this lane's column of the tile's momenta
    int qo[NG + 2];   // row offsets (in doubles) of slots 0..NG-1, p3, p4
};

// Momentum of slot j, read from LDS through an address the compiler cannot
// see through: no read is merged with another or moved out of its node.
template <typename T, int NG>
MEV mom4<double> mom_ld(const coop_ext<T, NG>& x, int j) {
    lds_cdouble* a = x.Q + x.qo[j];
    asm volatile("" : "+v"(a));
    return mom4<double>{a[0], a[64], a[128], a[192]};
}

// a ? x : y for momenta, as selects (both are computed)
MEV mom4<double> pick_mom(int a, const mom4<double>& x, const mom4<double>& y) {
    return mom4<double>{a ? x.e : y.e, a ? x.x : y.x, a ? x.y : y.y, a ? x.z : y.z};
}

// Per-process tables of the workgroup kernel: fmap(w)[k] is the flow of J
// that local flow k of the shared program becomes in wave w; bfrag() the
// packed float16 B fragments of the colour numerators for the mixed form.
template <class P>
struct coop_table;
