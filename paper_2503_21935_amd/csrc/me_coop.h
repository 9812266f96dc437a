// me_coop.h -- kernel for processes whose colour-flow amplitudes J are kept
// in LDS instead of registers (g g -> t tbar g g g: 120 flows, 1,920 bytes
// per event in float64).
//
// A workgroup of P::waves waves takes a tile of 64 events, one per lane; all
// waves hold the same events.  The process's program is written for one
// wave's share of the amplitudes; wave w runs it with the gluon inputs
// relabelled (slot j holds gluon P::perm(w, j)) and adds its contributions to
// the relabelled colour flows.  Per helicity: the tile's J is cleared, every
// wave builds its relabelled external wavefunctions and runs the program,
// adding into J in LDS; after a barrier each wave evaluates its share of the
// colour sum J^dag N J.  The per-lane partial sums over helicities are added
// across the waves at the end.  The result is the same spin- and
// colour-averaged |M|^2 as the one-wave kernel computes.
#pragma once
#include "me_kernels.h"
#include "me_lds.h"

#define ME_TILE 64

// External wavefunctions of one helicity for this wave's relabelled gluon
// slots (slot j holds gluon P::perm(wave, j)), from the tile's momenta in LDS.
template <class P, typename T>
MEV void coop_externals(coop_ext<T, P::ngluon>& x, int h, int wave) {
    constexpr int NP = P::npart, NG = P::ngluon;
#pragma unroll
    for (int j = 0; j < NG; ++j) {
        const int g = P::perm(wave, j);  // wave-uniform
        const int ip = (g < 2) ? g : g + 2;
        const double sg = (g < 2) ? 1.0 : -1.0;  // physical momentum from the incoming-flow q
        const mom4<double> q = mom_ld(x, j);
        const mom4<double> k{sg * q.e, sg * q.x, sg * q.y, sg * q.z};
        const vec4<double> e = gluon_eps(k, helicity_of<NP>(h, ip), g >= 2);
#pragma unroll
        for (int c = 0; c < 4; ++c) x.eps[j].v[c] = to_t<T>(e.v[c]);
    }
    const spinor<double> u = bar(u_spinor(mom_ld(x, NG), x.m, helicity_of<NP>(h, 2)));
    const spinor<double> v = v_spinor(mom_ld(x, NG + 1), x.m, helicity_of<NP>(h, 3));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        x.ubar3.s[c] = to_t<T>(u.s[c]);
        x.v4.s[c] = to_t<T>(v.s[c]);
    }
}

template <class P, int W>
MEV double coop_colour(int wave, const double* Jl) {
    if constexpr (W < P::waves) {
        if (wave == W) return P::template colour_part<W, double>(Jl);
        return coop_colour<P, W + 1>(wave, Jl);
    }
    return 0.0;
}

// Arguments as for k_me_gg; launched with blocks of 64 * P::waves threads,
// one block per 64 / 2^lg events (or entries of idx).  With lg > 0 the 2^lg
// lanes of an event take every 2^lg-th helicity of the list (the same count
// of passes for every lane, so the barriers stay uniform; a lane past the end
// of the list repeats its last helicity and discards the result).
// CM: colour sum on the matrix cores (colour_mfma16: wave w takes the tile's
// columns 16 w .. 16 w + 15 over all flows) instead of the VALU split by
// blocks of the symmetric matrix (colour_part).
template <class P, bool CM = false>
__global__ __launch_bounds__(ME_TILE * P::waves, 1) void k_me_gg_coop(
    const double* __restrict__ mom, int64_t nevt, double* __restrict__ out, const int* __restrict__ hels, int nh,
    me_params prm, double* __restrict__ qhel, const int* __restrict__ idx, const int* __restrict__ count, int lg) {
    constexpr int NP = P::npart, NG = P::ngluon;
    __shared__ double Jt[P::ncol * 2 * ME_TILE];
    __shared__ double Qt[(NG + 2) * 4 * ME_TILE];
    __shared__ double part[P::waves * ME_TILE];
    const int lane = threadIdx.x % ME_TILE;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / ME_TILE);
    const int grp = lane & ((1 << lg) - 1);
    const int64_t n = count ? (int64_t)*count : nevt;
    const int64_t first = (int64_t)blockIdx.x * (ME_TILE >> lg);
    if (first >= n) return;  // whole block: no barrier is left waiting
    int64_t i = first + (lane >> lg);
    const bool valid = i < n;
    if (!valid) i = n - 1;  // idle lanes repeat an event so that every wave runs the full program
    const int64_t ev = count ? (int64_t)idx[i] : i;
    if (wave == 0) {  // the tile's momenta: gluons in incoming-flow sign, then p3, p4
        const double2* pe = reinterpret_cast<const double2*>(mom + ev * (NP * 4));
#pragma unroll
        for (int r = 0; r < NG + 2; ++r) {
            const int ip = (r < 2) ? r : (r < NG) ? r + 2 : r - NG + 2;
            const double sg = (r >= 2 && r < NG) ? -1.0 : 1.0;
            const double2 a = pe[2 * ip], b = pe[2 * ip + 1];
            Qt[(4 * r + 0) * ME_TILE + lane] = sg * a.x;
            Qt[(4 * r + 1) * ME_TILE + lane] = sg * a.y;
            Qt[(4 * r + 2) * ME_TILE + lane] = sg * b.x;
            Qt[(4 * r + 3) * ME_TILE + lane] = sg * b.y;
        }
    }
    __syncthreads();
    coop_ext<double, NG> x;
    x.m = prm.mt;
    x.mw = prm.mt * prm.wt;
    x.g = prm.gs;
    x.mT = prm.mt;
    x.gT = prm.gs;
    x.Q = (lds_cdouble*)(Qt + lane);
#pragma unroll
    for (int j = 0; j < NG; ++j) x.qo[j] = 4 * ME_TILE * P::perm(wave, j);
    x.qo[NG] = 4 * ME_TILE * NG;
    x.qo[NG + 1] = 4 * ME_TILE * (NG + 1);
    static_assert(P::ncol <= 2 * ME_TILE, "flow map held in two registers");
    const int* fm = coop_table<P>::fmap(wave);
    const int fm0 = fm[lane];
    const int fm1 = (lane + ME_TILE < P::ncol) ? fm[lane + ME_TILE] : 0;
    double* Jl = Jt + lane;
    int wsel = wave;
    asm volatile("" : "+v"(wsel));  // per-lane copy: selects instead of branches in the program
    double acc = 0.0;
    const int passes = (nh + (1 << lg) - 1) >> lg;
#pragma unroll 1
    for (int it = 0; it < passes; ++it) {
        const int ih_raw = grp + (it << lg);
        const bool used = ih_raw < nh;
        const int h = hels[used ? ih_raw : nh - 1];
        for (int e = threadIdx.x; e < P::ncol * 2 * ME_TILE; e += ME_TILE * P::waves) Jt[e] = 0.0;
        __syncthreads();
        coop_externals<P, double>(x, h, wave);
        P::template amps_wave<double>(x, Jl, nullptr, fm0, fm1, wsel);
        __syncthreads();
        if constexpr (CM) {
            static_assert(P::waves == 4, "one 16-column block of the tile per wave");
            // Q of column c = 16 wave + lane % 16, whose helicity pass may differ from this lane's
            const int col = 16 * wave + (lane & 15);
            const bool col_used = (col & ((1 << lg) - 1)) + (it << lg) < nh;
            const double q =
                colour_mfma_group_sum(colour_mfma16<P::ncol>(Jt, 16 * wave, colour_table<P>::mfma_frag(), lane));
            acc += col_used ? q : 0.0;
            if (qhel) {
                if (lane < 16) part[col] = q;
                __syncthreads();
                if (wave == 0 && valid && used) qhel[ev * P::nhel + h] = part[lane] / P::lcd;
            }
        } else {
            const double q = coop_colour<P, 0>(wave, Jl);
            acc += used ? q : 0.0;
            if (qhel) {  // uniform: a kernel argument
                part[threadIdx.x] = q;
                __syncthreads();
                if (wave == 0 && valid && used) {
                    double s = 0.0;
                    for (int w = 0; w < P::waves; ++w) s += part[w * ME_TILE + lane];
                    qhel[ev * P::nhel + h] = s / P::lcd;
                }
            }
        }
        __syncthreads();
    }
    if constexpr (CM) {
        if (lane < 16) part[16 * wave + lane] = acc;  // the wave's columns, complete
    } else {
        part[threadIdx.x] = acc;  // this wave's share of every column
    }
    __syncthreads();
    if (wave == 0) {  // all 64 lanes of wave 0 take part in the group sum
        double s = 0.0;
        if constexpr (CM) {
            s = part[lane];
        } else {
            for (int w = 0; w < P::waves; ++w) s += part[w * ME_TILE + lane];
        }
        s = group_sum(s, lg);
        if (valid && grp == 0) out[ev] = s * (1.0 / (256.0 * P::identical * P::lcd));
    }
}
