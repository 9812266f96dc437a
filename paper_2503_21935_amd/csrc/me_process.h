// me_process.h -- per-event external state and the e+ e- -> mu+ mu- program.
#pragma once
#include "me_vertex.h"

// Physics constants handed to every kernel by value.
struct me_params {
    double gs;              // strong coupling sqrt(4 pi alpha_s)
    double mt, wt;          // top mass and width
    double e;               // electromagnetic coupling sqrt(4 pi alpha)
    double gz, gl, gr;      // Z coupling e/(sw cw) and chiral charges of charged leptons
    double mz, wz;          // Z mass and width
    double sw2;             // sin^2 theta_W
};

// Device-side access to a process's colour-matrix numerators (specialised by
// the generated process headers).
template <class P>
struct colour_table;

// Pointer into LDS (address space 3): reads compile to ds_read.
typedef __attribute__((address_space(3))) const double lds_cdouble;

// Row offset (in doubles) of momentum slot j in a 64-lane tile of momenta
// held in LDS as [slot][component][lane].
#define ME_MOM_ROW(j) (4 * 64 * (j))

// External wavefunctions of one event at one helicity for
// g g -> t tbar + (NG-2) g, and where its momenta are.  The momenta are kept
// in LDS, slots 0..NG-1 for the gluons counted as flowing into the diagram
// (q = p for the two incoming gluons, q = -p for outgoing ones), slot NG for
// p3 and NG+1 for p4, and read afresh where a node needs them (mom_ld), so
// that no helicity-independent value occupies registers across the program.
// Momenta, propagator denominators and couplings stay in float64 for every
// amplitude type T: the near-on-shell propagators cancel p^2 against m^2,
// which float32 cannot resolve.
template <typename T, int NG>
struct gg_ext {
    vec4<T> eps[NG];
    spinor<T> ubar3, v4;
    lds_cdouble* Q;   // this lane's column of the tile's momenta
    double m, mw, g;  // top mass, mass * width, strong coupling
    T mT, gT;         // the same in the amplitude type
};

// External state of a massless quark line with gluons and a photon/Z
// insertion (the quark-line + lepton-pair processes): the row and column
// spinors sit in ubar3 and v4, and the insertion gamma^mu (EL_mu P_L + ER_mu
// P_R) carries the boson propagators, couplings and the lepton current.
template <typename T, int NG>
struct qew_ext : gg_ext<T, NG> {
    vec4<T> EL, ER;
};

// Momentum of slot j, read from LDS through an address the compiler cannot
// see through: no read is merged with another or moved out of its node.
template <typename T, int NG>
MEV mom4<double> mom_ld(const gg_ext<T, NG>& x, int j) {
    lds_cdouble* a = x.Q + ME_MOM_ROW(j);
    asm volatile("" : "+v"(a));
    return mom4<double>{a[0], a[64], a[128], a[192]};
}

// e+(p1) e-(p2) -> mu+(p3) mu-(p4) through an s-channel photon and Z:
//   M = (eQ)^2 (Je.Jm)/s + gz^2 [Je'.Jm' - (Je'.k)(Jm'.k)/MZ^2] / (s - MZ^2 + i MZ WZ),
// with Je = vbar(p1) gamma u(p2), Jm = ubar(p4) gamma v(p3), primes for the
// chiral Z couplings (gl on the left-handed part, gr on the right-handed part).
struct proc_ee_mumu {
    static constexpr int npart = 4;
    static constexpr int ncol = 1;
    static constexpr int nhel = 16;
    static constexpr int lcd = 1;
    static constexpr int identical = 1;
    // external spinors 4 x 40, two split currents 2 x 72, contraction and propagators
    static constexpr double flops_amp = 4 * 40 + 2 * 72 + 4 * 30 + 16 + 60;
    static constexpr double flops_colour = 3;
    static constexpr double flops_executed = flops_amp;  // no shared wavefunctions to recompute
    static constexpr int n_amplitudes = 2;
    static constexpr int ndiag = 2;

    template <typename T>
    static MEV T me_hel(const mom4<T>* p, int hel, const me_params& prm) {
        auto lam = [&](int i) { return ((hel >> (3 - i)) & 1) ? 1 : -1; };
        const T zero = T(0);
        spinor<T> vb1 = bar(v_spinor(p[0], zero, lam(0)));
        spinor<T> u2 = u_spinor(p[1], zero, lam(1));
        spinor<T> v3 = v_spinor(p[2], zero, lam(2));
        spinor<T> ub4 = bar(u_spinor(p[3], zero, lam(3)));
        vec4<T> eL, eR, mL, mR;
        fbar_gamma_f_lr(vb1, u2, eL, eR);
        fbar_gamma_f_lr(ub4, v3, mL, mR);
        const mom4<T> k = p[0] + p[1];
        const T s = msq(k);
        const T e = T(prm.e), gz = T(prm.gz), gl = T(prm.gl), gr = T(prm.gr), mz = T(prm.mz);
        vec4<T> je, jm, jez, jmz;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            je.v[c] = eL.v[c] + eR.v[c];
            jm.v[c] = mL.v[c] + mR.v[c];
            jez.v[c] = gl * eL.v[c] + gr * eR.v[c];
            jmz.v[c] = gl * mL.v[c] + gr * mR.v[c];
        }
        const cx<T> a_gamma = (e * e / s) * dot(je, jm);  // (eQ)^2 with Q = -1
        const cx<T> prop_z = crecip(s - mz * mz, mz * T(prm.wz));
        const cx<T> kz = dot(jez, jmz) - dot(k, jez) * dot(k, jmz) * (T(1) / (mz * mz));
        const cx<T> a = a_gamma + (gz * gz) * (prop_z * kz);
        return a.r * a.r + a.i * a.i;
    }
};
