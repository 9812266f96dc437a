// me_colour_mfma.h -- the float64 colour sum J^dag N J of a tile of events on
// the matrix cores (v_mfma_f64_16x16x4f64).
//
// The colour-matrix quadratic form (the paper's Sec. 3: after the Feynman
// diagrams, each event and helicity needs Q = J^dag C J with the process's
// constant colour matrix) is a batched GEMM once the events of a tile are
// stacked: with A the matrix of rows (Re J_e, Im J_e) over the tile's events e,
// Q_e = sum over e's two rows of A N A^T (N = lcd * C: integer numerators,
// real symmetric).  The flows are cut into blocks of 16 (the last one padded)
// and, N being symmetric, only block pairs I <= J are formed:
//   Z^T[j][r] = sum_{I <= J} w_IJ sum_{k in I} N[j][k] A[r][k]   (j in block J)
//   Q_r      += sum_{j in J} A[r][j] Z^T[j][r]
// with w_II = 1 and w_IJ = 2 for I < J, folded into the constant N fragments.
// Each v_mfma_f64_16x16x4f64 takes 16 flows j x 4 flows k of w N (first
// operand, from a table in global memory) and 4 flows k x 16 rows r of A^T
// (second operand, read from the tile's J in LDS), accumulating Z^T for one
// block J and 16 rows; the re and im rows of the same 16 events share the N
// fragment.  The dot with A is done on the VALU from the accumulator layout.
//
// Lane layouts (gfx950, measured with an in-bounds probe): first operand lane
// l holds X[l % 16][l / 16] of a 16 x 4 block, second operand Y[l / 16][l % 16]
// of a 4 x 16 block, and accumulator register v of lane l holds
// D[4 v + l / 16][l % 16].
#pragma once
#include "me_process.h"

typedef double me_d4 __attribute__((ext_vector_type(4)));

// Flows in blocks of 16; block pairs I <= J numbered J (J + 1) / 2 + I.
template <int NCOL>
struct colour_mfma_shape {
    static_assert(NCOL % 4 == 0, "whole K steps of 4 flows");
    static constexpr int NB = (NCOL + 15) / 16;
    static constexpr int NPAIR = NB * (NB + 1) / 2;
    // N fragments per pair: 4 K steps of 64 doubles
    static constexpr int FRAG_DOUBLES = NPAIR * 4 * 64;
};

// Partial Q of the 16 events (columns) e0 .. e0 + 15 of the tile held in LDS as
// Jt[(2 k + c) 64 + e] (flow k, c = 0 re / 1 im, column e), for this lane: the
// return value summed over the four lane groups l / 16 (lanes l, l ^ 16,
// l ^ 32, l ^ 48) is Q of column e0 + l % 16, in numerator units.  frag: the
// process's N fragment table, [pair][K step][lane] doubles, w_IJ folded in.
// All 64 lanes of the wave must call it together.
template <int NCOL>
MEV double colour_mfma16(const double* __restrict__ Jt, int e0, const double* __restrict__ frag, int lane) {
    using S = colour_mfma_shape<NCOL>;
    const int r = lane & 15, g = lane >> 4;
    double acc = 0.0;
#pragma unroll
    for (int jb = 0; jb < S::NB; ++jb) {
        me_d4 zr = {0.0, 0.0, 0.0, 0.0}, zi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ib = 0; ib <= jb; ++ib) {
            const int pair = jb * (jb + 1) / 2 + ib;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                if (16 * ib + 4 * ks >= NCOL) continue;  // padded flows: nothing to add
                const int k = 16 * ib + 4 * ks + g;
                const double n = frag[(pair * 4 + ks) * 64 + lane];
                const double ar = Jt[(2 * k) * 64 + e0 + r];
                const double ai = Jt[(2 * k + 1) * 64 + e0 + r];
                zr = __builtin_amdgcn_mfma_f64_16x16x4f64(n, ar, zr, 0, 0, 0);
                zi = __builtin_amdgcn_mfma_f64_16x16x4f64(n, ai, zi, 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (16 * jb + 4 * v >= NCOL) continue;  // rows of padded flows
            const int j = 16 * jb + 4 * v + g;
            acc = fma(Jt[(2 * j) * 64 + e0 + r], zr[v], acc);
            acc = fma(Jt[(2 * j + 1) * 64 + e0 + r], zi[v], acc);
        }
    }
    return acc;
}

// Sum over the four lane groups: every lane receives Q of column e0 + lane % 16.
MEV double colour_mfma_group_sum(double v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}
