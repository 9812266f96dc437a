"""Exact colour algebra for the T-chain basis of g g -> t tbar + gluons.

The colour-flow amplitudes J_k multiply the basis chains
c_k = (T^{a_s1} ... T^{a_sn})_{i j} (s = the k-th ordering of the n gluons
along the top line), and the colour sum is J^dag C J with
C_kl = sum over colours of conj(c_k) c_l = Tr(T^{s_k n} .. T^{s_k 1} T^{s_l 1} .. T^{s_l n})
(Sec. 3 of the paper names this constant matrix and its quadratic form).

Each adjoint pair is removed with the Fierz identity
    T^a_ij T^a_kl = 1/2 (d_il d_kj - d_ij d_kl / N),
which turns every term into closed index loops; a term is then
(1/2)^n (-1/N)^u N^loops.  The loops are counted with union-find over the
index slots of the trace, so every entry is an exact rational.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction
from functools import reduce

NC = 3


def _trace_value(word):
    """Exact Tr(T^{w_0} ... T^{w_{L-1}}) for a word in which each label occurs twice."""
    L = len(word)
    pos = {}
    for m, a in enumerate(word):
        pos.setdefault(a, []).append(m)
    pairs = list(pos.values())
    total = Fraction(0)
    # slots: i_m = 2m, j_m = 2m + 1
    for choice in itertools.product((0, 1), repeat=len(pairs)):
        parent = list(range(2 * L))

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        def union(a, b):
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[ra] = rb

        for m in range(L):
            union(2 * m + 1, 2 * ((m + 1) % L))  # matrix product / trace: j_m = i_{m+1}
        n_u1 = 0
        for (m, mp), c in zip(pairs, choice):
            if c == 0:  # d_{i_m j_m'} d_{i_m' j_m}
                union(2 * m, 2 * mp + 1)
                union(2 * mp, 2 * m + 1)
            else:  # -1/N d_{i_m j_m} d_{i_m' j_m'}
                n_u1 += 1
                union(2 * m, 2 * m + 1)
                union(2 * mp, 2 * mp + 1)
        loops = len({find(x) for x in range(2 * L)})
        total += Fraction(1, 2 ** len(pairs)) * Fraction(-1, NC) ** n_u1 * Fraction(NC) ** loops
    return total


def orderings(n: int):
    """Basis order: lexicographic permutations of gluon labels 0..n-1."""
    return list(itertools.permutations(range(n)))


def colour_matrix_exact(n: int):
    """Return (numerators, lcd) with C = numerators / lcd, numerators integer [ncol][ncol]."""
    perms = orderings(n)
    index = {p: i for i, p in enumerate(perms)}
    ident = perms[0]
    # C_kl depends only on the relative ordering s_k^-1 s_l; evaluate each once.
    rel_value = {}
    for rel in perms:
        word = tuple(reversed(ident)) + tuple(rel)
        rel_value[rel] = _trace_value(word)
    ncol = len(perms)
    C = [[None] * ncol for _ in range(ncol)]
    for k, sk in enumerate(perms):
        inv = [0] * n
        for pos_, a in enumerate(sk):
            inv[a] = pos_
        for l, sl in enumerate(perms):
            rel = tuple(inv[a] for a in sl)
            C[k][l] = rel_value[rel]
    lcd = reduce(lambda a, b: a * b // math.gcd(a, b), (c.denominator for row in C for c in row), 1)
    num = [[int(c * lcd) for c in row] for row in C]
    return num, lcd


def mfma_fragments(num):
    """First-operand fragments of v_mfma_f64_16x16x4f64 for the blocked
    symmetric colour GEMM: flows in blocks of 16 (padded with zeros), block
    pairs I <= J numbered J (J + 1) / 2 + I, four K steps of 4 flows each.
    Entry [(pair * 4 + ks) * 64 + l] = w_IJ N[16 J + l % 16][16 I + 4 ks + l // 16]
    with w_II = 1, w_IJ = 2 (I < J), 0 outside N."""
    nc = len(num)
    nb = (nc + 15) // 16
    out = []
    for jb in range(nb):
        for ib in range(jb + 1):
            w = 1 if ib == jb else 2
            for ks in range(4):
                for l in range(64):
                    j, k = 16 * jb + l % 16, 16 * ib + 4 * ks + l // 16
                    out.append(w * num[j][k] if (j < nc and k < nc) else 0)
    return out
