"""Tree-level Feynman diagrams of g g -> t tbar + gluons and their colour factors.

A diagram is an ordered list of gluon subtrees ("blocks") attached along the
top line, from the outgoing top (row spinor ubar(p3)) to the outgoing antitop
(column spinor v(p4)).  A subtree is a gluon leaf, a three-gluon vertex joining
two subtrees, or a four-gluon vertex joining three subtrees in one of its three
colour channels.  Counting each four-gluon vertex once gives 3, 16, 123, 1240
diagrams for 2, 3, 4, 5 gluons (the counts the paper's processes have).

Feynman rules (all gluon momenta counted as flowing into the vertex):
  quark-gluon vertex   i g gamma^mu T^a
  three-gluon vertex   g f^{abc} V^{mu nu rho}(k_a, k_b, k_c),
                       V = g^{mu nu}(k_a-k_b)^rho + g^{nu rho}(k_b-k_c)^mu + g^{rho mu}(k_c-k_a)^nu
  four-gluon vertex    -i g^2 [ f^{abe}f^{cde}(g^{mu rho}g^{nu sig} - g^{mu sig}g^{nu rho})
                              + f^{ace}f^{bde}(g^{mu nu}g^{rho sig} - g^{mu sig}g^{nu rho})
                              + f^{ade}f^{bce}(g^{mu nu}g^{rho sig} - g^{mu rho}g^{nu sig}) ]
  gluon propagator     -i g_{mu nu} / k^2
  top propagator       i (pslash + m) / (p^2 - m^2 + i m Gamma)

Colour: with f^{xyr} T^r = -i [T^x, T^y] every subtree rooted at gluon r becomes
a nested commutator of its leaves, so each diagram's colour factor is a sum of
basis chains (T^{a_s1} ... T^{a_sn})_{ij} with coefficients in {+-1, +-i}.
The diagram amplitude A_d (product of the Lorentz parts) then feeds the
colour-flow amplitudes J_k += c_{d,k} A_d.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

# --------------------------------------------------------------------------
# Subtrees
# --------------------------------------------------------------------------
# ('g', a) | ('v3', X, Y) | ('v4', X, Y, Z, ch); children sorted by smallest leaf.


@lru_cache(maxsize=None)
def leaves(t) -> frozenset:
    if t[0] == "g":
        return frozenset([t[1]])
    kids = t[1:3] if t[0] == "v3" else t[1:4]
    out = frozenset()
    for k in kids:
        out |= leaves(k)
    return out


def _minleaf(t):
    return min(leaves(t))


def _two_splits(S):
    S = sorted(S)
    first, rest = S[0], S[1:]
    for r in range(0, len(rest)):
        for comb in itertools.combinations(rest, r):
            X = frozenset((first,) + comb)
            Y = frozenset(S) - X
            if Y:
                yield X, Y


def _three_splits(S):
    for X, R in _two_splits(S):
        if len(R) < 2:
            continue
        for Y, Z in _two_splits(R):
            yield X, Y, Z


@lru_cache(maxsize=None)
def trees(S: frozenset):
    """All subtrees whose leaves are S (four-gluon vertices once per colour channel)."""
    if len(S) == 1:
        return (("g", next(iter(S))),)
    out = []
    for X, Y in _two_splits(S):
        for tx in trees(X):
            for ty in trees(Y):
                out.append(("v3", tx, ty))
    for X, Y, Z in _three_splits(S):
        for tx in trees(X):
            for ty in trees(Y):
                for tz in trees(Z):
                    for ch in range(3):
                        out.append(("v4", tx, ty, tz, ch))
    return tuple(out)


def n_vertex4(t) -> int:
    if t[0] == "g":
        return 0
    kids = t[1:3] if t[0] == "v3" else t[1:4]
    return (1 if t[0] == "v4" else 0) + sum(n_vertex4(k) for k in kids)


# --------------------------------------------------------------------------
# Colour expansion
# --------------------------------------------------------------------------

def _mul(a, b):
    out = {}
    for ka, ca in a.items():
        for kb, cb in b.items():
            k = ka + kb
            out[k] = out.get(k, 0) + ca * cb
    return {k: v for k, v in out.items() if v != 0}


def _add(*terms):
    out = {}
    for sign, d in terms:
        for k, v in d.items():
            out[k] = out.get(k, 0) + sign * v
    return {k: v for k, v in out.items() if v != 0}


@lru_cache(maxsize=None)
def _colour_cached(t):
    return tuple(sorted(colour(t).items()))


def colour(t) -> dict:
    """Expansion of the subtree's colour (contracted with T^root) into ordered chains."""
    if t[0] == "g":
        return {(t[1],): 1}
    if t[0] == "v3":
        X, Y = dict(_colour_cached(t[1])), dict(_colour_cached(t[2]))
        # f^{XYr} T^r = -i [X, Y]
        return _add((-1j, _mul(X, Y)), (1j, _mul(Y, X)))
    X, Y, Z = (dict(_colour_cached(k)) for k in t[1:4])
    ch = t[4]

    def comm(A, B):
        return _add((1, _mul(A, B)), (-1, _mul(B, A)))

    # channel 0: f^{XYe} f^{Zre} T^r = -[[X,Y],Z]
    # channel 1: f^{XZe} f^{Yre} T^r = -[[X,Z],Y]
    # channel 2: f^{Xre} f^{YZe} T^r = -[[Y,Z],X]
    if ch == 0:
        c = comm(comm(X, Y), Z)
    elif ch == 1:
        c = comm(comm(X, Z), Y)
    else:
        c = comm(comm(Y, Z), X)
    return {k: -v for k, v in c.items()}


def diagram_colour(blocks) -> dict:
    out = {(): 1}
    for b in blocks:
        out = _mul(out, dict(_colour_cached(b)))
    return out


# --------------------------------------------------------------------------
# Diagrams
# --------------------------------------------------------------------------

def _ordered_partitions(items):
    items = tuple(items)
    if not items:
        yield ()
        return
    n = len(items)
    for r in range(1, n + 1):
        for first in itertools.combinations(items, r):
            rest = tuple(x for x in items if x not in first)
            for tail in _ordered_partitions(rest):
                yield (frozenset(first),) + tail


def diagrams(n: int):
    """All diagrams as tuples of blocks (four-gluon vertices expanded per channel)."""
    out = []
    for part in _ordered_partitions(range(n)):
        for combo in itertools.product(*(trees(B) for B in part)):
            out.append(tuple(combo))
    return out


def count_feynman_diagrams(n: int) -> int:
    """Number of Feynman diagrams, each four-gluon vertex counted once."""
    return sum(1 for d in diagrams(n) if all(_first_channel(b) for b in d))


def _first_channel(t) -> bool:
    if t[0] == "g":
        return True
    if t[0] == "v3":
        return _first_channel(t[1]) and _first_channel(t[2])
    return t[4] == 0 and all(_first_channel(k) for k in t[1:4])
