"""Evaluation plan for one helicity of g g -> t tbar + gluons.

The plan is a DAG of off-shell wavefunctions, each computed once per helicity
and reused by every diagram that contains it (the wavefunction reuse of the
paper's generated physics code, Sec. 2-3):

  * gluon currents W_S for gluon subsets S (a vertex acting on sub-currents,
    times the propagator -i/Q_S^2);
  * top-line partial currents: L(B1..Bj) = ubar(p3) (i g gamma.W_B1) S(P1) ...
    (row spinors) and R(Bj..Bk) = S(P) (i g gamma.W_Bj) ... v(p4) (column spinors);
  * the t tbar current V_T = (-i/(p3+p4)^2) ubar(p3) (i g gamma) v(p4) for diagrams
    whose gluons all meet in one tree;
  * one amplitude per diagram, added to the colour-flow amplitudes J_k with the
    diagram's colour coefficients.

With ``merge=False`` every Feynman diagram (every four-gluon colour channel)
has its own current chain and amplitude.  With ``merge=True`` currents whose
colour expansions agree up to a phase are summed before use (linearity), so
each colour structure is carried once; the result is the same sum of diagrams.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

from . import diagrams as D


@dataclass
class Current:
    id: int
    leaves: frozenset
    colour: dict            # ordering tuple -> coefficient (complex, unit modulus or sums)
    terms: list = field(default_factory=list)   # (coef, kind, child ids, channel)
    is_leaf: bool = False


def _mul(a, b):
    return D._mul(a, b)


def _comm(a, b):
    return D._add((1, _mul(a, b)), (-1, _mul(b, a)))


def _term_colour(kind, cols, ch):
    if kind == "v3":
        X, Y = cols
        return {k: -1j * v for k, v in _comm(X, Y).items()}
    X, Y, Z = cols
    if ch == 0:
        c = _comm(_comm(X, Y), Z)
    elif ch == 1:
        c = _comm(_comm(X, Z), Y)
    else:
        c = _comm(_comm(Y, Z), X)
    return {k: -v for k, v in c.items()}


def _normalise(col):
    first = min(col)
    c0 = col[first]
    key = tuple(sorted((k, complex(v / c0)) for k, v in col.items()))
    return c0, key, {k: v / c0 for k, v in col.items()}


def _clean(c):
    c = complex(c)
    r = round(c.real)
    i = round(c.imag)
    if abs(c.real - r) > 1e-12 or abs(c.imag - i) > 1e-12:
        raise ValueError(f"non-integer colour coefficient {c}")
    return complex(r, i)


class Plan:
    """Currents, fermion-line nodes and amplitudes for n gluons.

    With ``ew=True`` the fermion line also carries one colourless insertion
    (a photon/Z current from a lepton pair), block ``self.ew``, placed at every
    point of every block sequence; all gluons may then meet in one tree (the
    full-set currents are ordinary blocks)."""

    def __init__(self, n: int, merge: bool, ew: bool = False):
        self.n = n
        self.merge = merge
        self.ew_mode = ew
        self.currents: list[Current] = []
        self.by_set: dict[frozenset, list[int]] = {}
        self.root_groups: list[dict] = []  # full-set vertex sums, contracted with V_T
        self._build_currents()
        self.ew = None
        if ew:
            self.ew = self._new(leaves=frozenset(["E"]), colour={(): 1}, is_leaf=True).id
        self.L: dict[tuple, int] = {(): 0}   # block-id tuple -> node id (0 = ubar)
        self.R: dict[tuple, int] = {(): 0}   # (0 = v)
        self.L_order: list[tuple] = []
        self.R_order: list[tuple] = []
        self.amps: list[dict] = []
        self._build_amplitudes()

    # -- gluon currents ---------------------------------------------------
    def _new(self, **kw):
        c = Current(id=len(self.currents), **kw)
        self.currents.append(c)
        return c

    def _group(self, S, cands):
        """cands: list of (kind, child ids, ch).  Returns list of Current-like groups."""
        groups = {}
        order = []
        for kind, kids, ch in cands:
            cols = [self.currents[k].colour for k in kids]
            col = _term_colour(kind, cols, ch)
            if not col:
                continue
            if self.merge:
                c0, key, ncol = _normalise(col)
                if key not in groups:
                    groups[key] = dict(colour=ncol, terms=[])
                    order.append(key)
                groups[key]["terms"].append((_clean(c0), kind, kids, ch))
            else:
                key = (kind, kids, ch)
                groups[key] = dict(colour=col, terms=[(1, kind, kids, ch)])
                order.append(key)
        return [groups[k] for k in order]

    def _candidates(self, S):
        out = []
        for X, Y in D._two_splits(S):
            for cx in self.by_set[X]:
                for cy in self.by_set[Y]:
                    out.append(("v3", (cx, cy), 0))
        for X, Y, Z in D._three_splits(S):
            for cx in self.by_set[X]:
                for cy in self.by_set[Y]:
                    for cz in self.by_set[Z]:
                        for ch in range(3):
                            out.append(("v4", (cx, cy, cz), ch))
        return out

    def _build_currents(self):
        n = self.n
        for a in range(n):
            c = self._new(leaves=frozenset([a]), colour={(a,): 1}, is_leaf=True)
            self.by_set[frozenset([a])] = [c.id]
        for size in range(2, n + 1):
            for S in itertools.combinations(range(n), size):
                S = frozenset(S)
                groups = self._group(S, self._candidates(S))
                if size < n or self.ew_mode:
                    ids = []
                    for g in groups:
                        c = self._new(leaves=S, colour=g["colour"], terms=g["terms"])
                        ids.append(c.id)
                    self.by_set[S] = ids
                else:
                    self.root_groups.extend(groups)

    # -- fermion line and amplitudes -------------------------------------------
    def _block_sequences(self):
        for part in D._ordered_partitions(range(self.n)):
            if len(part) < 2 and not self.ew_mode:
                continue
            for combo in itertools.product(*(self.by_set[B] for B in part)):
                if self.ew_mode:
                    for pos in range(len(combo) + 1):
                        yield combo[:pos] + (self.ew,) + combo[pos:]
                else:
                    yield combo

    def _need(self, table, key):
        """Number of new nodes needed to obtain table[key] (prefix/suffix closure)."""
        cnt = 0
        for j in range(len(key), 0, -1):
            k = key[:j] if table is self.L else key[-j:]
            if k in table:
                break
            cnt += 1
        return cnt

    def _ensure_L(self, key):
        for j in range(1, len(key) + 1):
            k = key[:j]
            if k not in self.L:
                self.L[k] = len(self.L)
                self.L_order.append(k)
        return self.L[key]

    def _ensure_R(self, key):
        for j in range(1, len(key) + 1):
            k = key[-j:]
            if k not in self.R:
                self.R[k] = len(self.R)
                self.R_order.append(k)
        return self.R[key]

    def _build_amplitudes(self):
        # single-tree diagrams: full-set vertex sum contracted with V_T
        for g in self.root_groups:
            self.amps.append(dict(kind="root", terms=g["terms"], colour=g["colour"]))
        seqs = list(self._block_sequences())
        # longer chains first so that their prefixes/suffixes are shared by shorter ones
        seqs.sort(key=lambda s: (-len(s), s))
        for seq in seqs:
            k = len(seq)
            best = None
            for m in range(k):
                cost = self._need(self.L, seq[:m]) + self._need(self.R, seq[m + 1:])
                bal = abs(m - (k - 1) / 2)
                if best is None or (cost, bal) < best[0]:
                    best = ((cost, bal), m)
            m = best[1]
            li = self._ensure_L(seq[:m])
            ri = self._ensure_R(seq[m + 1:])
            col = {(): 1}
            for b in seq:
                col = _mul(col, self.currents[b].colour)
            self.amps.append(dict(kind="ffv", L=seq[:m], R=seq[m + 1:], W=seq[m], colour=col))

    # -- statistics ----------------------------------------------------------
    def stats(self):
        n_cur_terms = sum(len(c.terms) for c in self.currents if not c.is_leaf)
        n_root_terms = sum(len(a["terms"]) for a in self.amps if a["kind"] == "root")
        return dict(
            currents=sum(1 for c in self.currents if not c.is_leaf),
            current_terms=n_cur_terms,
            L_nodes=len(self.L_order),
            R_nodes=len(self.R_order),
            amplitudes=len(self.amps),
            root_terms=n_root_terms,
            colour_pairs=sum(len(a["colour"]) for a in self.amps),
        )
