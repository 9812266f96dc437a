"""Emit HIP source for one process from its evaluation plan.

Output: a header with one struct per process holding
  * compile-time sizes (particles, gluons, colour flows, helicities);
  * ``amps<T>(ext, J)``: one helicity's straight-line program (currents,
    top-line nodes, amplitudes, colour-flow accumulation into J);
  * ``colour_sum<T>(J)``: J^dag N J with the integer numerators N of the
    colour matrix (the caller divides by the common denominator);
  * the static algorithmic flop count of one helicity (FMA = 2 flops,
    division and square root = 1), used for roofline accounting.
"""
from __future__ import annotations

import math

from .colour import colour_matrix_exact, mfma_fragments, orderings
from .diagrams import count_feynman_diagrams
from .plan import Plan

# Floating-point operations of each primitive in me_vertex.h (FMA counted as 2).
FLOPS = dict(
    dot_cc=30, dot_rc=14, vvv=150, vvvv=116, row_slash=64, slash_col=64, row_prop=58, prop_col=58,
    scale_sp=24, row_col=30, fbar_gamma_f=72, vscale_c=24, vscale_r=8, vadd=8, jacc=2,
    mom_add=4, msq=7, recip=1, crecip=6, eps=24, spinor=40,
)


def _coef_ops(c):
    c = complex(c)
    if abs(abs(c) - 1) > 1e-12 or (c.real != 0 and c.imag != 0):
        raise ValueError(f"unexpected colour coefficient {c}")
    if c == 1:
        return "add"
    if c == -1:
        return "sub"
    if c == 1j:
        return "add_i"
    return "sub_i"


def emit_mfma_table(name, num):
    """The N fragments of the float64 matrix-core colour sum (colour.mfma_fragments)."""
    frag = mfma_fragments(num)
    out = [f"// float64 MFMA colour fragments, [block pair][K step][lane], weights 1 (diagonal) / 2 folded in",
           f"__device__ static const double colour_mfma_{name}[{len(frag)}] = {{"]
    for i in range(0, len(frag), 16):
        out.append("    " + ", ".join(f"{v}.0" for v in frag[i:i + 16]) + ",")
    out.append("};")
    return out


class GGEmitter:
    """g g -> t tbar + (n-2) gluons."""

    def __init__(self, name: str, n: int, merge: bool = True, cap: int = 8, cap_f32: int = None,
                 opaque: str = "all"):
        self.name = name
        self.cap = cap
        self.opaque = opaque
        self.cap_f32 = cap_f32 if cap_f32 is not None else cap
        self.n = n
        self.plan = Plan(n, merge)
        self.perms = orderings(n)
        self.kindex = {p: i for i, p in enumerate(self.perms)}
        self.num, self.lcd = colour_matrix_exact(n)
        self.lines = []
        self.flops = 0

    def w(self, s=""):
        self.lines.append("    " + s)

    # gluon current symbols
    def cur(self, cid):
        c = self.plan.currents[cid]
        if c.is_leaf:
            return f"x.eps[{next(iter(c.leaves))}]"
        return f"w{cid}"

    # ------------------------------------------------------------------
    # momenta
    # ------------------------------------------------------------------
    def qexpr(self, leaves):
        """Incoming-flow momentum of a gluon subset, as an expression."""
        terms = [f"q{a}" for a in sorted(leaves)]
        self.flops += FLOPS["mom_add"] * (len(terms) - 1)
        return terms[0] if len(terms) == 1 else "(" + " + ".join(terms) + ")"

    def prop_momentum(self, S):
        """Momentum of the top line after the gluons S (counted from the top end):
        p3 - Q_S, or equivalently Q_rest - p4.  The form that sums fewer of the
        two beam momenta (|p| = sqrt(s)/2) is used, which rounds less."""
        rest = set(range(self.n)) - set(S)
        nin = lambda X: sum(1 for a in X if a < 2)
        if S and (not rest or nin(S) <= nin(rest)):
            return f"p3 - {self.qexpr(S)}"
        if not S:
            return "p3"
        return f"{self.qexpr(rest)} - p4"

    def leaves_of(self, cid):
        return self.plan.currents[cid].leaves

    # ------------------------------------------------------------------
    # node symbols: every (re)computation of a node gets its own name
    # ------------------------------------------------------------------
    def sym(self, node):
        kind = node[0]
        if kind == "c":
            c = self.plan.currents[node[1]]
            if c.is_leaf:
                return f"x.eps[{next(iter(c.leaves))}]"
        if kind == "L" and node[1] == ():
            return "x.ubar3"
        if kind == "R" and node[1] == ():
            return "x.v4"
        return self.names[node]

    # Operands pass through an opaque copy (opq) so that LLVM cannot merge
    # subexpressions of one wavefunction across its uses and keep them alive
    # in between.  opaque = "all": every wavefunction operand; "eps": only the
    # external gluon polarisations, whose products are the ones worth keeping
    # apart (the other operands' copies cost a 64-bit move each and, measured,
    # more than the merging they prevent).
    def _opq(self, s):
        if self.opaque == "all" or (self.opaque == "eps" and s.startswith("x.eps[")):
            return "opq(" + s + ")"
        return s

    def cur(self, cid):
        return self._opq(self.sym(("c", cid)))

    def osym(self, node):
        return self._opq(self.sym(node))

    def deps(self, node):
        kind = node[0]
        if kind == "c":
            c = self.plan.currents[node[1]]
            out = []
            for t in c.terms:
                for k in t[2]:
                    if not self.plan.currents[k].is_leaf:
                        out.append(("c", k))
            return list(dict.fromkeys(out))
        if kind == "L":
            key = node[1]
            out = []
            if len(key) > 1:
                out.append(("L", key[:-1]))
            if not self.plan.currents[key[-1]].is_leaf:
                out.append(("c", key[-1]))
            return out
        if kind == "R":
            key = node[1]
            out = []
            if len(key) > 1:
                out.append(("R", key[1:]))
            if not self.plan.currents[key[0]].is_leaf:
                out.append(("c", key[0]))
            return out
        if kind == "vt":
            return []
        amp = self.plan.amps[node[1]]
        if amp["kind"] == "root":
            out = [("vt",)]
            for t in amp["terms"]:
                for k in t[2]:
                    if not self.plan.currents[k].is_leaf:
                        out.append(("c", k))
            return list(dict.fromkeys(out))
        out = []
        if amp["L"]:
            out.append(("L", amp["L"]))
        if not self.plan.currents[amp["W"]].is_leaf:
            out.append(("c", amp["W"]))
        if amp["R"]:
            out.append(("R", amp["R"]))
        return out

    def closure(self, node, acc=None):
        if acc is None:
            acc = set()
        for d in self.deps(node):
            if d not in acc:
                acc.add(d)
                self.closure(d, acc)
        return acc

    def amp_order(self, amps, clos, cap):
        """Greedy: next the amplitude that needs the fewest wavefunctions not
        computed before (ties: plan order)."""
        done = set()
        order = []
        remaining = list(amps)
        while remaining:
            best = min(remaining, key=lambda a: (len(clos[a] - done), a[1]))
            order.append(best)
            done |= clos[best]
            remaining.remove(best)
        return order

    def schedule(self, cap):
        """Order the amplitudes so that consecutive ones share wavefunctions, then
        walk them keeping at most ``cap`` wavefunctions alive: a node with no
        further use is dropped; if room is needed, the live node whose next use
        is furthest away is dropped and recomputed when needed again."""
        amps = [("a", i) for i in range(len(self.plan.amps))]
        clos = {a: self.closure(a) for a in amps}
        # phase 1: amplitude order (no eviction)
        order = self.amp_order(amps, clos, cap)
        # phase 2: simulate with a live-set cap
        uses = {}
        for t, a in enumerate(order):
            for d in clos[a]:
                uses.setdefault(d, []).append(t)
        live = set()
        ops = []
        self.peak_live = 0

        def next_use(node, t):
            for u in uses.get(node, []):
                if u >= t:
                    return u
            return 1 << 30

        def materialise(node, t, protect):
            if node in live:
                return
            for d in self.deps(node):
                materialise(d, t, protect)
            while len(live) >= cap:
                cands = [v for v in live if v not in protect]
                if not cands:
                    break
                # ties broken by the node itself, so that the emitted program does
                # not depend on set iteration order (string hashing per process)
                victim = max(cands, key=lambda v: (next_use(v, t), repr(v)))
                live.discard(victim)
            ops.append(node)
            live.add(node)
            self.peak_live = max(self.peak_live, len(live))

        for t, a in enumerate(order):
            protect = clos[a]
            for d in self.deps(a):
                materialise(d, t, protect)
            ops.append(a)
            for v in list(live):
                if next_use(v, t + 1) >= (1 << 30):
                    live.discard(v)
        return ops

    # ------------------------------------------------------------------
    # emission of one node
    # ------------------------------------------------------------------
    def node_momenta(self, node):
        """Names of the momenta a node's code reads."""
        kind = node[0]
        names = set()

        def add(S):
            names.update(f"q{a}" for a in S)

        def add_terms(terms):
            for coef, k, kids, ch in terms:
                if k == "v3":
                    for c in kids:
                        add(self.leaves_of(c))

        if kind == "c":
            c = self.plan.currents[node[1]]
            add(c.leaves)
            add_terms(c.terms)
        elif kind in ("L", "R"):
            key = node[1]
            S = set()
            for b in key:
                S |= set(self.leaves_of(b))
            if kind == "R":
                S = set(range(self.n)) - S
            rest = set(range(self.n)) - S
            nin = lambda X: sum(1 for a in X if a < 2)
            if S and (not rest or nin(S) <= nin(rest)):
                add(S)
                names.add("p3")
            elif not S:
                names.add("p3")
            else:
                add(rest)
                names.add("p4")
        elif kind == "vt":
            names.update(("p3", "p4"))
        else:
            amp = self.plan.amps[node[1]]
            if amp["kind"] == "root":
                add_terms(amp["terms"])
        order = [f"q{a}" for a in range(self.n)] + ["p3", "p4"]
        return [x for x in order if x in names]

    def new_name(self, node):
        self.counter += 1
        kind = node[0]
        prefix = {"c": "w", "L": "l", "R": "r", "vt": "vt"}[kind]
        nm = f"{prefix}{self.counter}"
        self.names[node] = nm
        return nm

    def vertex_sum(self, terms, indent="    "):
        """Emit s3 = sum c vvv(..), s4 = sum c vvvv(..); return the names used."""
        s3 = [t for t in terms if t[1] == "v3"]
        s4 = [t for t in terms if t[1] == "v4"]
        parts = []
        for nm, group in (("s3", s3), ("s4", s4)):
            if not group:
                continue
            parts.append(nm)
            first = True
            for coef, kind, kids, ch in group:
                if kind == "v3":
                    a, b = kids
                    expr = (f"vvv({self.cur(a)}, to_t<T>({self.qexpr(self.leaves_of(a))}), "
                            f"{self.cur(b)}, to_t<T>({self.qexpr(self.leaves_of(b))}))")
                    self.flops += FLOPS["vvv"]
                else:
                    a, b, cc = kids
                    expr = f"vvvv({self.cur(a)}, {self.cur(b)}, {self.cur(cc)}, {ch})"
                    self.flops += FLOPS["vvvv"]
                op = _coef_ops(coef)
                if first:
                    pre = {"add": "", "sub": "vscale(T(-1), ", "add_i": "vscale(mk(T(0), T(1)), ",
                           "sub_i": "vscale(mk(T(0), T(-1)), "}[op]
                    post = "" if op == "add" else ")"
                    self.w(f"{indent}vec4<T> {nm} = {pre}{expr}{post};")
                    first = False
                else:
                    fn = {"add": "vadd", "sub": "vsub", "add_i": "vadd_i", "sub_i": "vsub_i"}[op]
                    self.w(f"{indent}{fn}({nm}, {expr});")
                    self.flops += FLOPS["vadd"]
        return parts

    def emit_momenta(self, used):
        """Fresh reads of the momenta a node uses from the tile in LDS (slots:
        gluons 0..n-1, then p3, p4): nothing helicity-independent stays in
        registers between nodes."""
        slot = {f"q{a}": a for a in range(self.n)}
        slot.update(p3=self.n, p4=self.n + 1)
        self.w(" ".join(f"{nm} = mom_ld(x, {slot[nm]});" for nm in used))

    def emit_node(self, node):
        kind = node[0]
        # New SSA names for the momenta this node reads: helicity-independent
        # subexpressions (subset sums, propagator denominators) are recomputed
        # where needed instead of being merged into long-lived registers.
        used = self.node_momenta(node)
        if used:
            self.emit_momenta(used)
        if kind == "c":
            c = self.plan.currents[node[1]]
            self.w(f"// gluon current over {sorted(c.leaves)} ({len(c.terms)} vertex terms)")
            self.w("vec4<T> " + self.new_name(node) + ";")
            nm = self.names[node]
            self.w("{")
            self.w(f"    const T iq2 = T(1.0 / msq({self.qexpr(c.leaves)}));")
            self.flops += FLOPS["msq"] + FLOPS["recip"]
            parts = self.vertex_sum(c.terms)
            # W = (-i g / Q^2) s3 + (-g^2 / Q^2) s4
            if "s3" in parts and "s4" in parts:
                self.w(f"    {nm} = vscale(mk(T(0), -x.gT * iq2), s3);")
                self.w(f"    vacc({nm}, mk(-x.gT * x.gT * iq2, T(0)), s4);")
                self.flops += FLOPS["vscale_c"] + 32
            elif "s3" in parts:
                self.w(f"    {nm} = vscale(mk(T(0), -x.gT * iq2), s3);")
                self.flops += FLOPS["vscale_c"]
            else:
                self.w(f"    {nm} = vscale(-x.gT * x.gT * iq2, s4);")
                self.flops += FLOPS["vscale_r"]
            self.w("}")
        elif kind == "L":
            key = node[1]
            prev, last = key[:-1], key[-1]
            S = set()
            for b in key:
                S |= self.leaves_of(b)
            src = self.osym(("L", prev))
            nm = self.new_name(node)
            # L' = L (i g gamma.W) i (P + m)/D  with P = p3 - Q_union
            self.w(f"spinor<T> {nm};")
            self.w("{")
            self.w(f"    const mom4<double> P = {self.prop_momentum(S)};")
            self.w("    const cx<T> f = to_t<T>(x.g * crecip(msq(P) - x.m * x.m, x.mw));  // g/D")
            self.w(f"    {nm} = scale(-f, row_prop(row_slash({src}, {self.cur(last)}), to_t<T>(P), x.mT));")
            self.w("}")
            self.flops += FLOPS["mom_add"] + FLOPS["msq"] + 2 + FLOPS["crecip"] + 2 + FLOPS["row_slash"] + \
                FLOPS["row_prop"] + FLOPS["scale_sp"]
        elif kind == "R":
            key = node[1]
            first, rest = key[0], key[1:]
            S = set()
            for b in key:
                S |= self.leaves_of(b)
            src = self.osym(("R", rest))
            nm = self.new_name(node)
            # R' = i (P + m)/D (i g gamma.W) R  with P = Q_union - p4
            self.w(f"spinor<T> {nm};")
            self.w("{")
            self.w(f"    const mom4<double> P = {self.prop_momentum(set(range(self.n)) - S)};")
            self.w("    const cx<T> f = to_t<T>(x.g * crecip(msq(P) - x.m * x.m, x.mw));  // g/D")
            self.w(f"    {nm} = scale(-f, prop_col(to_t<T>(P), x.mT, slash_col({self.cur(first)}, {src})));")
            self.w("}")
            self.flops += FLOPS["mom_add"] + FLOPS["msq"] + 2 + FLOPS["crecip"] + 2 + FLOPS["slash_col"] + \
                FLOPS["prop_col"] + FLOPS["scale_sp"]
        elif kind == "vt":
            nm = self.new_name(node)
            self.w("// t tbar current (g/Q_T^2) ubar gamma v, Q_T = p3 + p4")
            self.w(f"const vec4<T> {nm} = vscale(T(x.g / msq(p3 + p4)), fbar_gamma_f(opq(x.ubar3), opq(x.v4)));")
            self.flops += FLOPS["mom_add"] + FLOPS["msq"] + FLOPS["recip"] + 1 + FLOPS["fbar_gamma_f"] + \
                FLOPS["vscale_r"]
        else:
            self.emit_amp(node[1])

    def emit_jacc(self, amp_sym, colour):
        # magnitude of the contribution, for the rounding-error estimate of the
        # float32 form (|re| + |im| bounds |a| within sqrt 2)
        self.w(f"    const T mag = TRACK ? fabs({amp_sym}.r) + fabs({amp_sym}.i) : T(0);")
        for order, c in sorted(colour.items()):
            self.w(f"    if constexpr (TRACK) S[{self.kindex[order]}] += mag;")
            k = self.kindex[order]
            op = _coef_ops(c)
            if op == "add":
                self.w(f"    J[{k}] += {amp_sym};")
            elif op == "sub":
                self.w(f"    J[{k}] -= {amp_sym};")
            elif op == "add_i":
                self.w(f"    J[{k}] += times_i({amp_sym});")
            else:
                self.w(f"    J[{k}] -= times_i({amp_sym});")
            self.flops += FLOPS["jacc"]

    def emit_amp(self, idx):
        amp = self.plan.amps[idx]
        self.w("{")
        if amp["kind"] == "root":
            self.w(f"    // single-tree diagrams, colour structure {idx}")
            parts = self.vertex_sum(amp["terms"])
            vt = self.osym(("vt",))
            # A = g dot(s3, VT) + (-i g^2) dot(s4, VT); VT carries g/Q_T^2
            if "s3" in parts and "s4" in parts:
                self.w(f"    const cx<T> a = x.gT * dot(s3, {vt}) + times_mi(x.gT * x.gT * dot(s4, {vt}));")
                self.flops += 2 * FLOPS["dot_cc"] + 6
            elif "s3" in parts:
                self.w(f"    const cx<T> a = x.gT * dot(s3, {vt});")
                self.flops += FLOPS["dot_cc"] + 2
            else:
                self.w(f"    const cx<T> a = times_mi(x.gT * x.gT * dot(s4, {vt}));")
                self.flops += FLOPS["dot_cc"] + 3
        else:
            L = self.osym(("L", amp["L"]))
            R = self.osym(("R", amp["R"]))
            self.w(f"    const cx<T> a = times_i(x.gT * row_col(row_slash({L}, {self.cur(amp['W'])}), {R}));")
            self.flops += FLOPS["row_slash"] + FLOPS["row_col"] + 2
        ch = getattr(self, "channel_of", {}).get(idx)
        if ch is not None:
            # single-diagram weight: |A|^2 into the denominator, and into the
            # numerator when this is the event's channel
            self.w("    { const T w2 = a.r * a.r + a.i * a.i;")
            self.w(f"      den += w2; num += (chan == {ch}) ? w2 : T(0); }}")
        self.emit_jacc("a", amp["colour"])
        self.w("}")

    def emit_amps(self):
        self.names = {}
        self.counter = 0
        self.mom_names = [f"q{a}" for a in range(self.n)] + ["p3", "p4"]
        # momenta: read from LDS by each node that uses them
        self.w("mom4<double> " + ", ".join([f"q{a}" for a in range(self.n)] + ["p3", "p4"]) + ";")
        ops = self.schedule(self.cap)
        self.n_ops = len(ops)
        for node in ops:
            self.emit_node(node)

    def emit_colour(self):
        N = self.num
        ncol = len(N)
        out = []
        out.append("    T acc = T(0);")
        for k in range(ncol):
            terms_r = [f"T({N[k][k]}) * J[{k}].r"]
            terms_i = [f"T({N[k][k]}) * J[{k}].i"]
            zr = f"T({N[k][k]}) * J[{k}].r"
            zi = f"T({N[k][k]}) * J[{k}].i"
            for l in range(k + 1, ncol):
                if N[k][l] == 0:
                    continue
                zr = f"fma(T({2 * N[k][l]}), J[{l}].r, {zr})"
                zi = f"fma(T({2 * N[k][l]}), J[{l}].i, {zi})"
            out.append(f"    {{ const T zr = {zr};")
            out.append(f"      const T zi = {zi};")
            out.append(f"      acc = fma(J[{k}].r, zr, fma(J[{k}].i, zi, acc)); }}")
        out.append("    return acc;")
        return out

    def colour_flops(self):
        ncol = len(self.num)
        return 2 * ncol * ncol + 6 * ncol

    def algorithmic_flops(self):
        """Flops of one helicity with every wavefunction computed exactly once."""
        keep = (self.lines, self.flops, self.cap)
        self.lines, self.flops, self.cap = [], 0, 1 << 30
        self.emit_amps()
        f = self.flops
        self.lines, self.flops, self.cap = keep
        return f

    # ------------------------------------------------------------------
    # single diagrams (multi-channel weights), on the unmerged plan
    # ------------------------------------------------------------------
    def _current_desc(self, cid):
        """Tree descriptor of a current of the unmerged plan, or None if it
        contains a four-gluon vertex."""
        c = self.plan.currents[cid]
        if c.is_leaf:
            return str(next(iter(c.leaves))), min(c.leaves)
        (coef, kind, kids, ch), = c.terms
        if kind != "v3":
            return None
        parts = [self._current_desc(k) for k in kids]
        if any(p is None for p in parts):
            return None
        parts.sort(key=lambda t: t[1])
        return "(" + parts[0][0] + "," + parts[1][0] + ")", min(parts[0][1], parts[1][1])

    def channels(self):
        """Descriptors of the amplitudes that are single diagrams built from
        three-point vertices: blocks of gluon trees along the top line from
        ubar(p3) to v(p4), '|'-separated, each tree as nested '(x,y)' with the
        part holding the smaller gluon label first.  Returns {amp index: channel}
        and the descriptor list in channel order."""
        if self.plan.merge:
            raise ValueError("channels need the unmerged plan")
        found = []
        for i, amp in enumerate(self.plan.amps):
            if amp["kind"] == "root":
                (coef, kind, kids, ch), = amp["terms"]
                if kind != "v3":
                    continue
                parts = [self._current_desc(k) for k in kids]
                if any(p is None for p in parts):
                    continue
                parts.sort(key=lambda t: t[1])
                found.append((i, "(" + parts[0][0] + "," + parts[1][0] + ")"))
            else:
                blocks = list(amp["L"]) + [amp["W"]] + list(amp["R"])
                parts = [self._current_desc(b) for b in blocks]
                if any(p is None for p in parts):
                    continue
                found.append((i, "|".join(p[0] for p in parts)))
        found.sort(key=lambda t: t[1])
        return {i: k for k, (i, _) in enumerate(found)}, [d for _, d in found]

    def render_mc(self) -> str:
        """Header of the multi-channel program: the unmerged plan (one amplitude
        per Feynman diagram and four-gluon colour channel) accumulating, besides
        J, the single-diagram sums of |A|^2 over the channels (denominator) and
        for the event's channel (numerator)."""
        self.channel_of, descs = self.channels()
        alg = self.algorithmic_flops()
        self.lines = []
        self.flops = 0
        self.emit_amps()
        body = self.lines
        executed = self.flops
        ext_flops = FLOPS["eps"] * self.n + 2 * FLOPS["spinor"]
        n = self.n
        nc = len(self.perms)
        h = []
        h.append(f"// Generated by paper_2503_21935_amd.gen for {self.name}: g g -> t tbar + {n - 2} g,")
        h.append(f"// multi-channel form: {len(self.plan.amps)} single-diagram amplitudes, {len(descs)} channels.")
        h.append("#pragma once")
        h.append('#include "me_vertex.h"')
        h.append('#include "me_process.h"')
        h.append("")
        h.append(f"struct proc_{self.name}_mc {{")
        h.append(f"    static constexpr int npart = {n + 2};")
        h.append(f"    static constexpr int ngluon = {n};")
        h.append(f"    static constexpr int ncol = {nc};")
        h.append(f"    static constexpr int nhel = {1 << (n + 2)};")
        h.append(f"    static constexpr int lcd = {self.lcd};")
        h.append(f"    static constexpr int identical = {math.factorial(n - 2)};")
        h.append(f"    static constexpr int nchan = {len(descs)};")
        h.append(f"    static constexpr double flops_amp = {alg + ext_flops};  // per helicity, excl. colour")
        h.append(f"    static constexpr double flops_executed = {executed + ext_flops};")
        h.append("")
        h.append("    // One helicity: J as in the merged program, plus sum |A_d|^2 over the")
        h.append("    // channel diagrams (den) and |A_chan|^2 (num).")
        h.append("    template <typename T, bool TRACK = false>")
        h.append(f"    static MEV void amps(gg_ext<T, {n}>& x, cx<T>* __restrict__ J, int chan, T& num, T& den, "
                 "T* __restrict__ S = nullptr) {")
        h.extend(body)
        h.append("    }")
        h.append("")
        h.append("    template <typename T>")
        h.append("    static MEV T colour_sum(const cx<T>* __restrict__ J) {")
        h.extend(self.emit_colour())
        h.append("    }")
        h.append("};")
        h.append("")
        h.append(f"// channel descriptors (host side), channel order")
        h.append(f"static const char* const channel_desc_{self.name}[{len(descs)}] = {{")
        for d in descs:
            h.append(f'    "{d}",')
        h.append("};")
        return "\n".join(h) + "\n"

    def render(self) -> str:
        alg = self.algorithmic_flops()
        self.lines = []
        self.flops = 0
        self.emit_amps()
        body = self.lines
        executed_flops = self.flops
        amp_flops = alg
        # float32 program: wavefunctions take half the registers, so more of
        # them stay alive and less is recomputed
        keep_cap = self.cap
        self.cap = self.cap_f32
        self.lines = []
        self.flops = 0
        self.emit_amps()
        body_f32 = self.lines
        executed_flops_f32 = self.flops
        self.cap = keep_cap
        ext_flops = FLOPS["eps"] * self.n + 2 * FLOPS["spinor"]
        n = self.n
        nc = len(self.perms)
        st = self.plan.stats()
        h = []
        h.append(f"// Generated by paper_2503_21935_amd.gen for {self.name}: g g -> t tbar + {n - 2} g.")
        h.append(f"// {st['currents']} gluon currents ({st['current_terms']} vertex terms), "
                 f"{st['L_nodes']}+{st['R_nodes']} top-line nodes, {st['amplitudes']} amplitudes, "
                 f"{st['colour_pairs']} colour-flow contributions per helicity; merge={self.plan.merge}.")
        h.append("#pragma once")
        h.append('#include "me_vertex.h"')
        h.append('#include "me_process.h"')
        h.append("")
        h.append(f"struct proc_{self.name} {{")
        h.append(f"    static constexpr int npart = {n + 2};")
        h.append(f"    static constexpr int ngluon = {n};")
        h.append(f"    static constexpr int ncol = {nc};")
        h.append(f"    static constexpr int nhel = {1 << (n + 2)};")
        h.append(f"    static constexpr int lcd = {self.lcd};")
        h.append(f"    static constexpr int identical = {math.factorial(n - 2)};")
        h.append(f"    static constexpr double flops_amp = {amp_flops + ext_flops};  // per helicity, excl. colour")
        h.append(f"    static constexpr double flops_executed = {executed_flops + ext_flops};  // incl. recomputation")
        h.append(f"    static constexpr double flops_colour = {self.colour_flops()};  // per helicity")
        h.append(f"    static constexpr int n_amplitudes = {st['amplitudes']};")
        h.append(f"    static constexpr int ndiag = {count_feynman_diagrams(n)};")
        h.append("")
        h.append("    // TRACK: also accumulate S[k] = sum of |contribution| to J[k] (error estimate)")
        h.append("    template <typename T, bool TRACK = false>")
        h.append("    static MEV void amps(gg_ext<T, " + str(n) + ">& x, cx<T>* __restrict__ J, "
                 "T* __restrict__ S = nullptr) {")
        h.extend(body)
        h.append("    }")
        h.append("")
        h.append(f"    // the same program scheduled for float32 (live-set cap {self.cap_f32}; "
                 f"{executed_flops_f32 + ext_flops} flops executed per helicity)")
        h.append("    template <typename T, bool TRACK = false>")
        h.append("    static MEV void amps_f32(gg_ext<T, " + str(n) + ">& x, cx<T>* __restrict__ J, "
                 "T* __restrict__ S = nullptr) {")
        h.extend(body_f32)
        h.append("    }")
        h.append("")
        h.append("    // J^dag N J with N = lcd * C (integer numerators, symmetric)")
        h.append("    template <typename T>")
        h.append("    static MEV T colour_sum(const cx<T>* __restrict__ J) {")
        h.extend(self.emit_colour())
        h.append("    }")
        h.append("")
        import numpy as np

        N = np.array(self.num, dtype=float)
        ev = np.linalg.eigvalsh(N)
        abs_lmax = float(np.linalg.eigvalsh(np.abs(N)).max())
        # a-priori relative error of J^dag N J when J is carried as float16 hi + lo
        # (2^-22 per element) and the products accumulate in float32:
        #   2 * 2^-22 * cond(N) + sqrt(ncol) * 2^-24 * lambda_max(|N|) / lambda_min(N)
        col_err = float(2 * 2.0 ** -22 * ev.max() / ev.min() + math.sqrt(nc) * 2.0 ** -24 * abs_lmax / ev.min())
        h.append(f"    static constexpr double abs_lambda_max = {abs_lmax!r};  // largest eigenvalue of |N|")
        h.append(f"    static constexpr double lambda_min = {float(ev.min())!r};  // smallest eigenvalue of N")
        h.append(f"    static constexpr double colour_err_f16 = {col_err!r};")
        h.append("};")
        h.append("")
        h.append(f"// colour-matrix numerators for device-side lookup, row-major [{nc}][{nc}]")
        h.append(f"__device__ __constant__ static const short colour_num_{self.name}[{nc * nc}] = {{")
        for row in self.num:
            h.append("    " + ", ".join(str(v) for v in row) + ",")
        h.append("};")
        h.extend(emit_mfma_table(self.name, self.num))
        h.append(f"template <> struct colour_table<proc_{self.name}> {{")
        h.append(f"    static MEV int get(int k, int l) {{ return colour_num_{self.name}[k * {nc} + l]; }}")
        h.append(f"    static MEV const double* mfma_frag() {{ return colour_mfma_{self.name}; }}")
        h.append("};")
        return "\n".join(h) + "\n"
