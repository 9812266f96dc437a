"""Emitter for a massless quark line with gluons and one photon/Z insertion.

The process family q-line + n gluons + (photon/Z -> lepton pair), among them
g ubar -> tau+ tau- g g ubar (the DY+3j subprocess of the paper's Sec. 3).
Diagrams are the block sequences of the gluon program (gluon trees along the
fermion line) with the colourless insertion placed at every point (Plan with
ew=True); the insertion is gamma^mu (EL_mu P_L + ER_mu P_R) with the boson
propagators, couplings and the lepton current folded into the vectors EL, ER
(built per helicity by the kernel's externals).  The colour basis is that of
the quark line with n gluons.

Momentum slots in LDS: gluons 0..n-1 (flowing into the diagram), then the
fermion-flow momentum leaving the row end ("p3"), the one leaving the column
end ("p4", so that p3 + p4 is the sum of all inflowing momenta, insertion
included), the insertion's inflowing momentum qE, and the two lepton momenta.
"""
from __future__ import annotations

import math

from .colour import colour_matrix_exact, orderings
from .emit import FLOPS, GGEmitter
from .plan import Plan


class QEWEmitter(GGEmitter):
    def __init__(self, name: str, spec: dict, merge: bool = True, cap: int = 12, opaque: str = "all"):
        self.name = name
        self.spec = spec
        self.cap = cap
        self.opaque = opaque
        self.cap_f32 = cap
        self.n = spec["n"]
        self.plan = Plan(self.n, merge, ew=True)
        self.perms = orderings(self.n)
        self.kindex = {p: i for i, p in enumerate(self.perms)}
        self.num, self.lcd = colour_matrix_exact(self.n)
        self.lines = []
        self.flops = 0
        self.gin = [inc for _, inc in spec["gluons"]]

    # -- momenta ----------------------------------------------------------------
    def qexpr(self, leaves):
        terms = [f"q{a}" for a in sorted(x for x in leaves if x != "E")]
        if "E" in leaves:
            terms.append("qE")
        self.flops += FLOPS["mom_add"] * (len(terms) - 1)
        return terms[0] if len(terms) == 1 else "(" + " + ".join(terms) + ")"

    def _universe(self):
        return set(range(self.n)) | {"E"}

    def _beams(self, X, end_incoming):
        return end_incoming + sum(1 for a in X if a != "E" and self.gin[a])

    def _prop_form(self, S):
        """('row', S) for p3 - Q_S or ('col', rest) for Q_rest - p4: the form
        that sums fewer beam momenta."""
        rest = self._universe() - set(S)
        row_in = 1 if self.spec["row"][1] == 1 else 0
        col_in = 1 if self.spec["col"][1] == 1 else 0
        if not S:
            return "row", set()
        if not rest:
            return "col", set()
        if self._beams(S, row_in) <= self._beams(rest, col_in):
            return "row", set(S)
        return "col", rest

    def prop_momentum(self, S):
        form, X = self._prop_form(S)
        if form == "row":
            return f"p3 - {self.qexpr(X)}" if X else "p3"
        return f"{self.qexpr(X)} - p4" if X else "-p4"

    def _node_set(self, key):
        S = set()
        for b in key:
            S |= set(self.leaves_of(b))
        return S

    def node_momenta(self, node):
        kind = node[0]
        names = set()

        def add(S):
            names.update(f"q{a}" for a in S if a != "E")
            if "E" in S:
                names.add("qE")

        if kind == "c":
            c = self.plan.currents[node[1]]
            add(c.leaves)
            for coef, k, kids, ch in c.terms:
                if k == "v3":
                    for cid in kids:
                        add(self.leaves_of(cid))
        elif kind in ("L", "R"):
            S = self._node_set(node[1])
            if kind == "R":
                S = self._universe() - S
            form, X = self._prop_form(S)
            add(X)
            names.add("p3" if form == "row" else "p4")
        order = [f"q{a}" for a in range(self.n)] + ["p3", "p4", "qE"]
        return [x for x in order if x in names]

    def emit_momenta(self, used):
        slot = {f"q{a}": a for a in range(self.n)}
        slot.update(p3=self.n, p4=self.n + 1, qE=self.n + 2)
        self.w(" ".join(f"{nm} = mom_ld(x, {slot[nm]});" for nm in used))

    # -- nodes --------------------------------------------------------------------
    def _is_ew(self, cid):
        return cid == self.plan.ew

    def emit_node(self, node):
        kind = node[0]
        if kind == "c":
            return super().emit_node(node)
        if kind == "a":
            used = self.node_momenta(node)
            if used:
                self.emit_momenta(used)
            return self.emit_amp(node[1])
        used = self.node_momenta(node)
        if used:
            self.emit_momenta(used)
        key = node[1]
        if kind == "L":
            blk = key[-1]
            src = self.osym(("L", key[:-1]))
            S = self._node_set(key)
        else:
            blk = key[0]
            src = self.osym(("R", key[1:]))
            S = self._universe() - self._node_set(key)
        nm = self.new_name(node)
        self.w(f"spinor<T> {nm};")
        self.w("{")
        self.w(f"    const mom4<double> P = {self.prop_momentum(S)};")
        if self._is_ew(blk):
            # L' = L (gamma.EL PL + gamma.ER PR) i Pslash / P^2
            self.w("    const cx<T> f = to_t<T>(crecip(msq(P), 0.0));  // 1/P^2")
            if kind == "L":
                self.w(f"    {nm} = scale(times_i(f), row_prop(row_ew({src}, x.EL, x.ER), to_t<T>(P), T(0)));")
                self.flops += FLOPS["row_slash"] + FLOPS["row_prop"]
            else:
                self.w(f"    {nm} = scale(times_i(f), prop_col(to_t<T>(P), T(0), ew_col(x.EL, x.ER, {src})));")
                self.flops += FLOPS["slash_col"] + FLOPS["prop_col"]
        else:
            # L' = L (i g gamma.W) i Pslash / P^2
            self.w("    const cx<T> f = to_t<T>(x.g * crecip(msq(P), 0.0));  // g/P^2")
            if kind == "L":
                self.w(f"    {nm} = scale(-f, row_prop(row_slash({src}, {self.cur(blk)}), to_t<T>(P), T(0)));")
                self.flops += FLOPS["row_slash"] + FLOPS["row_prop"]
            else:
                self.w(f"    {nm} = scale(-f, prop_col(to_t<T>(P), T(0), slash_col({self.cur(blk)}, {src})));")
                self.flops += FLOPS["slash_col"] + FLOPS["prop_col"]
        self.w("}")
        self.flops += FLOPS["mom_add"] + FLOPS["msq"] + FLOPS["crecip"] + FLOPS["scale_sp"]

    def emit_amp(self, idx):
        amp = self.plan.amps[idx]
        self.w("{")
        L = self.osym(("L", amp["L"]))
        R = self.osym(("R", amp["R"]))
        if self._is_ew(amp["W"]):
            self.w(f"    const cx<T> a = row_col(row_ew({L}, x.EL, x.ER), {R});")
        else:
            self.w(f"    const cx<T> a = times_i(x.gT * row_col(row_slash({L}, {self.cur(amp['W'])}), {R}));")
        self.flops += FLOPS["row_slash"] + FLOPS["row_col"] + 2
        self.emit_jacc("a", amp["colour"])
        self.w("}")

    def sym(self, node):
        kind = node[0]
        if kind == "L" and node[1] == ():
            return "x.ubar3"
        if kind == "R" and node[1] == ():
            return "x.v4"
        return super().sym(node)

    def emit_amps(self):
        self.names = {}
        self.counter = 0
        self.w("mom4<double> " + ", ".join([f"q{a}" for a in range(self.n)] + ["p3", "p4", "qE"]) + ";")
        ops = self.schedule(self.cap)
        self.n_ops = len(ops)
        for node in ops:
            self.emit_node(node)

    # -- header -------------------------------------------------------------------
    def render(self) -> str:
        alg = self.algorithmic_flops()
        self.lines = []
        self.flops = 0
        self.emit_amps()
        body = self.lines
        executed = self.flops
        sp = self.spec
        n, nc, np_ = self.n, len(self.perms), sp["npart"]
        # externals: n polarisation vectors, 4 spinors, the lepton current and the insertion
        ext_flops = FLOPS["eps"] * n + 4 * FLOPS["spinor"] + FLOPS["fbar_gamma_f"] + 96
        st = self.plan.stats()
        gp = ", ".join(str(p) for p, _ in sp["gluons"])
        gi = ", ".join(str(i) for _, i in sp["gluons"])
        h = []
        h.append(f"// Generated by paper_2503_21935_amd.gen for {self.name}: {sp['title']}.")
        h.append(f"// {st['currents']} gluon currents ({st['current_terms']} vertex terms), "
                 f"{st['L_nodes']}+{st['R_nodes']} quark-line nodes, {st['amplitudes']} amplitudes, "
                 f"{st['colour_pairs']} colour-flow contributions per helicity; merge={self.plan.merge}.")
        h.append("#pragma once")
        h.append('#include "me_vertex.h"')
        h.append('#include "me_process.h"')
        h.append("")
        h.append(f"struct proc_{self.name} {{")
        h.append(f"    static constexpr int npart = {np_};")
        h.append(f"    static constexpr int ngluon = {n};")
        h.append(f"    static constexpr int ncol = {nc};")
        h.append(f"    static constexpr int nhel = {1 << np_};")
        h.append(f"    static constexpr int lcd = {self.lcd};")
        h.append(f"    static constexpr double avg = {sp['avg']};  // spins x colours x identical final states")
        h.append(f"    // particles: gluons {{{gp}}} (incoming {{{gi}}}); quark line from the row end")
        h.append(f"    // (particle {sp['row'][0]}, {'incoming antiquark vbar' if sp['row'][1] else 'outgoing quark ubar'})"
                 f" to the column end (particle {sp['col'][0]}, "
                 f"{'incoming quark u' if sp['col'][1] else 'outgoing antiquark v'}); leptons l- {sp['lm']}, l+ {sp['lp']}")
        h.append(f"    static constexpr int gluon_part[{max(n, 1)}] = {{{gp if n else '0'}}};")
        h.append(f"    static constexpr int gluon_in[{max(n, 1)}] = {{{gi if n else '0'}}};")
        h.append(f"    static constexpr int row_part = {sp['row'][0]}, row_in = {sp['row'][1]};")
        h.append(f"    static constexpr int col_part = {sp['col'][0]}, col_in = {sp['col'][1]};")
        h.append(f"    static constexpr int lm_part = {sp['lm']}, lp_part = {sp['lp']};")
        h.append(f"    static constexpr double q_charge = {sp['quark'][0]!r}, q_t3 = {sp['quark'][1]!r};")
        h.append(f"    static constexpr double l_charge = {sp['lepton'][0]!r}, l_t3 = {sp['lepton'][1]!r};")
        h.append(f"    static constexpr double flops_amp = {alg + ext_flops};  // per helicity, excl. colour")
        h.append(f"    static constexpr double flops_executed = {executed + ext_flops};  // incl. recomputation")
        h.append(f"    static constexpr double flops_colour = {self.colour_flops()};  // per helicity")
        h.append(f"    static constexpr int n_amplitudes = {st['amplitudes']};")
        h.append(f"    static constexpr int ndiag = {self.feynman_diagrams()};")
        h.append("")
        h.append("    template <typename T, bool TRACK = false>")
        h.append(f"    static MEV void amps(qew_ext<T, {n}>& x, cx<T>* __restrict__ J, T* __restrict__ S = nullptr) {{")
        h.extend(body)
        h.append("    }")
        h.append("")
        h.append("    // J^dag N J with N = lcd * C (integer numerators, symmetric)")
        h.append("    template <typename T>")
        h.append("    static MEV T colour_sum(const cx<T>* __restrict__ J) {")
        h.extend(self.emit_colour())
        h.append("    }")
        h.append("};")
        return "\n".join(h) + "\n"

    def feynman_diagrams(self):
        """Diagrams with each four-gluon vertex counted once: block sequences of
        the unmerged plan whose four-gluon vertices are in their first channel."""
        p = Plan(self.n, False, ew=True)

        def first(cid):
            c = p.currents[cid]
            if c.is_leaf:
                return True
            (coef, kind, kids, ch), = c.terms
            return (kind == "v3" or ch == 0) and all(first(k) for k in kids)

        cnt = 0
        for a in p.amps:
            blocks = list(a["L"]) + [a["W"]] + list(a["R"])
            cnt += all(first(b) for b in blocks)
        return cnt
