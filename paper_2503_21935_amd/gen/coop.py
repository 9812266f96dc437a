"""Emission for processes whose colour-flow amplitudes do not fit in registers.

For g g -> t tbar g g g the 120 colour-flow amplitudes J of one event are
1,920 bytes in float64, more than a lane's register budget next to the
wavefunctions.  The kernel for such processes gives a workgroup of four
waves one 64-event tile and keeps J for the tile in LDS.

The four waves run one and the same program, on relabelled inputs.  The set
of diagrams (and of merged colour structures) is mapped onto itself by any
relabelling of the gluons, and the value of an amplitude evaluated with the
gluon inputs permuted is the value of the relabelled amplitude, with the
relabelled colour flows.  With the cyclic group Z4 acting on gluons 1..4
(gluon 0 fixed), the 945 amplitudes of one helicity fall into 243 orbits;
the program evaluates one representative per orbit, and wave w runs it on
inputs relabelled by the w-th group element, adding each contribution into
the relabelled colour flow.  Together the four waves produce every amplitude
once; an amplitude that a group element maps onto itself comes out of
several waves and is weighted by 1/(size of its stabiliser), an exact
power of two.

Per wave, contributions are gathered in a small window of registers (slots
assigned by furthest-next-use) and added into LDS with atomic float64 adds,
since all waves contribute to every J_k.  The colour sum J^dag N J is then
split between the waves by blocks of the symmetric colour matrix.
"""
from __future__ import annotations

import math
import random

from .emit import FLOPS, GGEmitter, _coef_ops
from .plan import _normalise


class _Names(dict):
    def __missing__(self, key):
        return "_"


def cyclic_group(n: int, waves: int = 4):
    """Element w maps local gluon slot j to gluon label perm[w][j]: a cyclic
    shift by w of labels 1..n-1 (label 0 fixed)."""
    m = n - 1
    if m % waves:
        raise ValueError("the cyclic group needs (gluons - 1) divisible by the number of waves")
    out = []
    for w in range(waves):
        out.append(tuple(0 if j == 0 else (j - 1 + w * (m // waves)) % m + 1 for j in range(n)))
    return out


class GGCoopEmitter(GGEmitter):
    """One program for all waves of a workgroup; wave w runs it on inputs
    relabelled by group element w and adds into the relabelled flows of J in LDS."""

    def __init__(self, name: str, n: int, merge: bool = True, cap: int = 12, window: int = 16,
                 waves: int = 4, cap_f32: int = None, opaque: str = "all"):
        super().__init__(name, n, merge, cap, cap_f32, opaque)
        self.window = window
        self.waves = waves
        self.group = cyclic_group(n, waves)
        self.coop = False
        self._costs = {}
        self.reps, self.weight = self.representatives()

    # ------------------------------------------------------------------
    # orbits of the amplitudes under the relabelling group
    # ------------------------------------------------------------------
    def _relabel_tables(self):
        plan = self.plan
        bykey = {}
        for c in plan.currents:
            _, key, _ = _normalise(c.colour)
            bykey[(c.leaves, key)] = c.id
        rootkey, seqkey = {}, {}
        for i, a in enumerate(plan.amps):
            if a["kind"] == "root":
                _, key, _ = _normalise(a["colour"])
                rootkey[key] = i
            else:
                seqkey[a["L"] + (a["W"],) + a["R"]] = i
        return bykey, rootkey, seqkey

    def relabel_amp(self, i, pi, tables):
        bykey, rootkey, seqkey = tables
        a = self.plan.amps[i]
        if a["kind"] == "root":
            col = {tuple(pi[x] for x in o): v for o, v in a["colour"].items()}
            return rootkey[_normalise(col)[1]]

        def cur(cid):
            c = self.plan.currents[cid]
            col = {tuple(pi[x] for x in o): v for o, v in c.colour.items()}
            return bykey[(frozenset(pi[x] for x in c.leaves), _normalise(col)[1])]

        return seqkey[tuple(cur(c) for c in a["L"] + (a["W"],) + a["R"])]

    def node_cost(self, node):
        if node not in self._costs:
            keep = (self.lines, self.flops, getattr(self, "names", None), getattr(self, "counter", 0))
            self.names, self.counter, self.lines, self.flops = _Names(), 0, [], 0
            self.emit_node(node)
            self._costs[node] = self.flops
            self.lines, self.flops, self.names, self.counter = keep
        return self._costs[node]

    def representatives(self, trials: int = 10):
        """One amplitude per orbit, chosen greedily (largest dependency sets
        first) to share as many wavefunctions as possible; returns the indices
        and the weights 1/|stabiliser|."""
        tables = self._relabel_tables()
        seen, orbits = set(), []
        for i in range(len(self.plan.amps)):
            if i in seen:
                continue
            orb = sorted({self.relabel_amp(i, pi, tables) for pi in self.group})
            seen |= set(orb)
            orbits.append(orb)
        if sum(len(o) for o in orbits) != len(self.plan.amps):
            raise RuntimeError("relabelling does not permute the amplitudes")
        clos = {i: self.closure(("a", i)) | {("a", i)} for i in range(len(self.plan.amps))}
        best = None
        for trial in range(trials):
            rnd = random.Random(trial)
            have, reps = set(), []
            for orb in sorted(orbits, key=lambda o: (-max(len(clos[i]) for i in o), rnd.random())):
                i = min(orb, key=lambda i: (sum(self.node_cost(d) for d in clos[i] - have), rnd.random()))
                have |= clos[i]
                reps.append((i, len(orb)))
            cost = sum(self.node_cost(d) for d in have)
            if best is None or cost < best[0]:
                best = (cost, reps)
        self.wave_flops = best[0]
        reps = sorted(best[1])
        return [i for i, _ in reps], {i: m / self.waves for i, m in reps}

    # ------------------------------------------------------------------
    # per-wave choice of the top-propagator momentum form
    # ------------------------------------------------------------------
    def _prop_mask(self, S):
        """Bit w set: wave w takes p3 - Q_S (fewer beam momenta than Q_rest - p4)."""
        rest = set(range(self.n)) - set(S)
        mask = 0
        for w, pi in enumerate(self.group):
            nin = lambda X: sum(1 for a in X if pi[a] < 2)
            if nin(S) <= nin(rest):
                mask |= 1 << w
        return mask

    def prop_momentum(self, S):
        """p3 - Q_S or Q_rest - p4, whichever sums fewer beam momenta for the
        gluon labels this wave holds in the slots S (chosen per wave at run time
        when the waves differ)."""
        if not self.coop:
            return super().prop_momentum(S)
        rest = set(range(self.n)) - set(S)
        if not S:
            return "p3"
        if not rest:
            return f"p3 - {self.qexpr(S)}"
        mask = self._prop_mask(S)
        if mask == (1 << self.waves) - 1:
            return f"p3 - {self.qexpr(S)}"
        if mask == 0:
            return f"{self.qexpr(rest)} - p4"
        return (f"pick_mom(({mask} >> wsel) & 1, p3 - {self.qexpr(S)}, {self.qexpr(rest)} - p4)")

    def node_momenta(self, node):
        if not self.coop or node[0] not in ("L", "R"):
            return super().node_momenta(node)
        S = set()
        for b in node[1]:
            S |= set(self.leaves_of(b))
        if node[0] == "R":
            S = set(range(self.n)) - S
        rest = set(range(self.n)) - S
        names = set()
        if not S:
            names.add("p3")
        elif not rest:
            names.update(f"q{a}" for a in S)
            names.add("p3")
        else:
            mask = self._prop_mask(S)
            if mask:
                names.update(f"q{a}" for a in S)
                names.add("p3")
            if mask != (1 << self.waves) - 1:
                names.update(f"q{a}" for a in rest)
                names.add("p4")
        order = [f"q{a}" for a in range(self.n)] + ["p3", "p4"]
        return [x for x in order if x in names]

    def amp_order(self, amps, clos, cap):
        """Cache-aware greedy: next the amplitude with the fewest wavefunctions
        not computed before, counting half for those computed before but no
        longer among the `cap` most recently used (they would be recomputed);
        ties: plan order.  At cap 16 this executes about 9 % fewer flops per
        wave than the plain greedy order for g g -> t tbar g g g."""
        done, recent, order = set(), [], []
        remaining = set(amps)
        while remaining:
            lv = set(recent)
            best = min(remaining, key=lambda a: (len(clos[a] - done) + 0.5 * len((clos[a] & done) - lv), a[1]))
            order.append(best)
            remaining.discard(best)
            done |= clos[best]
            for d in sorted(clos[best], key=repr):
                if d in recent:
                    recent.remove(d)
                recent.append(d)
            recent = recent[-cap:]
        return order

    # ------------------------------------------------------------------
    # register window over J
    # ------------------------------------------------------------------
    def plan_window(self, order):
        """Actions for every contribution, in emission order: ('hit', slot),
        ('fill', slot, evicted flow or None) or ('direct',)."""
        seqs = [[self.kindex[o] for o, _ in sorted(self.plan.amps[i]["colour"].items())] for i in order]
        uses = {}
        for t, fl in enumerate(seqs):
            for f in fl:
                uses.setdefault(f, []).append(t)
        ptr = {f: 0 for f in uses}
        slot_of = {}
        free = list(range(self.window))
        actions = []

        def next_use(f, t):
            u = uses[f]
            i = ptr[f]
            while i < len(u) and u[i] < t:
                i += 1
            ptr[f] = i
            return u[i] if i < len(u) else 1 << 30

        for t, fl in enumerate(seqs):
            acts = []
            for f in fl:
                if f in slot_of:
                    acts.append(("hit", slot_of[f]))
                    continue
                if free:
                    s = free.pop()
                    slot_of[f] = s
                    acts.append(("fill", s, None))
                    continue
                cands = [v for v in slot_of if v not in fl]
                if not cands:
                    acts.append(("direct",))
                    continue
                v = max(cands, key=lambda v: next_use(v, t))
                s = slot_of.pop(v)
                slot_of[f] = s
                acts.append(("fill", s, v))
            actions.append(acts)
        return actions, slot_of

    # ------------------------------------------------------------------
    # emission
    # ------------------------------------------------------------------
    def emit_jacc(self, amp_sym, colour):
        if not self.coop:
            return super().emit_jacc(amp_sym, colour)
        acts = self._acts[self._amp_pos]
        wt = self._weights[self._amp_pos]
        self._amp_pos += 1
        if any(a[0] != "hit" for a in acts):
            # fresh copies of the flow map: lane reads stay next to their use
            # instead of being merged into long-lived registers
            self.w("    opaque_int(fm0, fm1);")
        src = amp_sym
        if wt != 1:
            self.w(f"    const cx<T> aw = T({wt!r}) * {amp_sym};  // amplitude fixed by part of the group")
            self.flops += 2
            src = "aw"
        # magnitude of the contribution for the float32 form's error estimate
        self.w(f"    const T mag = TRACK ? fabs({src}.r) + fabs({src}.i) : T(0);")
        for (order, c), act in zip(sorted(colour.items()), acts):
            k = self.kindex[order]
            op = _coef_ops(c)
            val = {"add": src, "sub": f"-{src}", "add_i": f"times_i({src})", "sub_i": f"times_mi({src})"}[op]
            if act[0] == "hit":
                s = act[1]
                if op == "add":
                    self.w(f"    jw{s} += {src};")
                elif op == "sub":
                    self.w(f"    jw{s} -= {src};")
                else:
                    self.w(f"    jw{s} += {val};")
                self.w(f"    if constexpr (TRACK) sw{s} += mag;")
                self.flops += FLOPS["jacc"]
            elif act[0] == "fill":
                s, v = act[1], act[2]
                if v is not None:
                    self.w(f"    lds_acc(Jl, fmap_at<{v}>(fm0, fm1), jw{s});")
                    self.w(f"    if constexpr (TRACK) lds_acc_s(Sl, fmap_at<{v}>(fm0, fm1), sw{s});")
                    self.flops += FLOPS["jacc"]
                self.w(f"    jw{s} = {val};")
                self.w(f"    if constexpr (TRACK) sw{s} = mag;")
            else:
                self.w(f"    lds_acc(Jl, fmap_at<{k}>(fm0, fm1), {val});")
                self.w(f"    if constexpr (TRACK) lds_acc_s(Sl, fmap_at<{k}>(fm0, fm1), mag);")
                self.flops += FLOPS["jacc"]

    def emit_program(self, cap):
        full = self.plan.amps
        self.plan.amps = [full[i] for i in self.reps]
        weights = [self.weight[i] for i in self.reps]
        self.lines, self.flops = [], 0
        self.names, self.counter = {}, 0
        self.w("mom4<double> " + ", ".join([f"q{a}" for a in range(self.n)] + ["p3", "p4"]) + ";")
        self.coop = True
        try:
            ops = self.schedule(cap)
            order = [node[1] for node in ops if node[0] == "a"]
            self._acts, live = self.plan_window(order)
            self._weights = [weights[i] for i in order]
            self._amp_pos = 0
            self.w("cx<T> " + ", ".join(f"jw{s}" for s in range(self.window)) + ";")
            self.w("T " + ", ".join(f"sw{s}" for s in range(self.window)) + ";")
            for node in ops:
                self.emit_node(node)
        finally:
            self.coop = False
            self.plan.amps = full
        for f, s in sorted(live.items()):
            self.w(f"lds_acc(Jl, fmap_at<{f}>(fm0, fm1), jw{s});")
            self.w(f"if constexpr (TRACK) lds_acc_s(Sl, fmap_at<{f}>(fm0, fm1), sw{s});")
            self.flops += FLOPS["jacc"]
        return self.lines, self.flops

    def flow_maps(self):
        """fm[w][k]: the flow that local flow k of the program becomes in wave w."""
        return [[self.kindex[tuple(pi[a] for a in o)] for o in self.perms] for pi in self.group]

    # colour sum split by blocks of the symmetric matrix
    def colour_blocks(self):
        nc = len(self.perms)
        B = self.waves
        edges = [round(i * nc / B) for i in range(B + 1)]
        blocks = [list(range(edges[i], edges[i + 1])) for i in range(B)]
        pairs = []
        for i in range(B):
            for j in range(i, B):
                cost = len(blocks[i]) * (len(blocks[i]) + 1) // 2 if i == j else len(blocks[i]) * len(blocks[j])
                pairs.append((cost, i, j))
        load = [0] * self.waves
        assign = [[] for _ in range(self.waves)]
        for cost, i, j in sorted(pairs, key=lambda t: (-t[0], t[1], t[2])):
            w = min(range(self.waves), key=lambda w: (load[w], w))
            load[w] += cost
            assign[w].append((i, j))
        return blocks, [sorted(a) for a in assign], load

    def emit_colour_part(self, pairs, blocks):
        N = self.num
        out = ["T acc = T(0);"]
        held = None
        for i, j in pairs:
            if held != i:
                if held is not None:
                    out.append("}")
                out.append("{")
                for k in blocks[i]:
                    out.append(f"const cx<T> h{k} = lds_get(Jl, {k});")
                held = i
            for l in blocks[j]:
                if i == j:
                    ks = [k for k in blocks[i] if k <= l]
                    coef = {k: (N[l][k] if k == l else 2 * N[l][k]) for k in ks}
                    src = f"h{l}"
                else:
                    ks = list(blocks[i])
                    coef = {k: 2 * N[l][k] for k in ks}
                    src = None
                ks = [k for k in ks if coef[k] != 0]
                if not ks:
                    continue
                out.append("{")
                if src is None:
                    out.append(f"    const cx<T> jl = lds_get(Jl, {l});")
                    src = "jl"
                tr = f"T({coef[ks[0]]}) * h{ks[0]}.r"
                ti = f"T({coef[ks[0]]}) * h{ks[0]}.i"
                for k in ks[1:]:
                    tr = f"fma(T({coef[k]}), h{k}.r, {tr})"
                    ti = f"fma(T({coef[k]}), h{k}.i, {ti})"
                out.append(f"    const T tr = {tr};")
                out.append(f"    const T ti = {ti};")
                out.append(f"    acc = fma({src}.r, tr, fma({src}.i, ti, acc));")
                out.append("}")
        if held is not None:
            out.append("}")
        out.append("return acc;")
        return out

    def render(self) -> str:
        alg = self.algorithmic_flops()
        n = self.n
        nc = len(self.perms)
        st = self.plan.stats()
        ext_flops = FLOPS["eps"] * n + 2 * FLOPS["spinor"]
        body, executed = self.emit_program(self.cap)
        blocks, cassign, cload = self.colour_blocks()
        fmaps = self.flow_maps()
        nfixed = sum(1 for i in self.reps if self.weight[i] != 1)
        h = []
        h.append(f"// Generated by paper_2503_21935_amd.gen for {self.name}: g g -> t tbar + {n - 2} g,")
        h.append(f"// one program for the {self.waves} waves of a workgroup sharing J in LDS.")
        h.append(f"// {st['currents']} gluon currents ({st['current_terms']} vertex terms), "
                 f"{st['L_nodes']}+{st['R_nodes']} top-line nodes, {st['amplitudes']} amplitudes, "
                 f"{st['colour_pairs']} colour-flow contributions per helicity; merge={self.plan.merge}.")
        h.append(f"// Per wave: {len(self.reps)} orbit representatives ({nfixed} weighted), "
                 f"{int(self.wave_flops)} flops with every wavefunction once, {executed} executed "
                 f"(live-set cap {self.cap}); register window {self.window}.")
        h.append(f"// Relabelling of wave w (slot -> gluon): {self.group}")
        h.append("#pragma once")
        h.append('#include "me_vertex.h"')
        h.append('#include "me_process.h"')
        h.append('#include "me_lds.h"')
        h.append("")
        h.append(f"struct proc_{self.name} {{")
        h.append(f"    static constexpr int npart = {n + 2};")
        h.append(f"    static constexpr int ngluon = {n};")
        h.append(f"    static constexpr int ncol = {nc};")
        h.append(f"    static constexpr int nhel = {1 << (n + 2)};")
        h.append(f"    static constexpr int lcd = {self.lcd};")
        h.append(f"    static constexpr int identical = {math.factorial(n - 2)};")
        h.append(f"    static constexpr int waves = {self.waves};")
        h.append(f"    static constexpr double flops_amp = {alg + ext_flops};  // per helicity, excl. colour")
        h.append(f"    static constexpr double flops_executed = "
                 f"{self.waves * (executed + ext_flops)};  // all waves, incl. recomputation")
        h.append(f"    static constexpr double flops_colour = {self.colour_flops()};  // per helicity")
        h.append(f"    static constexpr int n_amplitudes = {st['amplitudes']};")
        h.append(f"    static constexpr int ndiag = {self._ndiag()};")
        h.append("")
        step = (n - 1) // self.waves
        h.append(f"    // slot j of wave w holds gluon perm(w, j): labels 1..{n - 1} shifted cyclically by {step} w")
        h.append("    static MEV int perm(int w, int j) {")
        h.append(f"        return j == 0 ? 0 : (j - 1 + {step} * w) % {n - 1} + 1;")
        h.append("    }")
        h.append("")
        h.append("    // One helicity's program on this wave's relabelled inputs x; contributions go")
        h.append("    // to flow fm[k] of the tile's J in LDS (Jl = this lane's column), fm[k] held in")
        h.append("    // lane k of fm0 (k < 64) or lane k - 64 of fm1.  wsel: the")
        h.append("    // wave index, held in a vector register so that the per-wave choices of the")
        h.append("    // propagator momentum are selects, not branches.")
        h.append("    // TRACK: also add |contribution| into S (Sl = this lane's column of S[k][lane]).")
        h.append("    template <typename T, bool TRACK = false>")
        h.append(f"    static MEV void amps_wave(coop_ext<T, {n}>& x, T* __restrict__ Jl, T* __restrict__ Sl, "
                 "int fm0, int fm1, const int wsel) {")
        h.extend("        " + line[4:] for line in body)
        h.append("    }")
        h.append("")
        h.append("    // wave PART's share of J^dag N J (N = lcd * C, integer numerators) for this lane;")
        h.append(f"    // blocks of flows {[(b[0], b[-1]) for b in blocks]}, pairs per wave {cassign},")
        h.append(f"    // matrix entries per wave {cload}")
        h.append("    template <int PART, typename T>")
        h.append("    static MEV T colour_part(const T* __restrict__ Jl) {")
        for p in range(self.waves):
            h.append(f"        {'if' if p == 0 else '} else if'} constexpr (PART == {p}) {{")
            h.extend("            " + line for line in self.emit_colour_part(cassign[p], blocks))
        h.append("        }")
        h.append("    }")
        import numpy as np

        Nm = np.array(self.num, dtype=float)
        ev = np.linalg.eigvalsh(Nm)
        abs_lmax = float(np.linalg.eigvalsh(np.abs(Nm)).max())
        col_err = float(2 * 2.0 ** -22 * ev.max() / ev.min() + math.sqrt(nc) * 2.0 ** -24 * abs_lmax / ev.min())
        h.append(f"    static constexpr double abs_lambda_max = {abs_lmax!r};  // largest eigenvalue of |N|")
        h.append(f"    static constexpr double lambda_min = {float(ev.min())!r};  // smallest eigenvalue of N")
        h.append(f"    static constexpr double colour_err_f16 = {col_err!r};")
        h.append("};")
        h.append("")
        # B fragments of v_mfma_f32_16x16x32_f16 for N (exact in float16): for K step ks
        # and column tile t, lane l holds N[32 ks + 8 (l/16) + v][16 t + l%16], v = 0..7,
        # packed two halves per 32-bit word (zero outside N)
        ks_n, nt_n = (nc + 31) // 32, (nc + 15) // 16
        if np.abs(Nm).max() > 2048 and np.any((np.abs(Nm) > 2048) & (Nm % 2 != 0)):
            raise ValueError("colour numerators not exact in float16")
        words = []
        for ks in range(ks_n):
            for t in range(nt_n):
                for l in range(64):
                    halves = []
                    for v in range(8):
                        k, col = 32 * ks + 8 * (l // 16) + v, 16 * t + l % 16
                        val = self.num[k][col] if (k < nc and col < nc) else 0
                        halves.append(int(np.array(val, dtype=np.float16).view(np.uint16)))
                    words += [halves[2 * i] | (halves[2 * i + 1] << 16) for i in range(4)]
        h.append(f"// colour-matrix B fragments, [K step {ks_n}][column tile {nt_n}][lane 64][4 words]")
        h.append(f"__device__ static const unsigned int coop_bfrag_{self.name}[{len(words)}] = {{")
        for i in range(0, len(words), 16):
            h.append("    " + ", ".join(f"0x{w:08x}u" for w in words[i:i + 16]) + ",")
        h.append("};")
        h.append("")
        h.append(f"// flow maps of the waves, [wave][local flow]")
        h.append(f"__device__ __constant__ static const int coop_fmap_{self.name}[{self.waves * nc}] = {{")
        for row in fmaps:
            h.append("    " + ", ".join(map(str, row)) + ",")
        h.append("};")
        from .emit import emit_mfma_table

        h.extend(emit_mfma_table(self.name, self.num))
        h.append(f"template <> struct colour_table<proc_{self.name}> {{")
        h.append(f"    static MEV const double* mfma_frag() {{ return colour_mfma_{self.name}; }}")
        h.append("};")
        h.append(f"template <> struct coop_table<proc_{self.name}> {{")
        h.append(f"    static MEV const int* fmap(int w) {{ return coop_fmap_{self.name} + w * {nc}; }}")
        h.append(f"    static MEV const unsigned int* bfrag() {{ return coop_bfrag_{self.name}; }}")
        h.append("};")
        return "\n".join(h) + "\n"

    def _ndiag(self):
        from .diagrams import count_feynman_diagrams

        return count_feynman_diagrams(self.n)
