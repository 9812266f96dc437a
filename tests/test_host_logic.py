"""Host-side checks that need no GPU: the C ABI library, the process
generator's diagram counts, colour algebra and evaluation plans."""
import ctypes
import re
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    """Every function declared in include/*.h (comments stripped)."""
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if not f.endswith(".h"):
            continue
        src = open(os.path.join(inc, f)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    import paper_2503_21935_amd as me

    L = me.lib()
    names = declared_functions()
    assert {"me_init", "me_eval", "me_free", "me_info", "mlp_create", "unweight_two_stage", "ps_rambo",
            "me_eval_mixed_noalloc", "me_strerror"} <= set(names), names
    for n in names:
        assert hasattr(L, n), f"libme.so does not export {n}"


def test_strerror_needs_no_device():
    import paper_2503_21935_amd as me

    assert me.strerror(me.ME_EPROCESS) == "unknown process"
    assert me.strerror(0) == "ok"


@pytest.mark.parametrize("n,count", [(1, 1), (2, 3), (3, 16), (4, 123), (5, 1240)])
def test_diagram_counts(n, count):
    from paper_2503_21935_amd.gen.diagrams import count_feynman_diagrams

    assert count_feynman_diagrams(n) == count


@pytest.mark.parametrize("n", [2, 3, 4])
def test_generator_colour_matrix_matches_oracle(n):
    import oracle
    from paper_2503_21935_amd.gen.colour import colour_matrix_exact

    num, lcd = colour_matrix_exact(n)
    np.testing.assert_allclose(np.array(num, float) / lcd, oracle.colour_matrix(n), atol=1e-13)
    assert lcd == {2: 3, 3: 9, 4: 54}[n]


@pytest.mark.parametrize("n", [2, 3, 4])
def test_plan_covers_every_diagram(n):
    """Unmerged plan: one amplitude per Feynman diagram and four-gluon colour channel,
    and the colour-flow contributions equal those of the diagram list."""
    from paper_2503_21935_amd.gen import diagrams as D
    from paper_2503_21935_amd.gen.plan import Plan

    p = Plan(n, merge=False)
    ds = D.diagrams(n)
    n_root_terms = sum(len(a["terms"]) for a in p.amps if a["kind"] == "root")
    n_ffv = sum(1 for a in p.amps if a["kind"] == "ffv")
    assert n_root_terms + n_ffv == len(ds)
    want = sum(len(D.diagram_colour(d)) for d in ds)
    assert p.stats()["colour_pairs"] == want


@pytest.mark.parametrize("n,diagrams,amplitudes", [(1, 2, 2), (2, 8, 8), (3, 50, 54)])
def test_quark_line_with_insertion_plan(n, diagrams, amplitudes):
    """Quark line + photon/Z insertion: every ordered partition of the gluons
    into trees (1, 1, 4 trees over 1, 2, 3 gluons, four-gluon vertices once)
    with the insertion at each of the k + 1 points of k blocks; the unmerged
    plan has one amplitude per diagram and four-gluon colour channel, and the
    merged plan carries the same colour-flow sums."""
    from paper_2503_21935_amd.gen import QEW_SPECS
    from paper_2503_21935_amd.gen.plan import Plan
    from paper_2503_21935_amd.gen.qew import QEWEmitter

    name = {1: "gux_taptamux", 2: "gux_taptamgux", 3: "gux_taptamggux"}[n]
    em = QEWEmitter(name, QEW_SPECS[name])
    assert em.feynman_diagrams() == diagrams
    unmerged, merged = Plan(n, merge=False, ew=True), Plan(n, merge=True, ew=True)
    assert len(unmerged.amps) == amplitudes
    assert all(a["kind"] == "ffv" for a in merged.amps)

    def flows(p):
        tot = {}
        for a in p.amps:
            for k, v in a["colour"].items():
                tot[k] = tot.get(k, 0) + abs(v)
        return tot

    assert set(flows(unmerged)) == set(flows(merged))


@pytest.mark.parametrize("n", [3, 4])
def test_merged_plan_colour_is_consistent(n):
    """Merged plan: summing the per-diagram colour expansions of each merged
    current reproduces its normalised colour times the term coefficients."""
    from paper_2503_21935_amd.gen.plan import Plan, _term_colour

    p = Plan(n, merge=True)
    for c in p.currents:
        if c.is_leaf:
            continue
        for coef, kind, kids, ch in c.terms:
            col = _term_colour(kind, [p.currents[k].colour for k in kids], ch)
            for k, v in col.items():
                assert abs(v - coef * c.colour[k]) < 1e-12


def test_generated_flop_counts_positive():
    from paper_2503_21935_amd.gen.emit import GGEmitter

    e = GGEmitter("gg_ttgg", 4, True, 6)
    e.render()
    assert e.algorithmic_flops() > 10000


@pytest.fixture(scope="module")
def coop5():
    from paper_2503_21935_amd.gen.coop import GGCoopEmitter

    return GGCoopEmitter("gg_ttggg", 5, True, cap=12, window=16, waves=4)


def test_workgroup_program_covers_every_amplitude_once(coop5):
    """The waves' relabelled copies of the representatives give every amplitude
    of g g -> t tbar g g g with total weight exactly 1."""
    e = coop5
    tables = e._relabel_tables()
    total = np.zeros(len(e.plan.amps))
    for i in e.reps:
        for pi in e.group:
            total[e.relabel_amp(i, pi, tables)] += e.weight[i]
    assert np.array_equal(total, np.ones(len(e.plan.amps)))
    assert len(e.reps) == 243


def test_workgroup_relabelled_colour_is_consistent(coop5):
    """Relabelling a representative's colour expansion gives the colour of the
    amplitude it maps to, up to one unit phase (absorbed by the Lorentz value)."""
    e = coop5
    tables = e._relabel_tables()
    for i in e.reps:
        for pi in e.group:
            j = e.relabel_amp(i, pi, tables)
            mine = {tuple(pi[a] for a in o): v for o, v in e.plan.amps[i]["colour"].items()}
            theirs = e.plan.amps[j]["colour"]
            assert set(mine) == set(theirs)
            ratios = {complex(theirs[k] / mine[k]) for k in mine}
            assert len({(round(r.real, 12), round(r.imag, 12)) for r in ratios}) == 1
            assert abs(abs(next(iter(ratios))) - 1) < 1e-12


def test_workgroup_flow_maps(coop5):
    fm = coop5.flow_maps()
    assert fm[0] == list(range(120))
    for row in fm:
        assert sorted(row) == list(range(120))


def test_register_window_replays_to_direct_sums(coop5):
    """Replaying the window actions (fill / hit / flush / direct) on random
    amplitude values gives the same J as adding every contribution directly."""
    from paper_2503_21935_amd.gen.emit import _coef_ops

    e = coop5
    rng = np.random.default_rng(0)
    order = list(range(len(e.plan.amps)))
    rng.shuffle(order)
    for window in (4, 16):
        e.window = window
        acts, live = e.plan_window(order)
        vals = rng.normal(size=len(e.plan.amps)) + 1j * rng.normal(size=len(e.plan.amps))
        direct = np.zeros(120, complex)
        J = np.zeros(120, complex)
        slots = {}
        for t, i in enumerate(order):
            for (o, c), act in zip(sorted(e.plan.amps[i]["colour"].items()), acts[t]):
                k = e.kindex[o]
                v = complex(c) * vals[i]
                direct[k] += v
                if act[0] == "hit":
                    slots[act[1]] = (slots[act[1]][0], slots[act[1]][1] + v)
                    assert slots[act[1]][0] == k
                elif act[0] == "fill":
                    if act[2] is not None:
                        old_k, old_v = slots[act[1]]
                        assert old_k == act[2]
                        J[old_k] += old_v
                    slots[act[1]] = (k, v)
                else:
                    J[k] += v
        for s, (k, v) in slots.items():
            assert live[k] == s
            J[k] += v
        np.testing.assert_allclose(J, direct, atol=1e-12)
    e.window = 16


def test_generated_programs_do_not_depend_on_hash_seed():
    """The emitted HIP source is a function of the process alone (no set
    iteration order leaks into the schedule), so builds are reproducible."""
    import subprocess
    import sys

    code = ("import sys, hashlib; sys.path.insert(0, %r)\n"
            "from paper_2503_21935_amd.gen.emit import GGEmitter\n"
            "from paper_2503_21935_amd.gen.coop import GGCoopEmitter\n"
            "a = GGEmitter('gg_ttgg', 4, True, cap=14, cap_f32=20).render()\n"
            "b = GGCoopEmitter('gg_ttggg', 5, True, cap=16, window=16).render()\n"
            "print(hashlib.sha256((a + b).encode()).hexdigest())\n") % ROOT
    digests = set()
    for seed in ("1", "2"):
        env = dict(os.environ, PYTHONHASHSEED=seed)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, check=True)
        digests.add(r.stdout.strip())
    assert len(digests) == 1


def test_binding_fails_loudly_without_the_library(monkeypatch):
    """No silent fallback: with libme.so absent the binding raises."""
    import paper_2503_21935_amd as me

    monkeypatch.setattr(me, "_lib", None)
    monkeypatch.setattr(me, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libme.so"))
    with pytest.raises(ImportError, match="no fallback"):
        me.lib()


def test_bench_refuses_more_than_one_gpu():
    """This build runs on one GPU: --gpus 2 exits with a message (before any GPU work)."""
    import json
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
