"""Host-side checks that need no GPU: the C ABI library, the process
generator's diagram counts, colour algebra and evaluation plans."""
import ctypes
import re
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "me.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(me_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2503_21935_amd as me

    L = me.lib()
    names = declared_functions()
    assert {"me_init", "me_eval", "me_free", "me_info"} <= set(names)
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
