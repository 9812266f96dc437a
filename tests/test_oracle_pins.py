"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something other than itself: textbook
closed forms, a trace computation in another gamma-matrix representation,
gauge invariance, the Parke-Taylor formula, an explicit-colour brute force,
an exact Fierz reduction of the colour matrix, symmetries, and a quad-precision
rerun.  A dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from inputs import process_points, rambo


def mdot(a, b):
    return a[..., 0] * b[..., 0] - (a[..., 1:] * b[..., 1:]).sum(-1)


def zero_width(p):
    q = dict(p)
    q["wt"] = 0.0
    return q


# --------------------------------------------------------------------------
# e+ e- -> mu+ mu-
# --------------------------------------------------------------------------

def ee_points(cos_list, roots=500.0, phi=0.3):
    """e+ along +z, e- along -z; mu- at angle theta to the e- direction."""
    E = roots / 2
    out = []
    for c in cos_list:
        s = math.sqrt(1 - c * c)
        mum = np.array([E, E * s * math.cos(phi), E * s * math.sin(phi), -E * c])
        mup = np.array([E, -mum[1], -mum[2], -mum[3]])
        out.append([[E, 0, 0, E], [E, 0, 0, -E], mup, mum])
    return np.array(out)


def ee_closed_form(c, p, roots=500.0):
    """Helicity closed form: (e^4/4)[(|A_LL|^2+|A_RR|^2)(1+c)^2 + (|A_LR|^2+|A_RL|^2)(1-c)^2],
    A_ij = 1 + g_i g_j/(sw^2 cw^2) s/(s - MZ^2 + i MZ WZ), g_L = -1/2 + sw^2, g_R = sw^2."""
    s = roots ** 2
    sw2 = p["sw2"]
    cw2 = 1 - sw2
    chi = s / (s - p["mz"] ** 2 + 1j * p["mz"] * p["wz"])

    def A(gi, gj):
        return 1 + gi * gj / (sw2 * cw2) * chi

    gL, gR = -0.5 + sw2, sw2
    return p["e"] ** 4 / 4 * ((abs(A(gL, gL)) ** 2 + abs(A(gR, gR)) ** 2) * (1 + c) ** 2
                              + (abs(A(gL, gR)) ** 2 + abs(A(gR, gL)) ** 2) * (1 - c) ** 2)


def test_ee_closed_form(params):
    cs = np.linspace(-0.99, 0.99, 23)
    got = oracle.me2("ee_mumu", ee_points(cs), params)
    want = np.array([ee_closed_form(c, params) for c in cs])
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


def test_ee_pure_qed_limit(params):
    """With the Z decoupled (huge mass) the result is e^4 (1 + cos^2)."""
    p = dict(params)
    p["mz"] = 1e9
    p["wz"] = 0.0
    cs = np.array([-0.7, -0.1, 0.4, 0.9])
    got = oracle.me2("ee_mumu", ee_points(cs), p)
    np.testing.assert_allclose(got, p["e"] ** 4 * (1 + cs ** 2), rtol=1e-9)


def _chiral_gammas():
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]
    I2, Z2 = np.eye(2), np.zeros((2, 2))
    g = [np.block([[Z2, I2], [I2, Z2]]).astype(complex)]
    for k in range(3):
        g.append(np.block([[Z2, s[k]], [-s[k], Z2]]))
    g5 = np.block([[-I2, Z2], [Z2, I2]]).astype(complex)
    return np.array(g), g5


def test_ee_trace_route(params):
    """Sum over spins by Dirac traces in the chiral representation (no spinors)."""
    G, G5 = _chiral_gammas()
    eta = np.diag([1.0, -1, -1, -1])
    p = params
    sw2 = p["sw2"]
    gz = p["e"] / math.sqrt(sw2 * (1 - sw2))
    gL, gR = -0.5 + sw2, sw2
    PL, PR = (np.eye(4) - G5) / 2, (np.eye(4) + G5) / 2
    mom = rambo(8, 500.0, (0.0, 0.0), 3)
    want = []
    for m in mom:
        p1, p2, p3, p4 = m
        k = p1 + p2
        s = mdot(k, k)
        sl = lambda v: np.einsum("m,mij->ij", eta @ v, G)
        verts = [(-1 * p["e"]) * G, gz * np.einsum("mij,jk->mik", G, gL * PL + gR * PR)]
        props = [eta / s, (eta - np.outer(eta @ k, eta @ k) / p["mz"] ** 2)
                 / (s - p["mz"] ** 2 + 1j * p["mz"] * p["wz"])]
        g0 = G[0]
        total = 0
        for b in range(2):
            for bp in range(2):
                Gb, Gbp = verts[b], verts[bp]
                Gbp_bar = np.array([g0 @ x.conj().T @ g0 for x in Gbp])
                Te = np.einsum("mij,jk,rkl,li->mr", Gb, sl(p2), Gbp_bar, sl(p1))
                Tm = np.einsum("mij,jk,rkl,li->mr", Gb, sl(p3), Gbp_bar, sl(p4))
                total += np.einsum("mn,rs,mr,ns->", props[b], props[bp].conj(), Te, Tm)
        want.append(total.real / 4)
    got = oracle.me2("ee_mumu", mom, p)
    np.testing.assert_allclose(got, want, rtol=1e-12)


def test_ee_helicity_selection(params):
    """Massless chirality: only 4 of the 16 helicity combinations survive (the rest are
    zero up to rounding of the Dirac-representation spinors)."""
    _, qh = oracle.me2("ee_mumu", rambo(16, 500.0, (0.0, 0.0), 0), params, per_helicity=True)
    nonzero = (np.abs(qh) > 1e-25 * qh.max()).any(axis=0)
    assert nonzero.sum() == 4


# --------------------------------------------------------------------------
# g g -> t tbar
# --------------------------------------------------------------------------

def ggtt_closed_form(mom, p):
    """Ellis-Stirling-Webber / Combridge: g^4 (1/(6 t1 t2) - 3/8)(t1^2 + t2^2 + rho - rho^2/(4 t1 t2)).
    Evaluated in x87 extended precision: the invariants p1.p3 cancel in the forward region."""
    mom = np.asarray(mom, dtype=np.longdouble)
    p = {k: np.longdouble(v) for k, v in p.items()}
    s = mdot(mom[:, 0] + mom[:, 1], mom[:, 0] + mom[:, 1])
    t1 = 2 * mdot(mom[:, 0], mom[:, 2]) / s
    t2 = 2 * mdot(mom[:, 1], mom[:, 2]) / s
    rho = 4 * p["mt"] ** 2 / s
    r = p["gs"] ** 4 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 ** 2 + t2 ** 2 + rho - rho ** 2 / (4 * t1 * t2))
    return r.astype(np.float64)


def test_ggtt_closed_form(params):
    p = zero_width(params)
    mom = process_points("gg_tt", 4096, 1)
    rel = np.abs(oracle.me2("gg_tt", mom, p) / ggtt_closed_form(mom, p) - 1)
    # The closed form assumes p3^2 = m^2 exactly; the float64 inputs miss it by an
    # ulp of E^2, which very forward tops (2 p1.p3 ~ m^2) amplify to ~1e-13.
    assert rel.max() < 1e-12
    assert np.median(rel) < 1e-14


def test_ggtt_massless_limit(params):
    """m -> 0: (1/6)(t^2+u^2)/(tu) - (3/8)(t^2+u^2)/s^2 times g^4."""
    p = zero_width(params)
    p["mt"] = 0.0
    mom = rambo(64, 13000.0, (0.0, 0.0), 9).astype(np.longdouble)
    p = {k: np.longdouble(v) for k, v in p.items()}
    s = mdot(mom[:, 0] + mom[:, 1], mom[:, 0] + mom[:, 1])
    t = mdot(mom[:, 0] - mom[:, 2], mom[:, 0] - mom[:, 2])
    u = mdot(mom[:, 1] - mom[:, 2], mom[:, 1] - mom[:, 2])
    want = p["gs"] ** 4 * ((t * t + u * u) / (6 * t * u) - 3 / 8 * (t * t + u * u) / s ** 2)
    got = oracle.me2("gg_tt", mom.astype(np.float64), {k: float(v) for k, v in p.items()})
    np.testing.assert_allclose(got, want.astype(np.float64), rtol=1e-13)


def test_width_effect_is_small(params):
    """With the fixed top width on the internal lines the result moves by O((Gt/mt)^2) at most."""
    mom = process_points("gg_tt", 1024, 1)
    a = oracle.me2("gg_tt", mom, params)
    b = oracle.me2("gg_tt", mom, zero_width(params))
    assert np.max(np.abs(a / b - 1)) < 2 * (params["wt"] / params["mt"]) ** 2


# --------------------------------------------------------------------------
# Colour matrix
# --------------------------------------------------------------------------

def fierz_colour_row(n):
    """Exact C_{0,l}: Tr(T^{a_n}..T^{a_1} T^{b_1}..T^{b_n}) with b = a permuted, reduced with
    T^a_ij T^a_kl = 1/2 (d_il d_kj - d_ij d_kl / N) on traces of words (N = 3)."""
    N = Fraction(3)

    def reduce(traces):
        # traces: tuple of words (tuples of labels); each label appears twice overall.
        labels = [x for w in traces for x in w]
        if not labels:
            return N ** len(traces)
        lab = labels[0]
        pos = [(ti, i) for ti, w in enumerate(traces) for i, x in enumerate(w) if x == lab]
        (t1, i1), (t2, i2) = pos
        others = [w for ti, w in enumerate(traces) if ti not in (t1, t2)]
        if t1 == t2:
            w = traces[t1]
            A, B = w[:i1], w[i1 + 1:i2]
            C = w[i2 + 1:]
            # Tr(A T B T C) = 1/2 [Tr(B) Tr(C A) - Tr(A B C)/N]
            t_a = tuple(others) + (B, C + A)
            t_b = tuple(others) + (A + B + C,)
        else:
            w1, w2 = traces[t1], traces[t2]
            A = w1[i1 + 1:] + w1[:i1]
            B = w2[i2 + 1:] + w2[:i2]
            # Tr(T A) Tr(T B) = 1/2 [Tr(A B) - Tr(A) Tr(B)/N]
            t_a = tuple(others) + (A + B,)
            t_b = tuple(others) + (A, B)
        return Fraction(1, 2) * (reduce(t_a) - reduce(t_b) / N)

    perms = list(itertools.permutations(range(n)))
    first = perms[0]
    row = []
    for s in perms:
        word = tuple(reversed(first)) + tuple(s)
        row.append(reduce((word,)))
    return perms, row


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_colour_matrix_exact(n):
    C = oracle.colour_matrix(n)
    perms, row = fierz_colour_row(n)
    # C_kl depends only on sigma_k^-1 sigma_l: fill the whole matrix from row 0.
    index = {p: i for i, p in enumerate(perms)}
    for k, sk in enumerate(perms):
        inv = np.argsort(sk)
        for l, sl in enumerate(perms):
            rel = tuple(int(inv[x]) for x in sl)
            assert abs(C[k, l] - float(row[index[rel]])) < 1e-12 * abs(C[0, 0])
    # diagonal C_F^n N, symmetric, positive definite
    assert abs(C[0, 0] - (4 / 3) ** n * 3) < 1e-12
    np.testing.assert_allclose(C, C.T, atol=1e-12)
    assert np.linalg.eigvalsh(C).min() > 0


def test_colour_matrix_ggtt():
    np.testing.assert_allclose(oracle.colour_matrix(2), [[16 / 3, -2 / 3], [-2 / 3, 16 / 3]], atol=1e-14)


# --------------------------------------------------------------------------
# g g -> t tbar + gluons
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_gauge_invariance(n, params):
    """eps(k_i) -> k_i/k_i^0 sends every colour-ordered amplitude to zero (Gt = 0)."""
    p = zero_width(params)
    mom = rambo(2, 13000.0, (173.0, 173.0) + (0.0,) * (n - 2), 40 + n)
    for ev in range(2):
        for h in (0, 3, 10, (1 << (n + 2)) - 1):
            ref = np.abs(oracle.ordered_amps(n, mom[ev], h, p)).max()
            for g in range(n):
                J = oracle.ordered_amps(n, mom[ev], h, p, gauge_gluon=g)
                assert np.abs(J).max() < 1e-11 * ref


def _mhv_ratios(n, mom, p, quad=False):
    gpart = [0, 1] + list(range(4, n + 2))
    npart = n + 2
    ratios = []
    for m in mom:
        out = m.copy()
        out[0] *= -1
        out[1] *= -1
        s = lambda a, b: abs(2 * mdot(out[a], out[b]))
        for h in range(1 << npart):
            lam = [1 if (h >> (npart - 1 - i)) & 1 else -1 for i in range(npart)]
            lo = [-l if i < 2 else l for i, l in enumerate(lam)]  # helicities, all outgoing
            negs = [i for i in range(npart) if lo[i] < 0]
            if len(negs) != 2 or not ((2 in negs) ^ (3 in negs)):
                continue
            gi = [i for i in negs if i not in (2, 3)][0]
            qneg = 2 if 2 in negs else 3
            other = 5 - qneg
            J = oracle.ordered_amps(n, m, h, p, quad=quad)
            for k, sig in enumerate(oracle.orderings(n)):
                chain = [2] + [gpart[a] for a in sig] + [3]
                den = np.prod([s(a, b) for a, b in zip(chain, chain[1:] + chain[:1])])
                ratios.append(abs(J[k]) ** 2 / (s(qneg, gi) ** 3 * s(other, gi) / den))
    return np.array(ratios)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_parke_taylor_mhv(n, params):
    """Massless quarks: |J_sigma|^2 = 2^n g^(2n) s_{q i}^3 s_{qbar i} / (s_{q s1} ... s_{sn qbar} s_{qbar q})
    for every MHV helicity configuration and ordering (Mangano-Parke)."""
    p = zero_width(params)
    p["mt"] = 0.0
    mom = rambo(2, 13000.0, (0.0,) * n, 60 + n)
    # Some orderings are suppressed by large cancellations between diagrams, so the
    # double build reaches only ~1e-9 there; the __float128 build pins the formula.
    r = _mhv_ratios(n, mom, p, quad=True)
    assert r.size > 0
    np.testing.assert_allclose(r, 2 ** n * p["gs"] ** (2 * n), rtol=1e-10)
    np.testing.assert_allclose(_mhv_ratios(n, mom, p), 2 ** n * p["gs"] ** (2 * n), rtol=1e-7)


@pytest.mark.parametrize("n,nev", [(2, 4), (3, 4), (4, 1)])
def test_colour_dressed_brute_force(n, nev, params):
    """Explicit colour sum with unordered full Feynman rules == colour-ordered route + C."""
    proc = {2: "gg_tt", 3: "gg_ttg", 4: "gg_ttgg"}[n]
    mom = process_points(proc, nev, 20 + n)
    want = oracle.me2(proc, mom, params)
    got = np.array([oracle.me2_dressed(n, m, params) for m in mom])
    np.testing.assert_allclose(got, want, rtol=1e-12)


def _boost_rotate(mom, beta, axis, angle, raxis):
    axis = axis / np.linalg.norm(axis)
    g = 1 / math.sqrt(1 - beta ** 2)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = g * beta * axis
    L[1:, 1:] += (g - 1) * np.outer(axis, axis)
    raxis = raxis / np.linalg.norm(raxis)
    K = np.array([[0, -raxis[2], raxis[1]], [raxis[2], 0, -raxis[0]], [-raxis[1], raxis[0], 0]])
    R = np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K
    Rf = np.eye(4)
    Rf[1:, 1:] = R
    return np.einsum("ij,...j->...i", Rf @ L, mom)


@pytest.mark.parametrize("proc", ["ee_mumu", "gg_tt", "gg_ttg", "gg_ttgg"])
def test_lorentz_invariance(proc, params):
    """Random boost and rotation.  At zero top width: a fixed width breaks gauge invariance at
    O(Gt/mt), and with it the frame independence of the physical-polarisation helicity sum."""
    p = zero_width(params)
    mom = process_points(proc, 6, 77)
    rng = np.random.default_rng(5)
    a = oracle.me2(proc, mom, p)
    moved = _boost_rotate(mom, 0.9 * rng.random(), rng.normal(size=3), 2 * math.pi * rng.random(),
                          rng.normal(size=3))
    b = oracle.me2(proc, moved, p)
    np.testing.assert_allclose(b, a, rtol=1e-11)


@pytest.mark.parametrize("proc,nf", [("gg_tt", 0), ("gg_ttg", 1), ("gg_ttgg", 2), ("gg_ttggg", 3)])
def test_bose_symmetry(proc, nf, params):
    nev = 3 if nf < 3 else 1
    mom = process_points(proc, nev, 88)
    a = oracle.me2(proc, mom, params)
    swapped = mom[:, [1, 0] + list(range(2, mom.shape[1]))]
    np.testing.assert_allclose(oracle.me2(proc, swapped, params), a, rtol=1e-12)
    if nf >= 2:
        idx = list(range(mom.shape[1]))
        idx[4], idx[-1] = idx[-1], idx[4]
        np.testing.assert_allclose(oracle.me2(proc, mom[:, idx], params), a, rtol=1e-12)


def test_quad_rerun_agrees(params):
    """The __float128 build reproduces the double results (no precision bug in the double path)."""
    for proc, nev in (("ee_mumu", 32), ("gg_tt", 32), ("gg_ttgg", 4)):
        mom = process_points(proc, nev, 5)
        np.testing.assert_allclose(oracle.me2(proc, mom, params, quad=True), oracle.me2(proc, mom, params),
                                   rtol=1e-12)


def test_helicity_terms_positive(params):
    mom = process_points("gg_ttg", 8, 3)
    _, qh = oracle.me2("gg_ttg", mom, params, per_helicity=True)
    assert (qh > 0).all()


# --------------------------------------------------------------------------
# Inputs (phase space)
# --------------------------------------------------------------------------

def test_rambo_kinematics():
    for proc in ("ee_mumu", "gg_tt", "gg_ttgg", "gg_ttggg"):
        mom = process_points(proc, 2000, 1)
        from inputs import PROCESS_KINEMATICS

        masses = np.array(PROCESS_KINEMATICS[proc]["masses"])
        m2 = mdot(mom[:, 2:], mom[:, 2:])
        E2 = mom[:, 2:, 0] ** 2
        assert np.max(np.abs(m2 - masses ** 2) / E2) < 1e-14
        bal = mom[:, 0] + mom[:, 1] - mom[:, 2:].sum(axis=1)
        assert np.max(np.abs(bal)) < 1e-12 * mom[0, 0, 0] * 2


def test_rambo_volume():
    """2-body massive: weight = beta/(8 pi); massless n-body: the closed-form volume."""
    from inputs import massless_volume

    _, w = rambo(100, 13000.0, (173.0, 173.0), 1, return_weight=True)
    beta = math.sqrt(1 - 4 * 173.0 ** 2 / 13000.0 ** 2)
    np.testing.assert_allclose(w, beta / (8 * math.pi), rtol=1e-13)
    _, w = rambo(10, 100.0, (0.0,) * 4, 1, return_weight=True)
    np.testing.assert_allclose(w, massless_volume(4, 1e4), rtol=1e-15)
    assert abs(massless_volume(2, 1.0) - 1 / (8 * math.pi)) < 1e-16


def test_rambo_seeded():
    a = process_points("gg_ttgg", 16, 2)
    b = process_points("gg_ttgg", 16, 2)
    c = process_points("gg_ttgg", 16, 3)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


# --------------------------------------------------------------------------
# Route 4: single diagrams (the multi-channel weights)
# --------------------------------------------------------------------------

def _double_factorial_odd(k):
    return 1 if k <= 0 else k * _double_factorial_odd(k - 2)


@pytest.mark.parametrize("n,total", [(2, 3), (3, 16), (4, 123), (5, 1240)])
def test_channel_diagram_count(n, total):
    """Three-point-only diagrams: sum over ordered set partitions of the gluons
    of the product of (2m - 3)!! (binary trees on m labelled leaves), counted
    here by set partitions times block orderings; the rest of the process's
    diagrams (3, 16, 123, 1240) contain a four-gluon vertex."""
    descs, _ = oracle.channel_diagrams(n)
    assert len(set(descs)) == len(descs)

    def set_partitions(items):
        if not items:
            yield []
            return
        first, rest = items[0], items[1:]
        for part in set_partitions(rest):
            for i in range(len(part)):
                yield part[:i] + [[first] + part[i]] + part[i + 1:]
            yield [[first]] + part

    count = sum(math.factorial(len(p)) * math.prod(_double_factorial_odd(2 * len(b) - 3) for b in p)
                for p in set_partitions(list(range(n))))
    assert len(descs) == count
    assert total - count == {2: 0, 3: 1, 4: 18, 5: 295}[n]


def _leaves(tree_desc):
    return [int(c) for c in tree_desc.replace("(", " ").replace(")", " ").replace(",", " ").split()]


def _tree(desc):
    import ast

    return ast.literal_eval(desc) if "(" in desc else int(desc)


def _ordered_coefficient(trees, sigma):
    """Coefficient of diagram (trees along the top line) in the colour-ordered
    amplitude of ordering sigma: 0 unless every block and every subtree is
    contiguous in sigma with the blocks in top-line order; otherwise the product
    over vertices of +1 (subtree with the smaller label first in sigma) or -1."""
    pos = {a: i for i, a in enumerate(sigma)}
    start = 0
    coef = 1

    def span(t):
        if isinstance(t, int):
            return [pos[t]]
        return span(t[0]) + span(t[1])

    def signs(t):
        if isinstance(t, int):
            return 1
        a, b = span(t[0]), span(t[1])
        s = 1 if max(a) < min(b) else -1
        return s * signs(t[0]) * signs(t[1])

    for t in trees:
        sp = sorted(span(t))
        if sp != list(range(start, start + len(sp))):
            return 0
        # each subtree contiguous
        def contiguous(u):
            if isinstance(u, int):
                return True
            s = sorted(span(u))
            return s == list(range(s[0], s[0] + len(s))) and contiguous(u[0]) and contiguous(u[1])

        if not contiguous(t):
            return 0
        coef *= signs(t)
        start += len(sp)
    return coef


@pytest.mark.parametrize("n", [2, 3, 4])
def test_single_diagrams_recombine_into_ordered_amplitudes(n, params):
    """For every gluon ordering sigma and helicity, the colour-ordered amplitude
    of the recursion with the four-gluon vertex left out equals the sum of the
    single three-point diagrams consistent with sigma, each with coefficient +-1:
    the diagram route and the Berends-Giele route agree term by term."""
    proc = {2: "gg_tt", 3: "gg_ttg", 4: "gg_ttgg"}[n]
    mom = process_points(proc, 2, 60 + n)[1]
    perms = oracle.orderings(n)
    nhel = 1 << (n + 2)
    rng = np.random.default_rng(n)
    for h in rng.choice(nhel, 6, replace=False):
        descs, A = oracle.diagram_amps(n, mom, int(h), params)
        trees = [[_tree(b) for b in d.split("|")] for d in descs]
        J3 = oracle.ordered_amps(n, mom, int(h), params, four_gluon=False)
        for k, sigma in enumerate(perms):
            c = np.array([_ordered_coefficient(t, sigma) for t in trees], dtype=float)
            want = J3[k]
            got = np.dot(c, A)
            scale = np.abs(A).max()
            assert abs(got - want) <= 1e-12 * scale, (n, h, sigma, got, want)
    if n == 2:  # no four-gluon diagrams: the full ordered amplitudes
        for h in range(nhel):
            descs, A = oracle.diagram_amps(n, mom, h, params)
            J = oracle.ordered_amps(n, mom, h, params)
            trees = [[_tree(b) for b in d.split("|")] for d in descs]
            for k, sigma in enumerate(perms):
                c = np.array([_ordered_coefficient(t, sigma) for t in trees], dtype=float)
                assert abs(np.dot(c, A) - J[k]) <= 1e-12 * np.abs(A).max()


def _relabel(desc, perm):
    """Descriptor of a diagram after gluon relabelling a -> perm[a], in canonical form."""
    def canon(t):
        if isinstance(t, int):
            return perm[t], perm[t]
        (a, ma), (b, mb) = canon(t[0]), canon(t[1])
        return ((a, b), min(ma, mb)) if ma < mb else ((b, a), min(ma, mb))

    def fmt(t):
        return str(t) if isinstance(t, int) else "(" + fmt(t[0]) + "," + fmt(t[1]) + ")"

    return "|".join(fmt(canon(_tree(b))[0]) for b in desc.split("|"))


def test_single_diagrams_bose_and_lorentz(params):
    """Exchanging the two final gluons maps every diagram onto its relabelled
    partner with the same helicity-summed |A|^2; a rotation of all momenta
    leaves every diagram's helicity sum unchanged.  (Single diagrams are not
    boost invariant: the polarisation vectors are transverse in the frame of
    the momenta, a gauge choice that only the sum of all diagrams forgets.)"""
    p = zero_width(params)
    mom = process_points("gg_ttgg", 3, 64)
    descs, s0 = oracle.diagram_sums("gg_ttgg", mom, p)
    index = {d: i for i, d in enumerate(descs)}
    swapped = mom[:, [0, 1, 2, 3, 5, 4]]
    _, s1 = oracle.diagram_sums("gg_ttgg", swapped, p)
    perm = [0, 1, 3, 2]
    for i, d in enumerate(descs):
        np.testing.assert_allclose(s1[:, index[_relabel(d, perm)]], s0[:, i], rtol=1e-12)
    rng = np.random.default_rng(9)
    moved = _boost_rotate(mom, 0.0, rng.normal(size=3), 1.1, rng.normal(size=3))
    _, s2 = oracle.diagram_sums("gg_ttgg", moved, p)
    np.testing.assert_allclose(s2, s0, rtol=1e-10)
