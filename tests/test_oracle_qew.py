"""Pins of the oracle's route 5: a massless quark line with gluons and a
gamma/Z -> lepton pair (the paper's DY+3j subprocess g ubar -> tau+ tau- g g
ubar, Sec. 3, and the smaller members of that family).

Each test checks the route against something other than itself: the
lowest-order Drell-Yan closed form, the e+ e- -> mu+ mu- closed form through
the same insertion with electron couplings, gauge invariance for every gluon
and for the photon current, the U(1) decoupling identity against the gluon
recursion of route 2, Lorentz invariance, Bose symmetry and a quad-precision
rerun.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from inputs import rambo

FAMILY = ("uux_taptam", "gux_taptamux", "gux_taptamgux", "gux_taptamggux")


def mdot(a, b):
    return a[..., 0] * b[..., 0] - (a[..., 1:] * b[..., 1:]).sum(-1)


def points(process, n, seed, roots=1000.0):
    spec = oracle.QEW_PROCESSES[process]
    return rambo(n, roots, (0.0,) * (spec["npart"] - 2), seed)


def dy_closed_form(mom, p, quark, lepton, colour_factor):
    """q(p1) qbar(p2) -> l+(p3) l-(p4), massless, averaged over spins (1/4):
    sum |M|^2 = 4 [(|A_LL|^2 + |A_RR|^2) u^2 + (|A_LR|^2 + |A_RL|^2) t^2] x colour,
    A_ij = e^2 Qq Ql / s + g_Z^2 g_i(q) g_j(l) / (s - M_Z^2 + i M_Z Gamma_Z),
    g_L = T3 - Q sin^2, g_R = -Q sin^2, u = (p1 - p3)^2, t = (p1 - p4)^2."""
    s = mdot(mom[:, 0] + mom[:, 1], mom[:, 0] + mom[:, 1])
    u = mdot(mom[:, 0] - mom[:, 2], mom[:, 0] - mom[:, 2])
    t = mdot(mom[:, 0] - mom[:, 3], mom[:, 0] - mom[:, 3])
    sw2 = p["sw2"]
    gz2 = p["e"] ** 2 / (sw2 * (1 - sw2))
    (Qq, T3q), (Ql, T3l) = quark, lepton
    gq = {"L": T3q - Qq * sw2, "R": -Qq * sw2}
    gl = {"L": T3l - Ql * sw2, "R": -Ql * sw2}
    dz = s - p["mz"] ** 2 + 1j * p["mz"] * p["wz"]

    def A(i, j):
        return p["e"] ** 2 * Qq * Ql / s + gz2 * gq[i] * gl[j] / dz

    tot = 4 * ((abs(A("L", "L")) ** 2 + abs(A("R", "R")) ** 2) * u ** 2
               + (abs(A("L", "R")) ** 2 + abs(A("R", "L")) ** 2) * t ** 2)
    return tot * colour_factor / 4


def test_drell_yan_closed_form(params):
    mom = points("uux_taptam", 64, 3, roots=200.0)
    got = oracle.qew_me2("uux_taptam", mom, params)
    want = dy_closed_form(mom, params, (2 / 3, 0.5), (-1, -0.5), 3 / 9)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)
    # near the Z pole too (the width term matters there)
    mom = points("uux_taptam", 16, 4, roots=params["mz"] + 0.3)
    np.testing.assert_allclose(oracle.qew_me2("uux_taptam", mom, params),
                               dy_closed_form(mom, params, (2 / 3, 0.5), (-1, -0.5), 3 / 9), rtol=1e-12)


def test_down_type_and_electron_couplings(params):
    """Other charges through the same insertion: a d quark line, and e+ e- ->
    mu+ mu- (electron couplings, no colour) against route 1."""
    spec = dict(oracle.QEW_PROCESSES["uux_taptam"], quark=(-1 / 3, -0.5))
    mom = points("uux_taptam", 32, 5, roots=300.0)
    np.testing.assert_allclose(oracle.qew_me2(spec, mom, params),
                               dy_closed_form(mom, params, (-1 / 3, -0.5), (-1, -0.5), 3 / 9), rtol=1e-12)
    # e+(p1) e-(p2) -> mu+(p3) mu-(p4): row e+ (incoming antifermion), column e-
    ee = dict(n=0, npart=4, row=(0, 1), col=(1, 1), lm=3, lp=2, gluons=(), quark=(-1.0, -0.5),
              lepton=(-1.0, -0.5), avg=4)
    mom = rambo(32, 500.0, (0.0, 0.0), 6)
    np.testing.assert_allclose(oracle.qew_me2(ee, mom, params, colour=np.array([[1.0]])),
                               oracle.me2("ee_mumu", mom, params), rtol=1e-12)


def _largest_amp(process, mom1, params):
    spec = oracle.QEW_PROCESSES[process] if isinstance(process, str) else process
    return max(np.abs(oracle.qew_amps(process, mom1, h, params)).max() for h in range(1 << spec["npart"]))


@pytest.mark.parametrize("process", FAMILY[1:])
def test_gluon_gauge_invariance(params, process):
    """eps -> q/q0 for any gluon: every colour-ordered amplitude vanishes (to
    rounding, relative to the event's largest amplitude)."""
    spec = oracle.QEW_PROCESSES[process]
    mom = points(process, 3, 7)
    for ev in range(3):
        ref = _largest_amp(process, mom[ev], params)
        for h in range(0, 1 << spec["npart"], 3):
            if np.abs(oracle.qew_amps(process, mom[ev], h, params)).max() < 1e-6 * ref:
                continue  # a vanishing helicity
            for a in range(spec["n"]):
                g = oracle.qew_amps(process, mom[ev], h, params, gauge_gluon=a)
                assert np.abs(g).max() <= 1e-11 * ref, (process, ev, h, a)


@pytest.mark.parametrize("process", FAMILY)
def test_photon_current_conservation(params, process):
    """The insertion's vectors replaced by its momentum k: the quark line
    contracted with k vanishes, order by order (relative to the amplitude with
    the insertion scaled to carry |k|)."""
    spec = oracle.QEW_PROCESSES[process]
    mom = points(process, 3, 8)
    for ev in range(3):
        ref = _largest_amp(process, mom[ev], params)
        for h in range(0, 1 << spec["npart"], 3):
            if np.abs(oracle.qew_amps(process, mom[ev], h, params)).max() < 1e-6 * ref:
                continue
            ins = oracle.qew_externals(process, mom[ev], h, params)
            scale = ref * abs(ins["qE"][0]) / max(np.abs(ins["EL"]).max(), np.abs(ins["ER"]).max())
            g = oracle.qew_amps(process, mom[ev], h, params, gauge_ew=True)
            assert np.abs(g).max() <= 1e-11 * scale, (process, ev, h)


@pytest.mark.parametrize("process", FAMILY[1:])
def test_u1_decoupling_against_gluon_recursion(params, process):
    """A colourless vector on the quark line is a gluon with an identity
    generator: summing route 2's colour-ordered amplitudes (three- and
    four-gluon vertices included) over the positions of an extra leg carrying
    the insertion gives route 5's amplitude for the order of the other gluons.
    A vector-like quark coupling (T3 = 0) makes the insertion gamma.E."""
    spec = dict(oracle.QEW_PROCESSES[process], quark=(2 / 3, 0.0))
    n = spec["n"]
    g = params["gs"]
    mom = points(process, 2, 9)
    orders = oracle.orderings(n)
    checked = 0
    for ev in range(2):
        ref = _largest_amp(spec, mom[ev], params)
        for h in range(0, 1 << spec["npart"], 5):
            got = oracle.qew_amps(spec, mom[ev], h, params)
            if np.abs(got).max() < 1e-6 * ref:
                continue  # a vanishing helicity
            ext = oracle.qew_externals(spec, mom[ev], h, params)
            np.testing.assert_allclose(ext["EL"], ext["ER"], rtol=1e-14, atol=0)
            q = np.vstack([ext["q"], ext["qE"][None]])
            eps = np.vstack([ext["eps"], (ext["EL"] / (1j * g))[None]])
            for k, sig in enumerate(orders):
                tot = 0
                for pos in range(n + 1):
                    s = list(sig[:pos]) + [n] + list(sig[pos:])
                    tot += oracle.bg_custom(q, eps, ext["prow"], ext["row"], ext["col"], s, g)
                assert abs(tot - got[k]) <= 1e-12 * ref, (ev, h, k)
                checked += 1
    assert checked > 0


@pytest.mark.parametrize("process", FAMILY)
def test_lorentz_invariance(params, process):
    mom = points(process, 16, 10)
    b = np.array([0.3, -0.2, 0.5])
    g = 1 / math.sqrt(1 - b @ b)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = g * b
    L[1:, 1:] += (g - 1) * np.outer(b, b) / (b @ b)
    boosted = np.einsum("ij,epj->epi", L, mom)
    np.testing.assert_allclose(oracle.qew_me2(process, boosted, params), oracle.qew_me2(process, mom, params),
                               rtol=1e-10)


def test_bose_symmetry_of_the_two_gluons(params):
    mom = points("gux_taptamggux", 16, 11)
    swapped = mom.copy()
    swapped[:, [4, 5]] = mom[:, [5, 4]]
    np.testing.assert_allclose(oracle.qew_me2("gux_taptamggux", swapped, params),
                               oracle.qew_me2("gux_taptamggux", mom, params), rtol=1e-12)


def test_helicity_conservation(params):
    """Massless quark and lepton lines conserve chirality: of the 2^7
    helicities a quarter survive (the rest vanish to rounding)."""
    spec = oracle.QEW_PROCESSES["gux_taptamggux"]
    mom = points("gux_taptamggux", 2, 12)
    _, qh = oracle.qew_me2("gux_taptamggux", mom, params, per_helicity=True)
    nz = (qh > 1e-12 * qh.max(axis=1, keepdims=True)).sum(axis=1)
    assert np.all(nz == (1 << spec["npart"]) // 4)


def test_quad_agreement(params):
    mom = points("gux_taptamggux", 4, 13)
    d = oracle.qew_me2("gux_taptamggux", mom, params)
    q = oracle.qew_me2("gux_taptamggux", mom, params, quad=True)
    np.testing.assert_allclose(d, q, rtol=1e-12)
