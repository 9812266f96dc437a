"""Pins of the phase-space oracle (oracle/ps_oracle.c): Philox4x32-10 against
its published known-answer vectors, the uniforms' distribution, and RAMBO
against closed forms, conservation laws and an independent numerical
integration of the massive three-body volume."""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def kat_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", kat_rows())
def test_philox_known_answers(ctr, key, want):
    assert oracle.philox4x32(ctr, key, 10) == want


def test_uniform_stream_distribution():
    """Uniforms of the event stream: strictly inside (0, 1), uniform by a KS
    test, first and second moments, and no correlation between neighbours."""
    from scipy import stats

    u = np.concatenate([oracle.event_uniforms(7, e, 16) for e in range(4000)])
    assert np.all((u > 0) & (u < 1))
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    n = u.size
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * math.sqrt(1 / 180 / n)
    c = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(c) < 5 / math.sqrt(n)
    # a different seed or event gives a different stream
    assert not np.array_equal(oracle.event_uniforms(7, 0, 16), oracle.event_uniforms(8, 0, 16))
    assert not np.array_equal(oracle.event_uniforms(7, 0, 16), oracle.event_uniforms(7, 1, 16))


def test_uniform_construction_from_the_words():
    """Uniform 2b of an event comes from words 0, 1 of Philox block b, uniform
    2b + 1 from words 2, 3 (53 bits, offset by half an ulp)."""
    seed, ev = (5 << 32) | 9, (3 << 32) | 11
    u = oracle.event_uniforms(seed, ev, 6)
    for b in range(3):
        w = oracle.philox4x32([ev & 0xFFFFFFFF, ev >> 32, b, 0], [seed & 0xFFFFFFFF, seed >> 32])
        for j in range(2):
            v = ((w[2 * j] << 32) | w[2 * j + 1]) >> 11
            assert u[2 * b + j] == (v + 0.5) * 2.0 ** -53


def volume_massless(n, s):
    return (2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2) / (
        math.factorial(n - 1) * math.factorial(n - 2))


@pytest.mark.parametrize("roots,masses", [(500.0, [0, 0]), (13000.0, [0, 0, 0]), (13000.0, [173.0, 173.0, 0, 0]),
                                          (13000.0, [173.0, 173.0, 0, 0, 0]), (400.0, [173.0, 173.0])])
def test_rambo_conservation_and_shell(roots, masses):
    mom, wt = oracle.rambo(roots, masses, 3, 0, 2000)
    # the conformal map divides by the mass of the sum of the generated q's,
    # which is small when they are nearly collinear: rounding grows there
    tot = mom[:, 2:].sum(axis=1)
    np.testing.assert_allclose(tot[:, 0], roots, rtol=1e-11)
    assert np.abs(tot[:, 1:]).max() < 1e-11 * roots
    m2 = mom[:, 2:, 0] ** 2 - (mom[:, 2:, 1:] ** 2).sum(-1)
    np.testing.assert_allclose(m2, np.broadcast_to(np.square(masses), m2.shape), atol=1e-9 * roots ** 2)
    assert np.all(wt > 0)
    np.testing.assert_array_equal(mom[:, 0], [[roots / 2, 0, 0, roots / 2]] * len(mom))
    np.testing.assert_array_equal(mom[:, 1], [[roots / 2, 0, 0, -roots / 2]] * len(mom))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7])
def test_rambo_massless_weight_is_the_volume(n):
    mom, wt = oracle.rambo(1000.0, [0.0] * n, 1, 0, 50)
    np.testing.assert_allclose(wt, volume_massless(n, 1000.0 ** 2), rtol=1e-13)


def test_rambo_two_body_massive_closed_form():
    """Two bodies: |k| = lambda^(1/2)(s, m1^2, m2^2) / (2 sqrt s) and the volume
    lambda^(1/2) / (8 pi s)."""
    roots, m1, m2 = 400.0, 173.0, 20.0
    s = roots ** 2
    lam = (s - (m1 + m2) ** 2) * (s - (m1 - m2) ** 2)
    mom, wt = oracle.rambo(roots, [m1, m2], 4, 0, 200)
    k = np.sqrt((mom[:, 2, 1:] ** 2).sum(-1))
    np.testing.assert_allclose(k, math.sqrt(lam) / (2 * roots), rtol=1e-13)
    np.testing.assert_allclose(wt, math.sqrt(lam) / (8 * math.pi * s), rtol=1e-12)


def test_rambo_three_body_energy_spectrum():
    """Massless three-body flat phase space is flat in (E1, E2) on the Dalitz
    triangle, so E1 has density 2 E / (sqrt(s)/2)^2 on [0, sqrt(s)/2]:
    in units of the endpoint sqrt(s)/2, mean 2/3, second moment 1/2, CDF x^2."""
    roots = 100.0
    mom, _ = oracle.rambo(roots, [0, 0, 0], 11, 0, 200000)
    e1 = mom[:, 2, 0] / (roots / 2)  # in units of the endpoint
    # density 2x on [0, 1]: mean 2/3, second moment 1/2, and its CDF x^2
    assert abs(e1.mean() - 2 / 3) < 5 * math.sqrt((1 / 2 - 4 / 9) / e1.size)
    assert abs((e1 ** 2).mean() - 1 / 2) < 5 * math.sqrt((1 / 3 - 1 / 4) / e1.size)
    from scipy import stats

    assert stats.kstest(e1, lambda x: np.clip(x, 0, 1) ** 2).pvalue > 1e-3
    # isotropy
    c = mom[:, 2, 3] / np.sqrt((mom[:, 2, 1:] ** 2).sum(-1))
    assert abs(c.mean()) < 5 / math.sqrt(3 * c.size)


def test_rambo_massive_three_body_volume_by_quadrature():
    """The mean RAMBO weight for three massive bodies equals the three-body
    volume from the two-body factorisation
    Phi_3(s) = int dM^2 / (2 pi) Phi_2(s; m1, M) Phi_2(M^2; m2, m3),
    Phi_2(s; a, b) = lambda^(1/2)(s, a^2, b^2) / (8 pi s), integrated numerically."""
    from scipy import integrate

    roots, m = 600.0, [173.0, 173.0, 30.0]
    s = roots ** 2

    def phi2(ss, a, b):
        lam = (ss - (a + b) ** 2) * (ss - (a - b) ** 2)
        return math.sqrt(max(lam, 0.0)) / (8 * math.pi * ss)

    lo, hi = (m[1] + m[2]) ** 2, (roots - m[0]) ** 2
    vol, _ = integrate.quad(lambda M2: phi2(s, m[0], math.sqrt(M2)) * phi2(M2, m[1], m[2]) / (2 * math.pi), lo, hi,
                            epsabs=0, epsrel=1e-10, limit=200)
    _, wt = oracle.rambo(roots, m, 21, 0, 400000)
    err = wt.std() / math.sqrt(wt.size)
    assert abs(wt.mean() - vol) < 5 * err, (wt.mean(), vol, err)
    assert err < 2e-2 * vol  # the comparison is meaningful
