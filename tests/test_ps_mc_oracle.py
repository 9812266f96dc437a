"""Pins of the oracle's multi-channel phase-space sampler (flat RAMBO, a Z
Breit-Wigner channel and a photon 1/M^2 channel on the invariant mass of a
final-state lepton pair; the next step after the matrix element in the
paper's outlook, Sec. 3).

Each test checks the sampler against something other than its own formulas:
the closed-form massless volume (the mean multi-channel weight is an
unbiased estimate of it), the window's share of flat phase space estimated
from flat RAMBO points, the exact distributions the channels are built to
follow (KS tests), isotropy of the decay, momentum conservation, and the
identity between the weight a channel gives its own points and the weight
computed from the final momenta alone.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle

ROOTS, MZ, WZ = 13000.0, 91.188, 2.4414


def mdot(a, b):
    return a[..., 0] * b[..., 0] - (a[..., 1:] * b[..., 1:]).sum(-1)


def volume(n, roots=ROOTS):
    return oracle.rambo(roots, [0.0] * n, 5, 0, 1)[1][0]


def pair_m2(mom, pair):
    P = mom[:, 2 + pair[0]] + mom[:, 2 + pair[1]]
    return mdot(P, P)


@pytest.mark.parametrize("n,pair,window,alpha", [
    (5, (1, 0), (50.0, ROOTS), (0.5, 0.3, 0.2)),
    (3, (1, 0), (50.0, ROOTS), (0.2, 0.6, 0.2)),
    (4, (0, 2), (80.0, 100.0), (0.1, 0.9, 0.0)),
    (5, (1, 0), (20.0, 2000.0), (0.3, 0.0, 0.7)),
])
def test_mean_weight_is_the_volume(n, pair, window, alpha):
    """With the flat channel present every point is reachable, so the mean
    multi-channel weight estimates the closed-form massless volume."""
    mom, w, ch, _ = oracle.ps_mc(ROOTS, n, pair, window, MZ, WZ, alpha, 11, 0, 1 << 16)
    V = volume(n)
    mean, err = w.mean() / V, w.std() / math.sqrt(len(w)) / V
    assert abs(mean - 1) < 5 * err, (mean, err)
    assert np.all(w > 0) and np.all(np.isfinite(w))


@pytest.mark.parametrize("c", [1, 2])
def test_single_channel_covers_the_window(c):
    """A resonance channel alone covers only the mass window: its mean weight
    is the window's share of the volume, estimated independently from flat
    RAMBO points."""
    n, pair, window = 4, (1, 0), (60.0, 4000.0)
    alpha = (0.0, 1.0, 0.0) if c == 1 else (0.0, 0.0, 1.0)
    _, w, ch, _ = oracle.ps_mc(ROOTS, n, pair, window, MZ, WZ, alpha, 12, 0, 1 << 16)
    assert np.all(ch == c)
    flat, fw = oracle.rambo(ROOTS, [0.0] * n, 13, 0, 1 << 16)
    m2 = pair_m2(flat, pair)
    inside = (m2 >= window[0] ** 2) & (m2 <= window[1] ** 2)
    share, share_err = inside.mean(), inside.std() / math.sqrt(inside.size)
    V = fw[0]
    mean, err = w.mean() / V, w.std() / math.sqrt(len(w)) / V
    assert abs(mean - share) < 5 * math.hypot(err, share_err), (mean, err, share, share_err)


@pytest.mark.parametrize("alpha", [(0.0, 1.0, 0.0), (0.0, 0.0, 1.0), (0.5, 0.5, 0.0), (0.2, 0.3, 0.5)])
def test_weight_from_momenta_matches_construction(alpha):
    """The density of a channel computed from the final momenta alone (the
    (n-1)-body configuration rebuilt from the pair) equals the one its own
    construction implies: 1/w = sum_c alpha_c g_c with g_c = 1/wc for the
    generating channel."""
    n, pair, window = 5, (1, 0), (50.0, ROOTS)
    _, w, ch, wc = oracle.ps_mc(ROOTS, n, pair, window, MZ, WZ, alpha, 14, 0, 4096)
    V = volume(n)
    a = np.array(alpha) / sum(alpha)
    for c in range(3):
        sel = ch == c
        if not sel.any():
            continue
        if a[c] == 1.0:
            np.testing.assert_allclose(w[sel], wc[sel], rtol=1e-9)
        elif c == 0:
            np.testing.assert_allclose(wc[sel], V, rtol=1e-12)
        else:
            # 1/w holds alpha_c / wc for the generating channel, alpha_0 / V for
            # the flat one, and (when its alpha is not 0) the third channel's part
            part = a[0] / V + a[c] / wc[sel]
            other = 3 - c
            if a[other] == 0:
                np.testing.assert_allclose(1 / w[sel], part, rtol=1e-9)
            else:
                assert np.all(1 / w[sel] >= part * (1 - 1e-9))


def test_breit_wigner_and_photon_mass_distributions():
    n, pair, window = 4, (1, 0), (50.0, 3000.0)
    a2, b2 = window[0] ** 2, window[1] ** 2
    mom, _, ch, _ = oracle.ps_mc(ROOTS, n, pair, window, MZ, WZ, (0.0, 0.5, 0.5), 15, 0, 1 << 14)
    m2 = pair_m2(mom, pair)
    lo, hi = math.atan((a2 - MZ ** 2) / (MZ * WZ)), math.atan((b2 - MZ ** 2) / (MZ * WZ))
    bw_cdf = lambda x: (np.arctan((x - MZ ** 2) / (MZ * WZ)) - lo) / (hi - lo)  # noqa: E731
    assert stats.kstest(m2[ch == 1], bw_cdf).pvalue > 1e-3
    log_cdf = lambda x: np.log(x / a2) / math.log(b2 / a2)  # noqa: E731
    assert stats.kstest(m2[ch == 2], log_cdf).pvalue > 1e-3
    assert np.all((m2 >= a2 * (1 - 1e-9)) & (m2 <= b2 * (1 + 1e-9)))


def test_decay_is_isotropic_and_momenta_balance():
    n, pair = 5, (1, 0)
    mom, _, ch, _ = oracle.ps_mc(ROOTS, n, pair, (50.0, ROOTS), MZ, WZ, (0.0, 1.0, 0.0), 16, 0, 1 << 14)
    P = mom[:, 2 + pair[0]] + mom[:, 2 + pair[1]]
    M = np.sqrt(mdot(P, P))
    # particle a in the pair's rest frame
    pa = mom[:, 2 + pair[0]]
    b = P[:, 1:] / P[:, :1]
    g = P[:, 0] / M
    bp = (b * pa[:, 1:]).sum(1)
    rest = pa[:, 1:] + ((g - 1) * bp / (b * b).sum(1) - g * pa[:, 0])[:, None] * b
    ct = rest[:, 2] / np.linalg.norm(rest, axis=1)
    assert stats.kstest(ct, "uniform", args=(-1, 2)).pvalue > 1e-3
    tot = mom[:, 2:].sum(1)
    np.testing.assert_allclose(tot, np.tile([ROOTS, 0, 0, 0], (len(tot), 1)), atol=1e-9 * ROOTS)
    np.testing.assert_allclose(mdot(mom[:, 2:], mom[:, 2:]), 0, atol=1e-6 * ROOTS)


def test_resonance_channel_reduces_the_variance_at_the_peak():
    """Importance sampling: for an integrand peaked like the Z line shape in the
    pair mass, the Breit-Wigner channel's weights vary far less than flat ones
    (a property of the construction, checked on the oracle's points)."""
    n, pair, window = 4, (1, 0), (50.0, ROOTS)

    def f(mom):
        m2 = pair_m2(mom, pair)
        return 1.0 / ((m2 - MZ ** 2) ** 2 + (MZ * WZ) ** 2)

    flat, fw = oracle.rambo(ROOTS, [0.0] * n, 17, 0, 1 << 14)
    mc, w, _, _ = oracle.ps_mc(ROOTS, n, pair, window, MZ, WZ, (0.1, 0.8, 0.1), 18, 0, 1 << 14)
    rv = lambda x: x.var() / x.mean() ** 2  # noqa: E731
    assert rv(fw * f(flat)) > 100 * rv(w * f(mc))
