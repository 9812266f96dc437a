"""GPU multi-channel phase-space sampling (ps_multichannel: flat, Z
Breit-Wigner and photon 1/M^2 channels on a lepton pair's mass) against the
CPU oracle on the same counter-based random streams."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

ROOTS, MZ, WZ = 13000.0, 91.188, 2.4414


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_21935_amd as me

    me.lib()
    return torch, me


def mdot(a, b):
    return a[..., 0] * b[..., 0] - (a[..., 1:] * b[..., 1:]).sum(-1)


CASES = [
    # name, nfinal, pair, window, alpha, seed, first, n
    ("dy3j", 5, (0, 1), (50.0, ROOTS), (0.5, 0.3, 0.2), 21, 0, 65536),
    ("dy1j_offset", 3, (1, 0), (50.0, ROOTS), (0.2, 0.6, 0.2), 22, (1 << 33) + 7, 4097),
    ("z_window", 4, (0, 2), (80.0, 100.0), (0.1, 0.9, 0.0), 23, 0, 10000),
    ("eight_photon", 8, (3, 6), (20.0, 2000.0), (0.3, 0.0, 0.7), 24, 5, 3001),
    ("flat_only", 5, (0, 1), (50.0, ROOTS), (1.0, 0.0, 0.0), 25, 0, 2048),
]


def kappa_of(nfinal, ch, seed, first, n):
    """The conformal map's enlargement of rounding, (Q0/M)^2, of the RAMBO
    stage each point went through: n bodies for the flat channel, n - 1 for
    the others (their first 4(n - 1) uniforms are the same)."""
    k_n = oracle.rambo(ROOTS, [0.0] * nfinal, seed, first, n, cond=True)[2]
    k_m = oracle.rambo(ROOTS, [0.0] * (nfinal - 1), seed, first, n, cond=True)[2]
    return np.where(ch == 0, k_n, k_m)


@pytest.mark.parametrize("name,nfinal,pair,window,alpha,seed,first,n", CASES)
def test_multichannel_matches_oracle(env, name, nfinal, pair, window, alpha, seed, first, n):
    """Channels bit for bit (the choice compares a uniform made from integers
    with the same normalised alphas on both sides); momenta component by
    component within (1e-13 + 4e-15 kappa) sqrt(s); weights within
    (1e-11 + 4e-15 kappa) (1 + gamma^2) relative, gamma^2 = P0^2/M^2 of the
    pair: its mass enters the Breit-Wigner density through P^2 = P0^2 - |P|^2,
    which loses that factor of relative precision when the pair is boosted."""
    torch, me = env
    print(f"[ps-mc] {name} n={n} first={first}", flush=True)
    mom, wt, ch = me.multichannel(ROOTS, nfinal, pair, window, MZ, WZ, alpha, seed, n, first_event=first)
    torch.cuda.synchronize()
    mom, wt, ch = mom.cpu().numpy(), wt.cpu().numpy(), ch.cpu().numpy()
    want_m, want_w, want_c, _ = oracle.ps_mc(ROOTS, nfinal, pair, window, MZ, WZ, alpha, seed, first, n)
    assert np.array_equal(ch, want_c)
    kappa = kappa_of(nfinal, want_c, seed, first, n)
    dev = np.abs(mom - want_m).max(axis=(1, 2)) / ROOTS
    ratio = dev / (1e-13 + 4e-15 * kappa)
    P = want_m[:, 2 + pair[0]] + want_m[:, 2 + pair[1]]
    gam2 = P[:, 0] ** 2 / mdot(P, P)
    rel_w = np.abs(wt / want_w - 1)
    ratio_w = rel_w / ((1e-11 + 4e-15 * kappa) * (1 + gam2))
    counts = np.bincount(ch, minlength=3)
    print(f"[ps-mc] {name}: channels {counts.tolist()}, max |dp|/sqrt(s) {dev.max():.2e} "
          f"(worst / bound {ratio.max():.2f}), weights max rel {rel_w.max():.2e} median {np.median(rel_w):.2e} "
          f"(worst / bound {ratio_w.max():.2f})", flush=True)
    assert ratio.max() < 1
    assert ratio_w.max() < 1


def test_multichannel_split_independent(env):
    """Event e of a call starting at `first` is event first + e of the stream."""
    torch, me = env
    a = me.multichannel(ROOTS, 5, (0, 1), (50.0, ROOTS), MZ, WZ, (0.4, 0.4, 0.2), 7, 1000)
    b = me.multichannel(ROOTS, 5, (0, 1), (50.0, ROOTS), MZ, WZ, (0.4, 0.4, 0.2), 7, 300, first_event=700)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x[700:], y)


def test_multichannel_full_size_properties(env):
    """2^20 points of the five-particle final state (the lepton pair and three
    partons), the size the sampler is timed at: every point conserves
    momentum and is massless; channel counts agree with alpha within 5
    binomial standard deviations; pairs made by the resonant channels lie in
    the window; a spread sample of events, each recomputed alone by the
    oracle, agrees with the GPU's."""
    torch, me = env
    n, nfinal, pair, window, alpha = 1 << 20, 5, (0, 1), (50.0, ROOTS), (0.5, 0.3, 0.2)
    print(f"[ps-mc] full size n={n}", flush=True)
    mom, wt, ch = me.multichannel(ROOTS, nfinal, pair, window, MZ, WZ, alpha, 31, n)
    torch.cuda.synchronize()
    fin = mom[:, 2:]
    tot = fin.sum(1) - mom[:, 0] - mom[:, 1]
    assert float(tot.abs().max()) < 1e-9 * ROOTS
    m2 = fin[..., 0] ** 2 - (fin[..., 1:] ** 2).sum(-1)
    assert float((m2.abs() / fin[..., 0] ** 2).max()) < 1e-12
    assert bool((wt > 0).all())
    counts = torch.bincount(ch.long(), minlength=3).cpu().numpy()
    for c in range(3):
        sd = np.sqrt(n * alpha[c] * (1 - alpha[c]))
        assert abs(counts[c] - n * alpha[c]) < 5 * sd
    P = fin[:, pair[0]] + fin[:, pair[1]]
    pm2 = (P[:, 0] ** 2 - (P[:, 1:] ** 2).sum(-1))[ch > 0]
    assert float(pm2.min()) >= window[0] ** 2 * (1 - 1e-9)
    assert float(pm2.max()) <= window[1] ** 2 * (1 + 1e-9)
    idx = np.unique(np.linspace(0, n - 1, 257).astype(np.int64))
    got_m = mom[idx].cpu().numpy()
    got_w = wt[idx].cpu().numpy()
    got_c = ch[idx].cpu().numpy()
    for j, e in enumerate(idx):
        wm, ww, wc, _ = oracle.ps_mc(ROOTS, nfinal, pair, window, MZ, WZ, alpha, 31, int(e), 1)
        assert got_c[j] == wc[0]
        assert np.abs(got_m[j] - wm[0]).max() < 1e-9 * ROOTS
        assert abs(got_w[j] / ww[0] - 1) < 1e-8
    print(f"[ps-mc] full size: channels {counts.tolist()}, {len(idx)} sampled events agree", flush=True)


def test_multichannel_rejects_bad_arguments(env):
    torch, me = env
    mom = torch.empty((4, 7, 4), dtype=torch.float64, device="cuda")
    for kw in [dict(pair=(0, 0)), dict(pair=(0, 5)), dict(window=(100.0, 50.0)), dict(alpha=(0.0, 0.0, 0.0)),
               dict(alpha=(-1.0, 1.0, 1.0)), dict(window=(0.0, 100.0))]:
        args = dict(pair=(0, 1), window=(50.0, ROOTS), alpha=(0.5, 0.3, 0.2))
        args.update(kw)
        with pytest.raises(me.MEError):
            me.ps_multichannel(ROOTS, 5, args["pair"], args["window"], MZ, WZ, args["alpha"], 1, 0, 4, mom)


def test_multichannel_then_matrix_element(env):
    """Multi-channel points made on the GPU feed me_eval of the DY+3j
    subprocess directly; w |M|^2 agrees with the oracle's sampler and matrix
    element on the same stream (points that fail the parton cuts included:
    the matrix element is finite there at these sizes)."""
    torch, me = env
    n, nfinal, pair, window, alpha = 512, 5, (0, 1), (50.0, ROOTS), (0.3, 0.4, 0.3)
    mom, wt, _ = me.multichannel(ROOTS, nfinal, pair, window, MZ, WZ, alpha, 41, n)
    m = me.MatrixElement("gux_taptamggux")  # its Z mass and width are MZ, WZ above
    got = (m.eval(mom) * wt).cpu().numpy()
    torch.cuda.synchronize()
    m.close()
    pts, w, _, _ = oracle.ps_mc(ROOTS, nfinal, pair, window, MZ, WZ, alpha, 41, 0, n)
    want = oracle.me2("gux_taptamggux", pts) * w
    rel = np.abs(got / want - 1)
    print(f"[ps-mc] gux_taptamggux w |M|^2 on GPU-made points: max rel {rel.max():.2e}", flush=True)
    assert rel.max() < 1e-10
