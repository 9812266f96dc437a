"""GPU phase-space sampling (ps_rambo: Philox4x32-10 + RAMBO on the GPU)
against the CPU oracle on the same counter-based random streams."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_21935_amd as me

    me.lib()
    return torch, me


CASES = [
    ("ee_mumu", 500.0, [0.0, 0.0], 0, 0, 16384),
    ("gg_tt", 13000.0, [173.0, 173.0], 1, 0, 4097),
    ("gg_ttgg", 13000.0, [173.0, 173.0, 0.0, 0.0], 2, 0, 65536),
    ("gg_ttgg_offset", 13000.0, [173.0, 173.0, 0.0, 0.0], 2, (1 << 33) + 12345, 1000),
    ("gg_ttggg", 13000.0, [173.0, 173.0, 0.0, 0.0, 0.0], 3, 0, 3001),
    ("eight_massive", 2000.0, [10.0 * i for i in range(8)], 9, 77, 513),
]


@pytest.mark.parametrize("name,roots,masses,seed,first,n", CASES)
def test_rambo_matches_oracle(env, name, roots, masses, seed, first, n):
    """Component by component within (1e-14 + 4e-15 kappa) sqrt(s), weights
    within (1e-13 + 4e-15 kappa) relative, where kappa = (Q0/M)^2 is the
    oracle's per-event enlargement of rounding by the conformal map (the
    generated q's of nearly collinear events have a small invariant mass M):
    libm's and the GPU's log and sincos differ in the last bits, and both
    sides then follow the same map."""
    torch, me = env
    print(f"[ps] {name} n={n} first={first}", flush=True)
    mom, wt = me.rambo(roots, masses, seed, n, first_event=first)
    torch.cuda.synchronize()
    mom, wt = mom.cpu().numpy(), wt.cpu().numpy()
    want_m, want_w, kappa = oracle.rambo(roots, masses, seed, first, n, cond=True)
    dev = np.abs(mom - want_m).max(axis=(1, 2)) / roots
    ratio = dev / (1e-14 + 4e-15 * kappa)
    print(f"[ps] {name}: max |dp|/sqrt(s) {dev.max():.2e}, median {np.median(dev):.2e}, "
          f"max kappa {kappa.max():.1e}, worst dev / bound {ratio.max():.2f}", flush=True)
    assert ratio.max() < 1
    rel_w = np.abs(wt / want_w - 1)
    assert np.all(rel_w < 1e-13 + 4e-15 * kappa)


def test_rambo_split_independent(env):
    """Event e of a call starting at `first` is event first + e of the stream:
    a sample made in two calls equals the sample made in one (bit for bit)."""
    torch, me = env
    masses = [173.0, 173.0, 0.0, 0.0]
    a, wa = me.rambo(13000.0, masses, 5, 1000)
    b, wb = me.rambo(13000.0, masses, 5, 400, first_event=600)
    torch.cuda.synchronize()
    assert torch.equal(a[600:], b) and torch.equal(wa[600:], wb)


def test_rambo_then_matrix_element(env):
    """Points made on the GPU feed me_eval directly; |M|^2 agrees with the
    oracle evaluated on the oracle's own points of the same stream."""
    torch, me = env
    masses = [173.0, 173.0, 0.0, 0.0]
    mom, _ = me.rambo(13000.0, masses, 2, 512)
    m = me.MatrixElement("gg_ttgg")
    got = m.eval(mom)
    torch.cuda.synchronize()
    pts, _ = oracle.rambo(13000.0, masses, 2, 0, 512)
    want = oracle.me2("gg_ttgg", pts)
    rel = np.abs(got.cpu().numpy() / want - 1)
    print(f"[ps] gg_ttgg |M|^2 on GPU-made points: max rel {rel.max():.2e}", flush=True)
    # the points themselves differ by ~1e-16 sqrt(s); |M|^2 is smooth in them
    assert rel.max() < 1e-9
    m.close()


def test_rambo_errors(env):
    torch, me = env
    out = torch.empty((8, 4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(me.MEError):
        me.ps_rambo(100.0, [60.0, 60.0], 1, 0, 8, out)  # masses above sqrt(s)
    with pytest.raises(me.MEError):
        me.ps_rambo(100.0, [0.0], 1, 0, 8, torch.empty((8, 3, 4), dtype=torch.float64, device="cuda"))
    me.ps_rambo(100.0, [0.0, 0.0], 1, 0, 0, out)  # nevt == 0: nothing
