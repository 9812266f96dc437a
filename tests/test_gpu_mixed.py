"""The mixed-precision form against the float64 oracle (run on an MI355X).

The mixed form computes amplitudes in float32 and the colour sum as a float16
hi/lo GEMM on the matrix cores; events whose estimated relative error exceeds
the tolerance are recomputed in float64.  The bar: after the rerun every
event is within the tolerance of the oracle (1e-5 here, the stated
tolerance of the form).
"""
import numpy as np
import pytest

import oracle
from inputs import process_points

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def me_mod(torch_cuda):
    import paper_2503_21935_amd as me

    me.lib()
    return me


# g g -> t tbar g g g: the oracle's 2^12 events are shared with the float64 parity test
@pytest.mark.parametrize("proc,n,seed", [("gg_tt", 65536, 1), ("gg_ttg", 8192, 7), ("gg_ttgg", 1 << 16, 2),
                                         ("gg_ttggg", 1 << 12, 3)])
def test_mixed_within_tolerance(me_mod, torch_cuda, oracle_points, proc, n, seed):
    torch = torch_cuda
    print(f"[mixed] {proc} n={n} seed={seed}", flush=True)
    mom, want = oracle_points(proc, n, seed)
    m = me_mod.MatrixElement(proc)
    m.set_precision(me_mod.ME_MIXED, TOL)
    t = torch.from_numpy(mom).cuda()
    got = m.eval(t)
    torch.cuda.synchronize()
    nfb = m.fallback_count()
    raw, est, flag = m.eval_mixed_diag(t)
    torch.cuda.synchronize()
    got, raw, est, flag = got.cpu().numpy(), raw.cpu().numpy(), est.cpu().numpy(), flag.cpu().numpy()
    rel = np.abs(got / want - 1)
    rel_raw = np.abs(raw / want - 1)
    print(f"[mixed] {proc}: fallback {nfb}/{n}; float32-form error p50 {np.median(rel_raw):.2e} "
          f"p99.9 {np.quantile(rel_raw, 0.999):.2e} max {rel_raw.max():.2e}; after rerun max {rel.max():.2e}",
          flush=True)
    assert nfb == int(flag.sum())
    assert np.all(np.isfinite(got))
    assert rel.max() <= TOL
    # The estimate is calibrated, not a bound: on these sets it lies above the
    # float32-form error of every event it lets through, except for a tail
    # measured on the 2^16 g g -> t tbar g g events (2 of 57,695 unflagged
    # events, error up to 2.0 x the estimate, both below the tolerance).  The
    # hard bar is the one above: every returned value within the tolerance.
    ok = flag == 0
    ratio = rel_raw[ok] / np.maximum(est[ok], 1e-300)
    miss = ratio > 1
    print(f"[mixed] {proc}: largest error / estimate over unflagged events {ratio.max():.2f}; "
          f"{int(miss.sum())} of {int(ok.sum())} unflagged events above their estimate", flush=True)
    assert miss.sum() <= max(2, 1e-4 * ok.sum()), "estimate below the actual error too often"
    assert np.all(rel_raw[ok][miss] <= TOL), "an event above its estimate is also above the tolerance"
    if proc == "gg_ttggg":
        assert not miss.any(), "g g -> t tbar g g g: estimate below the actual error"
    m.close()


def test_forced_fallback_is_float64(me_mod, torch_cuda):
    """A tolerance below float32 resolution sends every event to the float64 rerun."""
    torch = torch_cuda
    mom = process_points("gg_ttgg", 1000, 9)
    m = me_mod.MatrixElement("gg_ttgg")
    m.set_helicity_lanes(1)  # the rerun's float64 kernel takes one lane per event
    t = torch.from_numpy(mom).cuda()
    ref = m.eval(t).clone()
    m.set_precision(me_mod.ME_MIXED, 1e-14)
    got = m.eval(t)
    torch.cuda.synchronize()
    assert m.fallback_count() == 1000
    assert torch.equal(got, ref)
    m.close()


def test_forced_fallback_workgroup_kernel(me_mod, torch_cuda):
    """The same for the workgroup kernel of g g -> t tbar g g g: the rerun goes
    through the float64 kernel's index form.  Its LDS sums are atomic, so the
    two float64 evaluations agree to rounding, not bit for bit."""
    torch = torch_cuda
    mom = process_points("gg_ttggg", 100, 9)
    m = me_mod.MatrixElement("gg_ttggg")
    m.set_helicity_lanes(1)
    t = torch.from_numpy(mom).cuda()
    ref = m.eval(t).clone()
    m.set_precision(me_mod.ME_MIXED, 1e-14)
    got = m.eval(t)
    torch.cuda.synchronize()
    assert m.fallback_count() == 100
    torch.testing.assert_close(got, ref, rtol=1e-13, atol=0)
    m.close()


def test_mixed_ragged_workgroup_kernel(me_mod, torch_cuda):
    """Partial tiles of the workgroup kernel's mixed form, and repeated calls."""
    torch = torch_cuda
    m = me_mod.MatrixElement("gg_ttggg")
    m.set_precision(me_mod.ME_MIXED, TOL)
    for n, seed in ((65, 3), (1, 4)):
        mom = process_points("gg_ttggg", n, seed)
        got = m.eval(torch.from_numpy(mom).cuda()).cpu().numpy()
        want = oracle.me2("gg_ttggg", mom)
        assert np.abs(got / want - 1).max() <= TOL
    m.close()


def test_mixed_ragged_and_repeated(me_mod, torch_cuda):
    """Partial last wave, and a smaller second call reusing the grown scratch."""
    torch = torch_cuda
    m = me_mod.MatrixElement("gg_ttgg")
    m.set_precision(me_mod.ME_MIXED, TOL)
    for n, seed in ((1000, 3), (77, 4), (1, 5)):
        mom = process_points("gg_ttgg", n, seed)
        got = m.eval(torch.from_numpy(mom).cuda()).cpu().numpy()
        want = oracle.me2("gg_ttgg", mom)
        assert np.abs(got / want - 1).max() <= TOL
    m.close()


def test_mixed_full_size_sampled(me_mod, torch_cuda):
    """2^20 gg -> t tbar g g points in one mixed launch; a seeded sample vs the oracle."""
    torch = torch_cuda
    n = 1 << 20
    mom = process_points("gg_ttgg", n, 2)
    m = me_mod.MatrixElement("gg_ttgg")
    m.set_precision(me_mod.ME_MIXED, TOL)
    got = m.eval(torch.from_numpy(mom).cuda()).cpu().numpy()
    nfb = m.fallback_count()
    idx = np.sort(np.random.default_rng(1).choice(n, 1024, replace=False))
    rel = np.abs(got[idx] / oracle.me2("gg_ttgg", mom[idx]) - 1)
    print(f"[mixed] 2^20 gg_ttgg: fallback {nfb} ({nfb / n:.2%}); sample max {rel.max():.2e}", flush=True)
    assert rel.max() <= TOL
    assert np.all(np.isfinite(got)) and np.all(got > 0)
    m.close()


def test_mixed_mode_ee_stays_float64(me_mod, torch_cuda):
    torch = torch_cuda
    mom = process_points("ee_mumu", 256, 0)
    m = me_mod.MatrixElement("ee_mumu")
    m.set_precision(me_mod.ME_MIXED, TOL)
    got = m.eval(torch.from_numpy(mom).cuda()).cpu().numpy()
    np.testing.assert_allclose(got, oracle.me2("ee_mumu", mom), rtol=1e-12)
    with pytest.raises(me_mod.MEError) as e:
        m.eval_mixed_diag(torch.from_numpy(mom).cuda())
    assert e.value.status == me_mod.ME_ESTATE
    m.close()
