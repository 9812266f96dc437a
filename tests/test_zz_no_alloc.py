"""The allocation-free mixed evaluation (me_eval_mixed_noalloc) against me_eval
in the mixed form, through the C ABI, on two calls in a row (the second
smaller), plus its size limit."""
import numpy as np
import pytest

import oracle
from inputs import process_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_21935_amd as me

    me.lib()
    return torch, me


@pytest.mark.parametrize("proc,sizes", [("gg_ttgg", (4096, 1000)), ("gg_ttggg", (200, 70)), ("ee_mumu", (512, 33))])
def test_noalloc_matches_me_eval(env, proc, sizes):
    torch, me = env
    tol = 1e-5
    m = me.MatrixElement(proc)
    m.set_precision(me.ME_MIXED, tol)
    mom_all = process_points(proc, sizes[0], 11)
    for n in sizes:  # the second call is smaller: the shared scratch keeps the first call's contents
        print(f"[noalloc] {proc} n={n}", flush=True)
        mom_np = mom_all[:n]
        mom = torch.from_numpy(mom_np).cuda()
        want = torch.empty(n, dtype=torch.float64, device="cuda")
        me.me_eval(m.ctx, mom, n, want)
        got = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        me.me_eval_mixed_noalloc(m.ctx, mom, n, got)
        torch.cuda.synchronize()
        got, want = got.cpu().numpy(), want.cpu().numpy()
        if proc == "gg_ttggg":
            # the float32 workgroup kernel adds four waves' contributions with LDS
            # atomics, so unflagged events differ from call to call at float32
            # rounding; each call is within the tolerance of the exact value
            np.testing.assert_allclose(got, want, rtol=2 * tol, atol=0)
        else:
            assert np.array_equal(got, want)
        sel = np.arange(0, n, max(1, n // 16))
        ref = oracle.me2(proc, mom_np[sel])
        assert np.max(np.abs(got[sel] / ref - 1)) < tol
    m.close()


def test_noalloc_size_limit(env):
    torch, me = env
    m = me.MatrixElement("gg_tt")
    m.set_precision(me.ME_MIXED, 1e-5)
    lim = 1 << 20
    # buffers large enough for lim + 1 events: the library itself must refuse the size
    mom = torch.zeros((lim + 1, 4, 4), dtype=torch.float64, device="cuda")
    out = torch.empty(lim + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(me.MEError) as e:
        me.me_eval_mixed_noalloc(m.ctx, mom, lim + 1, out)  # rejected on the host before any launch
    assert e.value.status == me.ME_EINVAL
    me.me_eval_mixed_noalloc(m.ctx, mom, 0, out)  # nevt == 0 launches nothing
    # the largest accepted size runs (zero momenta give NaN, which the mixed form flags for the rerun)
    mom_np = process_points("gg_tt", lim, 1, precise=False)
    mom = torch.from_numpy(mom_np).cuda()
    out = out[:lim]
    me.me_eval_mixed_noalloc(m.ctx, mom, lim, out)
    want = torch.empty(lim, dtype=torch.float64, device="cuda")
    me.me_eval(m.ctx, mom, lim, want)
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    m.close()
