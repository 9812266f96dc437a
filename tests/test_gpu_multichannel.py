"""The multi-channel form (single-diagram weights) against the oracle's
explicit single diagrams (route 4), through the C ABI."""
import numpy as np
import pytest

import oracle
from inputs import process_points
from test_gpu_parity import check_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_21935_amd as me

    me.lib()
    return torch, me


@pytest.mark.parametrize("proc,n,seed", [("gg_tt", 1000, 31), ("gg_ttg", 200, 32), ("gg_ttgg", 67, 33)])
def test_channel_weights_match_oracle(env, proc, n, seed):
    """Every event's |M|^2 (the float64 parity bar) and its weight in every
    channel (1e-10 relative: a ratio of sums of squares, as well conditioned as
    the amplitudes themselves): the GPU channels are matched to the oracle's
    diagrams by their descriptors, and each event is evaluated once per channel."""
    torch, me = env
    print(f"[mc] {proc} n={n}", flush=True)
    mom = process_points(proc, n, seed)
    m = me.MatrixElement(proc)
    descs = m.channels()
    odescs, sums = oracle.diagram_sums(proc, mom)
    assert sorted(descs) == sorted(odescs) and len(descs) == len(odescs)
    col = {d: i for i, d in enumerate(odescs)}
    want_alpha = sums / sums.sum(axis=1, keepdims=True)
    want_me2 = oracle.me2(proc, mom)
    t = torch.from_numpy(mom).cuda()
    worst = 0.0
    for c, d in enumerate(descs):
        chan = torch.full((n,), c, dtype=torch.int32, device="cuda")
        me2, alpha = m.eval_multichannel(t, chan)
        torch.cuda.synchronize()
        me2, alpha = me2.cpu().numpy(), alpha.cpu().numpy()
        if c == 0:
            check_parity(proc, mom, me2, want=want_me2)
        ref = want_alpha[:, col[d]]
        dev = np.abs(alpha - ref) / ref
        worst = max(worst, float(dev.max()))
        assert np.all(dev <= 1e-10), (d, float(dev.max()))
    print(f"[mc] {proc}: {len(descs)} channels, worst relative alpha deviation {worst:.2e}", flush=True)
    m.close()


def test_mixed_channels_in_one_launch(env):
    """Events of different channels in one launch (the paper's case): each gets
    its own channel's weight, a channel id outside the table gives 0, and the
    weights of all channels of an event add up to 1."""
    torch, me = env
    n = 777
    mom = process_points("gg_ttgg", n, 34)
    m = me.MatrixElement("gg_ttgg")
    nchan = len(m.channels())
    rng = np.random.default_rng(34)
    chan = rng.integers(-1, nchan + 1, size=n).astype(np.int32)
    t = torch.from_numpy(mom).cuda()
    me2, alpha = m.eval_multichannel(t, torch.from_numpy(chan).cuda())
    total = torch.zeros(n, dtype=torch.float64, device="cuda")
    for c in range(nchan):
        _, a = m.eval_multichannel(t, torch.full((n,), c, dtype=torch.int32, device="cuda"))
        total += a
        sel = torch.from_numpy(chan == c).cuda()
        assert torch.equal(alpha[sel], a[sel])
    torch.cuda.synchronize()
    outside = (chan < 0) | (chan >= nchan)
    assert np.all(alpha.cpu().numpy()[outside] == 0.0)
    np.testing.assert_allclose(total.cpu().numpy(), 1.0, rtol=1e-12)
    check_parity("gg_ttgg", mom, me2.cpu().numpy())
    m.close()


def test_no_multichannel_form(env):
    torch, me = env
    m = me.MatrixElement("gg_ttggg")
    assert m.channels() == []
    mom = torch.from_numpy(process_points("gg_ttggg", 4, 1)).cuda()
    with pytest.raises(me.MEError) as e:
        m.eval_multichannel(mom, torch.zeros(4, dtype=torch.int32, device="cuda"))
    assert e.value.status == me.ME_ESTATE
    m.close()
