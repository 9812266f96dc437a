"""The surrogate network's HIP kernels and the two-stage unweighting (MI355X).

Forward and backward are compared with the float64 CPU reference run on the
same BF16-rounded weights and inputs, rounding the activations (and, in the
backward pass, the pre-activation gradients) to BF16 where the kernels store
them; Adam is compared with its closed form; unweighting decisions with the
CPU reference of the algorithm on the same uniforms.
"""
import numpy as np
import pytest

import oracle
from inputs import process_points, uniforms
from oracle import mlp_ref as R

pytestmark = pytest.mark.gpu


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


def emulated_forward(theta, x, keep=False):
    """Float64 forward with BF16 weights, inputs and stored activations."""
    layers, w_out, b_out = R.unpack(theta)
    h = R.bf16_round(x)
    zs, hs = [], [h]
    for W, b in layers:
        z = h @ R.bf16_round(W).T + b
        h = R.bf16_round(R.silu(z))
        zs.append(z)
        hs.append(h)
    y = h @ w_out + b_out[0]
    return (y, zs, hs) if keep else y


def emulated_grad(theta, x, t, magnitudes=False):
    """Gradient with the kernels' BF16 roundings; with magnitudes=True also the
    sums of |terms| behind every entry (the scale of its rounding error)."""
    y, zs, hs = emulated_forward(theta, x, keep=True)
    layers, w_out, _ = R.unpack(theta)
    m = len(t)
    dy = 2 * (y - t) / m
    g_layers, a_layers = [None] * len(layers), [None] * len(layers)
    g_wout = hs[-1].T @ dy
    a_wout = np.abs(hs[-1]).T @ np.abs(dy)
    g_bout = np.array([dy.sum()])
    a_bout = np.array([np.abs(dy).sum()])
    dz = R.bf16_round(np.outer(dy, w_out) * R.silu_prime(zs[-1]))
    for l in range(len(layers) - 1, -1, -1):
        g_layers[l] = (dz.T @ hs[l], dz.sum(axis=0))
        a_layers[l] = (np.abs(dz).T @ np.abs(hs[l]), np.abs(dz).sum(axis=0))
        if l > 0:
            dz = R.bf16_round((dz @ R.bf16_round(layers[l][0])) * R.silu_prime(zs[l - 1]))
    parts, amag = [], []
    for (gW, gb), (aW, ab) in zip(g_layers, a_layers):
        parts += [gW.ravel(), gb]
        amag += [aW.ravel(), ab]
    g = np.concatenate(parts + [g_wout, g_bout])
    if magnitudes:
        return g, np.concatenate(amag + [a_wout, a_bout])
    return g


def features_np(mom):
    s = (mom[:, 0, 0] + mom[:, 1, 0]) ** 2 - ((mom[:, 0, 1:] + mom[:, 1, 1:]) ** 2).sum(-1)
    return (mom.reshape(len(mom), -1) / np.sqrt(s)[:, None]).astype(np.float32)


def test_features(me_mod, torch_cuda):
    torch = torch_cuda
    mom = process_points("gg_ttgg", 1000, 4)
    x = me_mod.features(torch.from_numpy(mom).cuda()).cpu().numpy()
    np.testing.assert_allclose(x, features_np(mom), rtol=1e-7)


def test_forward_matches_reference(me_mod, torch_cuda):
    torch = torch_cuda
    net = me_mod.Surrogate(seed=11)
    theta = net.get_params().astype(np.float64)
    x = features_np(process_points("gg_ttgg", 3000, 4))  # not a multiple of 64
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    emu = emulated_forward(theta, x.astype(np.float64))
    exact = R.forward(theta, x.astype(np.float64))
    rel_emu = np.linalg.norm(y - emu) / np.linalg.norm(emu)
    rel_exact = np.linalg.norm(y - exact) / np.linalg.norm(exact)
    print(f"[mlp] forward: vs BF16-emulating reference {rel_emu:.2e}, vs float64 {rel_exact:.2e}", flush=True)
    assert rel_emu < 2e-3
    assert rel_exact < 3e-2
    net.close()


def test_backward_matches_reference(me_mod, torch_cuda):
    torch = torch_cuda
    net = me_mod.Surrogate(seed=12)
    theta = net.get_params().astype(np.float64)
    x = features_np(process_points("gg_ttgg", 512, 5))
    t = np.random.default_rng(3).normal(size=512).astype(np.float32)
    g, loss = net.backward(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = g.cpu().numpy().astype(np.float64)
    ge = emulated_grad(theta, x.astype(np.float64), t.astype(np.float64))
    lref, gx = R.loss_and_grad(theta, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss.item() / lref - 1) < 1e-2
    # per parameter tensor, norm-wise
    n_in, W = 24, 256
    offs = [0]
    for fi in (n_in, W, W, W):
        offs += [offs[-1] + W * fi, offs[-1] + W * fi + W]
    offs += [offs[-1] + W, offs[-1] + W + 1]
    worst = 0.0
    for a, b in zip(offs[:-1], offs[1:]):
        rel = np.linalg.norm(g[a:b] - ge[a:b]) / max(np.linalg.norm(ge[a:b]), 1e-30)
        rel_x = np.linalg.norm(g[a:b] - gx[a:b]) / max(np.linalg.norm(gx[a:b]), 1e-30)
        worst = max(worst, rel)
        assert rel < 1e-2, (a, b, rel)
        assert rel_x < 5e-2, (a, b, rel_x)
    print(f"[mlp] backward: worst tensor vs BF16-emulating reference {worst:.2e}", flush=True)
    net.close()


def test_forward_elementwise(me_mod, torch_cuda):
    """Every sample's output against the BF16-emulating reference, within 2^-6
    of the sum of the magnitudes of the output layer's terms for that sample
    (a flipped BF16 rounding of an activation moves it by at most 2^-8 of
    itself; a wrong row or column of any layer moves whole outputs by O(1))."""
    torch = torch_cuda
    net = me_mod.Surrogate(seed=16)
    theta = net.get_params().astype(np.float64)
    x = features_np(process_points("gg_ttgg", 2111, 4))
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    emu, zs, hs = emulated_forward(theta, x.astype(np.float64), keep=True)
    _, w_out, b_out = R.unpack(theta)
    scale = np.abs(hs[-1]) @ np.abs(w_out) + abs(b_out[0])
    ratio = np.abs(y - emu) / scale
    print(f"[mlp] forward per sample: max |y - emu| / scale {ratio.max():.2e}, median {np.median(ratio):.2e}",
          flush=True)
    assert ratio.max() < 2.0 ** -6
    net.close()


def test_backward_elementwise(me_mod, torch_cuda):
    """Every gradient entry against the BF16-emulating reference, within 2^-5 of
    the sum of the magnitudes of the batch terms that make up that entry."""
    torch = torch_cuda
    net = me_mod.Surrogate(seed=17)
    theta = net.get_params().astype(np.float64)
    x = features_np(process_points("gg_ttgg", 1024, 9))
    t = np.random.default_rng(9).normal(size=1024).astype(np.float32)
    g, _ = net.backward(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = g.cpu().numpy().astype(np.float64)
    ge, mag = emulated_grad(theta, x.astype(np.float64), t.astype(np.float64), magnitudes=True)
    ratio = np.abs(g - ge) / np.maximum(mag, 1e-30)
    worst = int(np.argmax(ratio))
    print(f"[mlp] backward per entry: max |g - emu| / magnitude {ratio.max():.2e} (entry {worst}), "
          f"median {np.median(ratio):.2e}", flush=True)
    assert ratio.max() < 2.0 ** -5
    net.close()


def test_adam_three_steps(me_mod, torch_cuda):
    """Three consecutive training steps on a fixed batch against the CPU Adam
    fed the same gradients (taken from the GPU's own backward pass at each
    step): exercises the step counter and the bias correction beyond t = 1."""
    torch = torch_cuda
    net = me_mod.Surrogate(seed=18)
    theta = net.get_params().astype(np.float64)
    x = torch.from_numpy(features_np(process_points("gg_ttgg", 512, 10))).cuda()
    t = torch.from_numpy(np.random.default_rng(10).normal(size=512).astype(np.float32)).cuda()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    lrs = [1e-3, 7e-4, 4e-4]
    for step, lr in enumerate(lrs, start=1):
        g, _ = net.backward(x, t)  # the gradient train_step computes at the current weights
        g = g.cpu().numpy().astype(np.float64)
        net.train_step(x, t, None, lr)
        torch.cuda.synchronize()
        theta, m, v = R.adam_step(theta, m, v, g, step, lr)
        got = net.get_params().astype(np.float64)
        # float32 master weights: the update itself is computed to ~1e-7 of lr
        np.testing.assert_allclose(got, theta, rtol=0, atol=2e-6 * lr + 2e-7, err_msg=f"step {step}")
        theta = got  # continue from the GPU's float32 weights
    net.close()


def test_fused_step_matches_layered(me_mod, torch_cuda):
    """The one-kernel training step (cooperative, grid-wide barriers) against the
    layered GEMM path: every gradient entry within 2^-6 of the magnitude sum
    behind it, the loss to 1e-5, and three Adam steps to the same weights."""
    torch = torch_cuda
    x = torch.from_numpy(features_np(process_points("gg_ttgg", 2048, 12))).cuda()
    t = torch.from_numpy(np.random.default_rng(12).normal(size=2048).astype(np.float32)).cuda()
    nets = [me_mod.Surrogate(seed=19), me_mod.Surrogate(seed=19)]
    nets[1].set_fused_step(False)
    theta = nets[0].get_params().astype(np.float64)
    (gf, lf), (gl, ll) = [n.backward(x, t) for n in nets]
    gf, gl = gf.cpu().numpy().astype(np.float64), gl.cpu().numpy().astype(np.float64)
    _, mag = emulated_grad(theta, features_np(process_points("gg_ttgg", 2048, 12)).astype(np.float64),
                           t.cpu().numpy().astype(np.float64), magnitudes=True)
    ratio = np.abs(gf - gl) / np.maximum(mag, 1e-30)
    print(f"[mlp] fused vs layered gradient: max |diff| / magnitude {ratio.max():.2e}", flush=True)
    assert ratio.max() < 2.0 ** -6
    assert abs(lf.item() / ll.item() - 1) < 1e-5
    perm = torch.from_numpy(np.random.default_rng(13).permutation(2048)[:1024].astype(np.int32)).cuda()
    for lr in (1e-3, 7e-4, 4e-4):
        for n in nets:
            n.train_step(x, t, perm, lr)
    torch.cuda.synchronize()
    pf, pl = nets[0].get_params(), nets[1].get_params()
    # Adam moves each weight by about lr sign(g): entries whose batch sum is
    # rounding noise may move either way, every other one moves alike
    d = np.abs(pf.astype(np.float64) - pl)
    print(f"[mlp] fused vs layered after 3 steps: p99 {np.quantile(d, 0.99):.2e}, p99.9 {np.quantile(d, 0.999):.2e}, "
          f"max {d.max():.2e}", flush=True)
    assert np.quantile(d, 0.99) < 1e-5
    assert d.max() <= 2 * (1e-3 + 7e-4 + 4e-4)
    for n in nets:
        n.close()


def test_train_steps_one_launch(me_mod, torch_cuda):
    """Several Adam steps in one call (one cooperative launch) against the same
    steps taken one call at a time: per-step losses and final weights agree (the
    bias corrections are computed on the device there, on the host here), both
    with an index list and with consecutive row blocks (idx None)."""
    torch = torch_cuda
    n, nsteps = 512, 4
    x = torch.from_numpy(features_np(process_points("gg_ttgg", n * nsteps, 21))).cuda()
    t = torch.from_numpy(np.random.default_rng(21).normal(size=n * nsteps).astype(np.float32)).cuda()
    lrs = [1e-3, 8e-4, 6e-4, 3e-4]
    lr_dev = torch.tensor(lrs, dtype=torch.float32, device="cuda")
    idx = torch.from_numpy(np.random.default_rng(22).permutation(n * nsteps).astype(np.int32)).cuda()
    for use_idx in (True, False):
        a, b = me_mod.Surrogate(seed=23), me_mod.Surrogate(seed=23)
        la = torch.zeros(nsteps, dtype=torch.float32, device="cuda")
        lb = torch.zeros(nsteps, dtype=torch.float32, device="cuda")
        a.train_steps(x, t, idx if use_idx else None, n, lr_dev, la)
        for s_ in range(nsteps):
            if use_idx:
                b.train_step(x, t, idx[s_ * n:(s_ + 1) * n], lrs[s_], lb[s_:s_ + 1])
            else:
                b.train_step(x[s_ * n:(s_ + 1) * n], t[s_ * n:(s_ + 1) * n], None, lrs[s_], lb[s_:s_ + 1])
        torch.cuda.synchronize()
        pa, pb = a.get_params().astype(np.float64), b.get_params().astype(np.float64)
        d = np.abs(pa - pb)
        la, lb = la.cpu().numpy(), lb.cpu().numpy()
        print(f"[mlp] {nsteps} steps in one launch (idx {use_idx}): max |dw| {d.max():.2e}, "
              f"losses {la} vs {lb}", flush=True)
        np.testing.assert_allclose(la, lb, rtol=1e-5)
        assert d.max() <= 1e-6
        a.close()
        b.close()


def test_adam_step(me_mod, torch_cuda):
    torch = torch_cuda
    net = me_mod.Surrogate(seed=13)
    theta = net.get_params()
    x = torch.from_numpy(features_np(process_points("gg_ttgg", 256, 6))).cuda()
    t = torch.from_numpy(np.random.default_rng(4).normal(size=256).astype(np.float32)).cuda()
    g, _ = net.backward(x, t)
    g = g.cpu().numpy().astype(np.float64)
    lr = 1e-3
    net.train_step(x, t, None, lr)
    torch.cuda.synchronize()
    new = net.get_params().astype(np.float64)
    want, _, _ = R.adam_step(theta.astype(np.float64), 0.0, 0.0, g, 1, lr)
    np.testing.assert_allclose(new, want, rtol=0, atol=2e-6 * lr + 1e-7)
    net.close()


def test_training_learns_log_me2(me_mod, torch_cuda):
    """A short training run on oracle-labelled gg -> t tbar g g points lowers the loss."""
    torch = torch_cuda
    n = 1 << 14
    mom = process_points("gg_ttgg", n, 4)
    lab = np.log(oracle.me2("gg_ttgg", mom))
    mu, sig = lab.mean(), lab.std()
    t = torch.from_numpy(((lab - mu) / sig).astype(np.float32)).cuda()
    x = me_mod.features(torch.from_numpy(mom).cuda())
    net = me_mod.Surrogate(seed=14)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(5)
    first = None
    for epoch in range(6):
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).cuda()
        for b in range(0, n, 512):
            net.train_step(x, t, perm[b:b + 512], 1e-3, loss)
            if first is None:
                torch.cuda.synchronize()
                first = loss.item()
    y = net.forward(x)
    mse = torch.mean((y - t) ** 2).item()
    print(f"[mlp] training: first batch loss {first:.3f}, after 6 epochs mse {mse:.3f}", flush=True)
    assert mse < 0.5 * first
    net.close()


def test_unweighting_matches_reference(me_mod, torch_cuda):
    torch = torch_cuda
    n = 8192
    mom, w_ps = process_points("gg_ttgg", n, 5, return_weight=True)
    u = uniforms(n, 2, 55)
    me2 = oracle.me2("gg_ttgg", mom)
    lab = np.log(me2)
    mu, sig = float(lab.mean()), float(lab.std())
    ctx = me_mod.MatrixElement("gg_ttgg")
    net = me_mod.Surrogate(seed=15)
    tm = torch.from_numpy(mom).cuda()
    y = net.forward(me_mod.features(tm)).cpu().numpy().astype(np.float64)
    s = np.exp(sig * y + mu) * w_ps
    w = me2 * w_ps
    s_max = float(np.quantile(s, 0.7))
    r_max = float(np.quantile(w / s, 0.7))
    out_idx = torch.empty(n, dtype=torch.int32, device="cuda")
    out_w = torch.empty(n, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    me_mod.unweight_two_stage(ctx.ctx, net.h, tm, torch.from_numpy(w_ps).cuda(), n, torch.from_numpy(u).cuda(),
                              mu, sig, s_max, r_max, out_idx, out_w, cnt)
    torch.cuda.synchronize()
    n1, n2 = cnt.cpu().numpy().tolist()
    got_idx = out_idx[:n2].cpu().numpy()
    got_w = out_w[:n2].cpu().numpy()
    order = np.argsort(got_idx)
    got_idx, got_w = got_idx[order], got_w[order]
    acc1, acc2, wt = R.two_stage(s, w, u[:, 0], u[:, 1], s_max, r_max)
    assert n1 == int(acc1.sum())
    assert np.array_equal(got_idx, np.nonzero(acc2)[0])
    np.testing.assert_allclose(got_w, wt[acc2], rtol=1e-9)
    print(f"[unweight] {n} points: stage 1 kept {n1}, accepted {n2}", flush=True)
    ctx.close()
    net.close()


def test_surrogate_gain_and_unbiasedness(me_mod, torch_cuda):
    """What the trained network gains: on g g -> t tbar g g points (generator
    cuts as in the benchmark) the two-stage unweighting needs several times
    fewer exact matrix elements per effective unweighted event than
    unweighting with the exact matrix element alone, and its estimate of the
    mean weight stays unbiased (within 5 standard deviations computed from each
    point's exact acceptance probability and output weight)."""
    import math

    from inputs import gluon_cuts

    torch = torch_cuda
    dev = torch.device("cuda")
    ctx = me_mod.MatrixElement("gg_ttgg")
    # training set labelled by the float64 GPU kernel
    mom_tr = process_points("gg_ttgg", 1 << 17, 4, precise=False)
    mom_tr = mom_tr[gluon_cuts(mom_tr)]
    mt = torch.from_numpy(mom_tr).to(dev)
    lab = torch.log(ctx.eval(mt))
    mu, sig = float(lab.mean()), float(lab.std())
    t = ((lab - mu) / sig).float()
    x = me_mod.features(mt)
    net = me_mod.Surrogate(seed=21)
    rng = np.random.default_rng(8)
    n = (len(t) // 4096) * 4096
    steps = 0
    total = 6 * (n // 4096)
    for _ in range(6):
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(dev)
        for b in range(n // 4096):
            lr = 0.5e-3 * (1 + math.cos(math.pi * steps / total))
            net.train_step(x, t, perm[b * 4096:(b + 1) * 4096], lr)
            steps += 1
    # maxima from an independent calibration sample
    mom_c, w_c = process_points("gg_ttgg", 1 << 17, 6, return_weight=True, precise=False)
    w_c = w_c * gluon_cuts(mom_c)
    mc = torch.from_numpy(mom_c).to(dev)
    s_c = (torch.exp(sig * net.forward(me_mod.features(mc)).double() + mu) * torch.from_numpy(w_c).to(dev)).cpu().numpy()
    we_c = (ctx.eval(mc) * torch.from_numpy(w_c).to(dev)).cpu().numpy()
    pos = s_c > 0
    s_max = float(np.quantile(s_c[pos], 0.999))
    r_max = float(np.quantile(we_c[pos] / s_c[pos], 0.999))
    w_max = float(np.quantile(we_c[pos], 0.999))
    # unweighting sample
    nu = 1 << 18
    mom_u, w_u = process_points("gg_ttgg", nu, 5, return_weight=True, precise=False)
    w_u = w_u * gluon_cuts(mom_u)
    u = uniforms(nu, 2, 55)
    tm, tw, tu = (torch.from_numpy(a).to(dev) for a in (mom_u, w_u, u))
    out_idx = torch.empty(nu, dtype=torch.int32, device=dev)
    out_w = torch.empty(nu, dtype=torch.float64, device=dev)
    cnt = torch.zeros(2, dtype=torch.int32, device=dev)
    me_mod.unweight_two_stage(ctx.ctx, net.h, tm, tw, nu, tu, mu, sig, s_max, r_max, out_idx, out_w, cnt)
    torch.cuda.synchronize()
    n1, n2 = cnt.cpu().numpy().tolist()
    wt2 = out_w[:n2].cpu().numpy()
    neff2 = wt2.sum() ** 2 / (wt2 ** 2).sum()
    s = (torch.exp(sig * net.forward(me_mod.features(tm)).double() + mu) * tw).cpu().numpy()
    w = (ctx.eval(tm) * tw).cpu().numpy()
    # exact-only unweighting of the same points: every point with w_ps > 0 needs the exact ME
    n_exact_only = int((w_u > 0).sum())
    acc1 = u[:, 0] < np.minimum(1.0, w / w_max)
    wt1 = np.maximum(1.0, w / w_max)[acc1]
    neff1 = wt1.sum() ** 2 / (wt1 ** 2).sum()
    gain = (n_exact_only / neff1) / (n1 / neff2)
    print(f"[gain] exact calls per effective event: exact-only {n_exact_only / neff1:.0f}, "
          f"two-stage {n1 / neff2:.0f} (stage 1 kept {n1} of {nu}, accepted {n2}); gain {gain:.1f}", flush=True)
    assert gain > 2.0
    # unbiasedness: E[s_max r_max * sum of output weights] = sum of w
    ok = s > 0
    ratio = np.where(ok, w / np.where(ok, s, 1.0), 0.0)
    p_acc = np.where(ok, np.minimum(1, s / s_max) * np.minimum(1, ratio / r_max), 0.0)
    out_wt = np.maximum(1, s / s_max) * np.maximum(1, ratio / r_max)
    c2 = (s_max * r_max * out_wt) ** 2 * p_acc
    var = np.sum(c2 - w ** 2)
    est = s_max * r_max * wt2.sum()
    print(f"[gain] mean-weight estimate {est / nu:.4e} vs exact {w.sum() / nu:.4e} "
          f"({(est - w.sum()) / math.sqrt(var):+.2f} sigma)", flush=True)
    assert abs(est - w.sum()) < 5 * math.sqrt(var)
    ctx.close()
    net.close()
