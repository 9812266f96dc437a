"""Pins of the CPU surrogate reference (oracle/mlp_ref.py) and of the
unweighting reference: finite differences, closed forms, exact expectations."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as R


def small_net(seed=0, n_in=5, width=7, depth=3):
    rng = np.random.default_rng(seed)
    th = rng.normal(size=R.n_params(n_in, width, depth)) * 0.5
    return th, (n_in, width, depth)


def test_param_count():
    assert R.n_params(24, 256, 4) == 204033


def test_silu_prime_matches_difference_quotient():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (R.silu(z + h) - R.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(R.silu_prime(z), fd, rtol=1e-7, atol=1e-9)


def test_gradient_finite_differences_all_parameters():
    th, dims = small_net()
    rng = np.random.default_rng(1)
    x = rng.normal(size=(64, dims[0]))
    t = rng.normal(size=64)
    _, g = R.loss_and_grad(th, x, t, *dims)
    fd = np.empty_like(th)
    for i in range(th.size):
        h = 1e-6 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        yp = R.forward(tp, x, *dims)
        ym = R.forward(tm, x, *dims)
        fd[i] = (np.mean((yp - t) ** 2) - np.mean((ym - t) ** 2)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_gradient_finite_differences_full_size_sampled():
    rng = np.random.default_rng(2)
    th = rng.uniform(-1, 1, size=R.n_params()) * 0.06
    x = rng.normal(size=(64, 24)) * 0.3
    t = rng.normal(size=64)
    _, g = R.loss_and_grad(th, x, t)
    for i in rng.choice(th.size, 40, replace=False):
        h = 1e-6 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (np.mean((R.forward(tp, x) - t) ** 2) - np.mean((R.forward(tm, x) - t) ** 2)) / (2 * h)
        # central differences of a loss of order 1 carry ~2e-16/h = 2e-10 of rounding
        assert abs(g[i] - fd) <= 1e-6 * abs(fd) + 5e-10


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2: theta -= lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = R.adam_step(th, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    np.testing.assert_allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_every_step():
    """With the same gradient g at every step, the bias-corrected moments are
    exactly g and g^2 at every t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so
    each update is lr g / (|g| + eps).  A bias correction with the wrong power
    of b1 or b2 breaks this from t = 2 on."""
    rng = np.random.default_rng(11)
    th0 = rng.normal(size=40)
    g = rng.normal(size=40) * np.logspace(-4, 2, 40)
    th, m, v = th0.copy(), np.zeros(40), np.zeros(40)
    lr = 3e-3
    for t in range(1, 6):
        new, m, v = R.adam_step(th, m, v, g, t, lr)
        np.testing.assert_allclose(new - th, -lr * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=0, err_msg=f"t={t}")
        np.testing.assert_allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12)
        np.testing.assert_allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)
        th = new


def test_adam_sign_flip_second_step():
    """Gradient g then -g: m_2 = 0.9*0.1 g - 0.1 g = -0.01 g, bias-corrected by
    1 - 0.81 = 0.19; v_2 = 0.999*0.001 g^2 + 0.001 g^2 = 0.001999 g^2, corrected
    by 1 - 0.998001 = 0.001999, i.e. exactly g^2.  The second update is
    therefore -lr (-0.01/0.19) g / (|g| + eps) = +lr g / (19 (|g| + eps))."""
    rng = np.random.default_rng(12)
    th0 = rng.normal(size=30)
    g = rng.normal(size=30)
    lr = 1e-2
    th1, m, v = R.adam_step(th0, np.zeros(30), np.zeros(30), g, 1, lr)
    th2, m, v = R.adam_step(th1, m, v, -g, 2, lr)
    np.testing.assert_allclose(th2 - th1, lr * g / (19 * (np.abs(g) + 1e-8)), rtol=1e-9)


def test_training_lowers_the_loss():
    th, dims = small_net(4)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(256, dims[0]))
    t = np.sin(x[:, 0]) + 0.5 * x[:, 1] ** 2
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0, _ = R.loss_and_grad(th, x, t, *dims)
    for step in range(1, 301):
        _, g = R.loss_and_grad(th, x, t, *dims)
        th, m, v = R.adam_step(th, m, v, g, step, 1e-2)
    l1, _ = R.loss_and_grad(th, x, t, *dims)
    assert l1 < 0.2 * l0


def test_bf16_round():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -2.5, 3.0e38, 1e-40])
    got = R.bf16_round(vals)
    assert got[0] == 1.0
    assert got[1] == 1.0                      # tie -> even
    assert got[2] == 1.0 + 2.0 ** -7          # above the tie -> up
    assert got[3] == -2.5
    assert abs(got[4] / 3.0e38 - 1) < 2 ** -8


def test_two_stage_expectation_exact():
    """Integrated over both uniforms, accepted x weight = w / (s_max r_max) for every point
    (midpoint rule over a 1000 x 1000 grid of (u1, u2), through two_stage itself)."""
    rng = np.random.default_rng(6)
    n = 20
    s = rng.uniform(0.2, 3.0, size=n)
    w = s * rng.uniform(0.4, 4.0, size=n)
    s_max, r_max = 1.5, 2.0
    g = (np.arange(1000) + 0.5) / 1000
    u1 = np.repeat(g, g.size)
    u2 = np.tile(g, g.size)
    tot = np.empty(n)
    for i in range(n):
        _, _, wt = R.two_stage(np.full(u1.size, s[i]), np.full(u1.size, w[i]), u1, u2, s_max, r_max)
        tot[i] = wt.mean()
    np.testing.assert_allclose(tot, w / (s_max * r_max), rtol=2e-2)


def test_two_stage_special_cases():
    rng = np.random.default_rng(7)
    n = 1000
    w = rng.uniform(0.1, 1.0, size=n)
    u1, u2 = rng.random(n), rng.random(n)
    # surrogate equal to the exact weight, r_max = 1: stage 2 always accepts
    a1, a2, wt = R.two_stage(w, w, u1, u2, s_max=1.0, r_max=1.0)
    assert np.array_equal(a1, a2)
    # constant surrogate: stage 1 accepts with probability s/s_max, stage 2 is hit-or-miss on w
    a1, a2, wt = R.two_stage(np.full(n, 0.5), w, u1, u2, s_max=0.5, r_max=2.0)
    assert a1.all()
    assert np.array_equal(a2, u2 < w / 0.5 / 2.0)
