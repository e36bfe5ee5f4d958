"""Pins of the oracle's learned-stage pieces: GELU, BF16 rounding, gradients, Adam, features,
the assembled correction (checked against the additive-Schwarz formula of Sec. 5.3) and the
energy behaviour of the accepted step."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import assemble, mlp
from tests import oracle_cases as oc


def test_gelu_closed_forms():
    x = np.linspace(-4, 4, 41)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-15)      # Phi(x) + Phi(-x) = 1
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-16
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(x)).max() < 1e-8


def test_bf16_rounding():
    e = 2.0 ** -7                                      # bf16 spacing at 1 (7 stored bits)
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + e / 2) == 1.0                 # halfway: ties to even
    assert mlp.bf16(1.0 + e + e / 2) == 1.0 + 2 * e     # halfway above an odd mantissa: up
    assert mlp.bf16(1.0 + e / 2 + 2.0 ** -20) == 1.0 + e
    assert mlp.bf16(-3.0) == -3.0
    x = np.random.default_rng(0).standard_normal(1000)
    assert np.abs(mlp.bf16(x) - x).max() <= np.abs(x).max() * 2.0 ** -8


def test_gradients_against_central_differences():
    rng = np.random.default_rng(3)
    p = mlp.init_params(20, 7, seed=5)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((9, 20))
    T = rng.standard_normal((9, 7))
    Y, cache = mlp.forward(p, X)
    loss, dY = mlp.mse(Y, T)
    g = mlp.backward(p, cache, dY)
    h = 1e-6
    for k in p:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.mse(mlp.forward(p, X)[0], T)
            flat[idx] = old - h
            lm, _ = mlp.mse(mlp.forward(p, X)[0], T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].ravel()[idx]) <= 1e-6 * max(1e-3, abs(fd)), (k, idx)


def test_adam_first_step_closed_form():
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -4.0, 1e-3])}
    z = {"w": np.zeros(3)}
    p1, m, v = mlp.adam(p, g, z, z, 1, lr=0.01)
    # bias-corrected moments equal g and g^2: the step is -lr g / (|g| + eps)
    assert np.allclose(p1["w"], p["w"] - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=0, atol=1e-15)


def _tank(dim=2):
    """A small sigma-mapped tank: 2D 4 x 2 elements at P = 3, or 3D 2 x 2 x 2 at P = 2 (depth
    and surface varying along x and y)."""
    wl = W.tank(4, 2, 3, Lx=0.4) if dim == 2 else W.tank3d(2, 2, 2, 2, L=0.4)
    m = oc.fine_mesh(wl)
    A = assemble.assemble_operator(m)
    return wl, m, A


def _sizes(m):
    """(inputs, outputs) of the stage network for mesh m."""
    n = m.NP ** m.dim
    return (5 if m.dim == 2 else 7) * n, n


@pytest.mark.parametrize("dim", [2, 3])
def test_features_scale_invariance_and_linearity(dim):
    wl, m, A = _tank(dim)
    p = mlp.init_params(*_sizes(m), seed=1)
    r = W.random_vector(m.N, 2)
    r[m.dirichlet_nodes()] = 0
    X1, s1 = mlp.features(m, r)
    X2, s2 = mlp.features(m, 3.5 * r)
    assert X1.shape == (m.E, _sizes(m)[0])
    assert np.abs(X1 - X2).max() < 1e-14 and np.allclose(s2, 3.5 * s1)
    c1 = mlp.correction(m, p, r, emulate=False)
    c2 = mlp.correction(m, p, 3.5 * r, emulate=False)
    assert np.abs(c2 - 3.5 * c1).max() < 1e-12 * np.abs(c2).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_network_is_skipped(dim):
    wl, m, A = _tank(dim)
    p = {k: np.zeros_like(v) for k, v in mlp.init_params(*_sizes(m), 0).items()}
    b = W.random_vector(m.N, 4)
    b[m.dirichlet_nodes()] = 0
    x0 = np.zeros(m.N)
    x1, ok = mlp.stage(A, m, p, b, x0)
    assert not ok and np.array_equal(x1, x0)


@pytest.mark.parametrize("dim", [2, 3])
def test_exact_local_solves_reproduce_additive_schwarz(dim):
    """With the network replaced by the exact element solve y_e = (a_e/s_e) (R_e A R_e^T)^{-1} r_e,
    the gather / scaling / weighted assembly plumbing gives W sum_e R_e^T (R_e A R_e^T)^{-1} R_e r,
    the non-overlapping Schwarz preconditioner of Sec. 5.3, computed here independently."""
    wl, m, A = _tank(dim)
    n = m.NP ** dim
    Ad = A.toarray()
    r = W.random_vector(m.N, 6)
    r[m.dirichlet_nodes()] = 0
    g, mm, a = mlp.element_scales(m)
    X, s = mlp.features(m, r)
    # "network": exact local solves
    Y = np.zeros((m.E, n))
    for e in range(m.E):
        idx = m.l2g[e]
        Y[e] = (a[e] / s[e]) * np.linalg.solve(Ad[np.ix_(idx, idx)], r[idx])
    ce = (s / a)[:, None] * Y
    c = np.bincount(m.l2g.ravel(), weights=ce.ravel(), minlength=m.N) / mlp.multiplicity(m)
    c[m.dirichlet_nodes()] = 0
    # Schwarz formula with explicit 0/1 restriction matrices and W = (sum R R^T)^{-1}
    S = np.zeros((m.N, m.N))
    Wd = np.zeros(m.N)
    for e in range(m.E):
        Rm = np.zeros((n, m.N))
        Rm[np.arange(n), m.l2g[e]] = 1.0
        S += Rm.T @ np.linalg.inv(Rm @ Ad @ Rm.T) @ Rm
        Wd += np.diag(Rm.T @ Rm)
    ref = (S @ r) / Wd
    ref[m.dirichlet_nodes()] = 0
    assert np.abs(c - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_accepted_stage_does_not_increase_energy_error(dim):
    wl, m, A = _tank(dim)
    rng = np.random.default_rng(8)
    xs = assemble.solve_direct(A, W.random_vector(m.N, 9))
    b = A @ xs
    for seed in range(5):
        p = mlp.init_params(*_sizes(m), seed)
        x0 = xs + 0.1 * rng.standard_normal(m.N)
        x0[m.dirichlet_nodes()] = xs[m.dirichlet_nodes()]
        x1, ok = mlp.stage(A, m, p, b, x0, emulate=False)
        e0, e1 = xs - x0, xs - x1
        assert e1 @ (A @ e1) <= e0 @ (A @ e0) * (1 + 1e-12)


def test_adam_two_steps_by_hand():
    """Two Adam steps with gradients 1 then -2 (lr 0.01), worked by hand:
    m1 = 0.1, v1 = 0.001, step 1 = -0.01 (1 / (1 + 1e-8));
    m2 = 0.9 * 0.1 + 0.1 * (-2) = -0.11, v2 = 0.999 * 0.001 + 0.001 * 4 = 0.004999,
    m2_hat = -0.11 / 0.19 = -0.578947368..., v2_hat = 0.004999 / 0.001999 = 2.500750375...,
    sqrt(v2_hat) = 1.581376...,
    step 2 = -0.01 * m2_hat / (sqrt(v2_hat) + 1e-8) = +0.0036610352..."""
    p = {"w": np.array([0.5])}
    z = {"w": np.zeros(1)}
    p1, m1, v1 = mlp.adam(p, {"w": np.array([1.0])}, z, z, 1, lr=0.01)
    assert abs(m1["w"][0] - 0.1) < 1e-16 and abs(v1["w"][0] - 0.001) < 1e-18
    assert abs(p1["w"][0] - (0.5 - 0.01 / (1.0 + 1e-8))) < 1e-16
    p2, m2, v2 = mlp.adam(p1, {"w": np.array([-2.0])}, m1, v1, 2, lr=0.01)
    assert abs(m2["w"][0] + 0.11) < 1e-15 and abs(v2["w"][0] - 0.004999) < 1e-17
    m2_hat = -0.11 / 0.19
    v2_hat = 0.004999 / 0.001999
    assert abs(m2_hat + 0.5789473684210527) < 1e-15 and abs(v2_hat - 2.5007503751875937) < 1e-14
    step2 = 0.01 * 0.5789473684210527 / (math.sqrt(2.5007503751875937) + 1e-8)
    assert abs(step2 - 0.0036610352) < 1e-10
    assert abs(p2["w"][0] - (p1["w"][0] + step2)) < 1e-15


def test_adam_constant_gradient_trajectory():
    """With a constant gradient the bias-corrected moments are g and g^2 at every step, so t
    steps at a fixed rate move each weight by t lr g / (|g| + eps): pins the step-dependent
    bias corrections beyond the first step."""
    g = {"w": np.array([0.3, -4.0, 2e-3])}
    p0 = {"w": np.array([1.0, -2.0, 0.5])}
    p, m, v = p0, {"w": np.zeros(3)}, {"w": np.zeros(3)}
    for t in range(1, 13):
        p, m, v = mlp.adam(p, g, m, v, t, lr=0.01)
        step = 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
        assert np.allclose(p["w"], p0["w"] - t * step, rtol=0, atol=1e-13), t


def test_cosine_schedule_values():
    assert mlp.cosine_lr(2e-3, 1, 100) == 2e-3
    assert abs(mlp.cosine_lr(2e-3, 51, 100) - 1e-3) < 1e-18          # half way: lr0 / 2
    assert abs(mlp.cosine_lr(2e-3, 26, 100) - 1e-3 * (1 + math.sqrt(0.5))) < 1e-15
    assert 0 < mlp.cosine_lr(2e-3, 100, 100) < 2e-3 * 1e-3


def test_full_batch_training_lowers_the_loss():
    rng = np.random.default_rng(4)
    p = mlp.init_params(20, 6, seed=2)
    X = rng.standard_normal((64, 20))
    T = np.tanh(X[:, :6] - 0.5 * X[:, 6:12])
    p1, losses = mlp.train_full_batch(p, X, T, 60, 3e-3, emulate=False)
    assert losses[-1] < 0.5 * losses[0]
    # one step equals one explicit forward / backward / Adam step at the schedule's first rate
    q, l1 = mlp.train_full_batch(p, X, T, 1, 3e-3, total_steps=60, emulate=False)
    Y, cache = mlp.forward(p, X)
    loss, dY = mlp.mse(Y, T)
    g = mlp.backward(p, cache, dY)
    z = {k: np.zeros_like(v) for k, v in p.items()}
    r, _, _ = mlp.adam(p, g, z, z, 1, lr=3e-3)
    assert l1[0] == loss and all(np.array_equal(q[k], r[k]) for k in p)
