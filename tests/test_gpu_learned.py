"""GPU parity of the learned smoothing stage against the CPU oracle (oracle/mlp.py).

Bars: the BF16-operand / FP32-accumulate network against the oracle's BF16 emulation within 1e-4
(relative Frobenius; residual differences come from FP32 vs FP64 accumulation order flipping a
few BF16 roundings of hidden activations) and against the pure FP64 network within 2e-2;
gradients within 1e-3 per tensor; features within 1e-6; one stage's update within 1e-3 and the
same accept/skip decision.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble, mlp, pmg
from tests import oracle_cases as oc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_14977_amd import binding as B  # noqa: E402
from paper_2411_14977_amd import cases, learned  # noqa: E402

N_IN, N_OUT = 405, 81


def T64(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def T32(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def frob(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def params(seed, scale=1.0, bias=0.1):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(N_IN, N_OUT, seed)
    for k in p:
        if k.startswith("W"):
            p[k] = p[k] * scale
        else:
            p[k] = rng.standard_normal(p[k].shape) * bias
    # the blob stores FP32: give the oracle the same values
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def blob(p):
    return B.blob_pack(N_IN, N_OUT, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"])


def test_blob_roundtrip():
    p = params(1)
    q = B.blob_unpack(blob(p))
    for k in p:
        assert np.array_equal(p[k], q[k])
    assert len(blob(p)) == B.sem_mlp_blob_size(N_IN, N_OUT)


def test_mlp_forward_matches_oracle():
    p = params(2)
    X = np.random.default_rng(3).standard_normal((1000, N_IN)).astype(np.float32).astype(np.float64)
    Y = H(B.sem_mlp_forward(blob(p), T32(X), N_OUT))
    Ye, _ = mlp.forward(p, X, emulate=True)
    Yd, _ = mlp.forward(p, X, emulate=False)
    print(f"[gpu] forward vs emulation {frob(Y, Ye):.2e}, vs fp64 {frob(Y, Yd):.2e}", flush=True)
    assert frob(Y, Ye) <= 1e-4
    assert frob(Y, Yd) <= 2e-2


def test_mlp_gradients_match_oracle():
    p = params(4)
    rng = np.random.default_rng(5)
    n = 300  # not a multiple of 16: padded rows must not contribute
    X = rng.standard_normal((n, N_IN)).astype(np.float32).astype(np.float64)
    Tt = rng.standard_normal((n, N_OUT)).astype(np.float32).astype(np.float64)
    npar = sum(v.size for v in p.values())
    g, loss = B.sem_mlp_gradients(blob(p), T32(X), T32(Tt), npar)
    Y, cache = mlp.forward(p, X, emulate=True)
    lref, dY = mlp.mse(Y, Tt)
    gref = mlp.backward(p, cache, dY, emulate=True)
    assert abs(loss - lref) <= 1e-5 * lref
    off = 0
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        gk = g[off:off + p[k].size].reshape(p[k].shape).astype(np.float64)
        off += p[k].size
        e = frob(gk, gref[k])
        print(f"[gpu] grad {k}: {e:.2e}", flush=True)
        assert e <= 1e-3, k


@pytest.mark.parametrize("n,nin,nout", [(1100, 1200, 50), (70, 30, 40)])
def test_mlp_gradients_other_shapes(n, nin, nout):
    """Loss and gradients at shapes the stage's own network does not have: more than 64 16-wide
    k-steps in the products (input width 1200 padded to 1216; 1100 rows padded to 1104), and
    output widths that leave a partial 64-column block (40 -> 48 padded)."""
    rng = np.random.default_rng(17)
    p = mlp.init_params(nin, nout, 23)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    bl = B.blob_pack(nin, nout, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"])
    X = rng.standard_normal((n, nin)).astype(np.float32).astype(np.float64)
    Tt = rng.standard_normal((n, nout)).astype(np.float32).astype(np.float64)
    npar = sum(v.size for v in p.values())
    g, loss = B.sem_mlp_gradients(bl, T32(X), T32(Tt), npar)
    Y, cache = mlp.forward(p, X, emulate=True)
    lref, dY = mlp.mse(Y, Tt)
    gref = mlp.backward(p, cache, dY, emulate=True)
    assert abs(loss - lref) <= 1e-5 * lref
    off = 0
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        gk = g[off:off + p[k].size].reshape(p[k].shape).astype(np.float64)
        off += p[k].size
        e = frob(gk, gref[k])
        print(f"[gpu] grad {k} ({n} x {nin} -> {nout}): {e:.2e}", flush=True)
        assert e <= 1e-3, k


def _train_mesh_case():
    h_fn, eta_fn = W.training_geometry(0)
    x = oc.fine_x_nodes(8, 8, 2 * np.pi)
    from oracle import mesh
    m = mesh.Mesh2D(8, 4, 8, 2 * np.pi, h_fn(x), eta_fn(x))
    sv, _ = learned.training_solver(0, layout="c1")
    return m, sv


def test_features_match_oracle():
    m, sv = _train_mesh_case()
    rng = np.random.default_rng(6)
    r = rng.standard_normal(m.N)
    r[m.dirichlet_nodes()] = 0
    e = rng.standard_normal(m.N)
    X = torch.zeros(m.E, N_IN, dtype=torch.float32, device="cuda")
    Tt = torch.zeros(m.E, N_OUT, dtype=torch.float32, device="cuda")
    B.sem_learned_features(sv.ctx, T64(r), T64(e), X, Tt)
    Xo, s = mlp.features(m, r)
    To = mlp.targets(m, e, s)
    assert np.abs(H(X) - Xo).max() <= 1e-6 * np.abs(Xo).max()
    assert np.abs(H(Tt) - To).max() <= 1e-6 * np.abs(To).max()
    # element-block-solve targets
    B.sem_learned_features(sv.ctx, T64(r), None, X, Tt)
    A = assemble.assemble_operator(m)
    Tl = mlp.local_targets(m, A, r, s)
    assert np.abs(H(X) - Xo).max() <= 1e-6 * np.abs(Xo).max()
    assert np.abs(H(Tt) - Tl).max() <= 1e-6 * np.abs(Tl).max()
    sv.close()


def params_p(P, seed, scale=1.0, bias=0.1):
    n = (P + 1) ** 2
    rng = np.random.default_rng(seed)
    p = mlp.init_params(5 * n, n, seed)
    for k in p:
        p[k] = p[k] * scale if k.startswith("W") else rng.standard_normal(p[k].shape) * bias
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


STAGE_CASES = [
    # (Nx, Nz, P, Lx, weight scale, seed): 64 elements (4 full tiles of 16) at P = 8 with
    # positive, negative (always rejected) and small weights; ragged tiles at P = 4 and P = 3;
    # the fused kernels (residual, assembly with the apply of c) wherever the columns fit
    (16, 4, 8, 1.6, 1.0, 7),
    (16, 4, 8, 1.6, -1.0, 8),
    (16, 4, 8, 1.6, 0.3, 9),
    (5, 3, 4, 0.5, 1.0, 10),
    (7, 2, 3, 0.7, 0.5, 11),
    # columns of 60 elements at P = 8: too tall for the fused kernels (operator with side
    # buffer, separate assembly)
    (2, 60, 8, 0.2, 1.0, 12),
]


@pytest.mark.parametrize("Nx,Nz,P,Lx,scale,seed", STAGE_CASES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_learned_stage_matches_oracle(Nx, Nz, P, Lx, scale, seed, prec):
    wl = W.tank(Nx, Nz, P, Lx=Lx, name=f"tank{Nx}x{Nz}p{P}")
    m = oc.fine_mesh(wl)
    A = assemble.assemble_operator(m)
    p = params_p(P, seed, scale=scale)
    n = (P + 1) ** 2
    rng = np.random.default_rng(seed)
    dn = m.dirichlet_nodes()
    b = W.random_vector(m.N, seed)
    b[dn] = 0.0   # the stage acts on the V-cycle's correction problem: zero surface data
    x0 = 0.1 * rng.standard_normal(m.N)
    x0[dn] = 0.0
    s = cases.make_solver(wl, prec=prec)
    s.learned_load(B.blob_pack(5 * n, n, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"]),
                   enable=True)
    x = T64(x0)
    acc = B.sem_learned_stage(s.ctx, T64(b), x)
    x1o, ok = mlp.stage(A, m, p, b, x0, emulate=True)
    assert acc == ok
    d_gpu, d_ref = H(x) - x0, x1o - x0
    if ok:
        # f32: the residual feeding the network and the update are FP32 (relative 1e-6 of r)
        assert frob(d_gpu, d_ref) <= 1e-3, frob(d_gpu, d_ref)
    else:
        assert np.array_equal(H(x), x0) if prec == "f64" else frob(H(x), x0) <= 1e-6
    s.close()


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_zero_network_leaves_vcycle_unchanged(mode):
    # c = 0 -> the step is rejected (0/0) and the V-cycle continues from the unchanged residual,
    # bit for bit, in every placement
    wl = W.tank(16, 4, 8, Lx=1.6, name="tank8")
    s = cases.make_solver(wl, prec="f32")
    r = W.random_vector(s.n_global, 11)
    nzn = wl.Nz * wl.P + 1
    r[nzn - 1::nzn] = 0.0
    z0 = H(s.vcycle(T64(r)))
    p = {k: np.zeros_like(v) for k, v in params(1).items()}
    s.learned_load(blob(p), enable=mode)
    z1 = H(s.vcycle(T64(r)))
    assert np.array_equal(z0, z1)
    s.close()


def test_training_reduces_loss():
    X, Tt = learned.harvest(n_surfaces=2, n_bump=2, n_white=1, n_cycles=4, n_random=2,
                            max_pairs=512)
    assert X.shape == (512, N_IN) and Tt.shape == (512, N_OUT)
    assert torch.isfinite(X).all() and torch.isfinite(Tt).all()
    bl, losses = learned.train(X, Tt, epochs=20, batch=64, lr=1e-3, seed=3)
    print(f"[gpu] training losses first {losses[0]} last {losses[-1]}", flush=True)
    assert np.all(np.isfinite(losses))
    # the per-epoch training figure is one batch's; judge the fit on the whole set instead:
    # the trained network must beat the zero predictor (loss mean(T^2)) by a wide margin
    npar = sum(v.size for v in params(1).values())
    _, full = B.sem_mlp_gradients(bl, X, Tt, npar)
    zero = float((Tt.double() ** 2).mean())
    print(f"[gpu] full-set loss {full:.4f} vs zero predictor {zero:.4f}", flush=True)
    assert full < 0.5 * zero
    assert losses[-1, 1] < losses[0, 1]


def test_learned_solve_meets_the_oracle_bar():
    X, Tt = learned.harvest(n_surfaces=4, n_bump=2, n_white=2, n_cycles=6, n_random=4)
    bl, losses = learned.train(X, Tt, epochs=30, batch=256, lr=1e-3, seed=5)
    wl = W.tank(32, 8, 8, Lx=3.2, name="tank32")
    m = oc.fine_mesh(wl)
    A = assemble.assemble_operator(m)
    b = oc.rhs(wl, m)
    xd = assemble.solve_direct(A, b)
    res = {}
    for prec in ("f64", "f32"):
        for use in (0, 1, 2, 3):   # off, before pre-smoothing's restriction, before post, both
            s = cases.make_solver(wl, prec=prec)
            if use:
                s.learned_load(bl, enable=use)
            x, info, st = s.solve(T64(b), tol=1e-10)
            err = np.linalg.norm(H(x) - xd) / np.linalg.norm(xd)
            res[(prec, use)] = (info.iters, info.learned_skips, err)
            assert info.rel_res <= 1e-10 and err <= 1e-8, (prec, use, err)
            s.close()
    print(f"[gpu] learned solve (iters, skips, err): {res}", flush=True)


# ---- training pairs and training through the context (sem_learned_harvest, sem_learned_train) --
def _harvest_case():
    """The c1-layout training geometry at P = 8 (32 elements) with its oracle hierarchy."""
    h_fn, eta_fn = W.training_geometry(0)
    x = oc.fine_x_nodes(8, 8, 2 * np.pi)
    args = dict(dim=2, Nx=8, Nz=4, Lx=2 * np.pi, h=h_fn(x), eta=eta_fn(x))
    Hh = pmg.Hierarchy(args, [8, 4, 2, 1])
    pmg.estimate_lambdas(Hh)
    sv, source = learned.training_solver(0, layout="c1")
    for l, L in enumerate(Hh.levels[:-1]):
        sv.set_lambda(l, L.lam)
    return Hh, sv


def _oracle_harvest(Hh, b, cycles):
    """Rows of every element at the stage point of each defect-correction cycle (oracle)."""
    L0 = Hh.levels[0]
    m = L0.mesh
    sc = mlp.element_scales(m)
    x = np.zeros(L0.N)
    Xs, Ts = [], []
    for _ in range(cycles):
        r = b - L0.A @ x
        xpre = Hh.smooth(0, r, np.zeros(L0.N), pre=True)
        rpre = r - L0.A @ xpre
        X, s = mlp.features(m, rpre, sc)
        Xs.append(X)
        Ts.append(mlp.local_targets(m, L0.A, rpre, s, sc))
        x = x + Hh.vcycle(r)
    return np.concatenate(Xs), np.concatenate(Ts)


def test_harvest_matches_oracle():
    Hh, sv = _harvest_case()
    L0 = Hh.levels[0]
    E, n = L0.mesh.E, 81
    b = W.random_vector(L0.N, 77)
    b[L0.dn] = 0.0
    cycles = 3
    X = torch.zeros(cycles * E, 5 * n, dtype=torch.float32, device="cuda")
    Tt = torch.zeros(cycles * E, n, dtype=torch.float32, device="cuda")
    rows = B.sem_learned_harvest(sv.ctx, T64(b), cycles, 0, 5, X, Tt)
    assert rows == cycles * E
    Xo, To = _oracle_harvest(Hh, b, cycles)
    eX = np.abs(H(X) - Xo).max() / np.abs(Xo).max()
    eT = np.abs(H(Tt) - To).max() / np.abs(To).max()
    print(f"[gpu] harvest vs oracle: features {eX:.2e}, targets {eT:.2e}", flush=True)
    assert eX <= 1e-6 and eT <= 1e-6
    # sampled rows: each cycle's rows are distinct elements of that cycle's oracle rows
    per = 7
    Xs = torch.zeros(cycles * per, 5 * n, dtype=torch.float32, device="cuda")
    Ts = torch.zeros(cycles * per, n, dtype=torch.float32, device="cuda")
    assert B.sem_learned_harvest(sv.ctx, T64(b), cycles, per, 6, Xs, Ts) == cycles * per
    Xs, Ts = H(Xs), H(Ts)
    for k in range(cycles):
        ref = Xo[k * E:(k + 1) * E]
        hit = []
        for row in Xs[k * per:(k + 1) * per]:
            d = np.abs(ref - row).max(axis=1)
            hit.append(int(np.argmin(d)))
            assert d.min() <= 1e-6 * np.abs(ref).max()
        assert len(set(hit)) == per
    # cycles = 0: the rows of b itself
    X0 = torch.zeros(E, 5 * n, dtype=torch.float32, device="cuda")
    T0 = torch.zeros(E, n, dtype=torch.float32, device="cuda")
    assert B.sem_learned_harvest(sv.ctx, T64(b), 0, 0, 1, X0, T0) == E
    Xb, sb = mlp.features(L0.mesh, b)
    assert np.abs(H(X0) - Xb).max() <= 1e-6 * np.abs(Xb).max()
    assert np.abs(H(T0) - mlp.local_targets(L0.mesh, L0.A, b, sb)).max() <= 1e-6 * np.abs(H(T0)).max()
    sv.close()


def test_learned_train_adam_matches_oracle():
    """Three full-batch Adam steps with the cosine schedule from given weights: the change of
    every parameter tensor against the oracle's FP64 Adam on its BF16-emulated gradients."""
    wl = W.tank(16, 4, 8, Lx=1.6, name="tank8")
    s = cases.make_solver(wl, prec="f32")
    p0 = params(41, scale=1.0, bias=0.1)
    rng = np.random.default_rng(42)
    nrow = 256
    X = rng.standard_normal((nrow, N_IN)).astype(np.float32).astype(np.float64)
    Tt = (0.5 * rng.standard_normal((nrow, N_OUT))).astype(np.float32).astype(np.float64)
    steps, lr = 3, 1e-3
    bl = B.sem_learned_train(s.ctx, T32(X), T32(Tt), epochs=steps, batch=nrow, lr=lr,
                             val_frac=0.0, seed=9, init=blob(p0))
    got = B.blob_unpack(bl)
    ref, losses = mlp.train_full_batch(dict(p0), X, Tt, steps, lr, emulate=True)
    worst = 0.0
    for k in p0:
        e = frob(got[k] - p0[k], ref[k] - p0[k])
        worst = max(worst, e)
        print(f"[gpu] Adam {k}: change {np.linalg.norm(ref[k] - p0[k]):.3e}, error {e:.2e}", flush=True)
        assert e <= 2e-2, k
    # the network is now loaded into the context (placement off until enabled)
    B.sem_learned_enable(s.ctx, 3)
    s.close()


@pytest.mark.parametrize("mode", [1, 3])
def test_stage_switched_off_after_three_rejected_iterations(mode):
    """A network whose every correction is rejected: after three iterations in a row with every
    application rejected the stage is off for the rest of the solve, which then equals the plain
    solve bit for bit (a rejected stage leaves the cycle unchanged); the next solve starts with
    the stage on again."""
    wl = W.tank(16, 4, 8, Lx=1.6, name="tank8")
    s = cases.make_solver(wl, prec="f32")
    b = cases.make_rhs(wl, s)
    x0, i0, _ = s.solve(b, tol=1e-10)
    # the zero network: c = 0, so every judge sees 0/0 and rejects the application
    p = {k: np.zeros_like(v) for k, v in params(1).items()}
    s.learned_load(blob(p), enable=mode)
    per = 2 if mode == 3 else 1
    for _ in range(2):
        x1, i1, _ = s.solve(b, tol=1e-10)
        print(f"[gpu] rejected stage mode {mode}: off after {i1.stage_off_at}, skips "
              f"{i1.learned_skips}, iterations {i1.iters} vs {i0.iters}", flush=True)
        assert i1.stage_off_at == 3
        assert i1.learned_skips >= 3 * per
        assert i1.iters == i0.iters and torch.equal(x0, x1)
    s.close()


# ---- the plain smoother as the judge of the stage (sem_learned_judge) -------------------------
def _judge_case(prec):
    wl = W.tank(16, 4, 8, Lx=1.6, name="tank8")
    Ho = oc.hierarchy(wl)
    pmg.estimate_lambdas(Ho)
    s = cases.make_solver(wl, prec=prec)
    for l, L in enumerate(Ho.levels[:-1]):
        s.set_lambda(l, L.lam)
    m = Ho.levels[0].mesh
    return wl, Ho, s, oc.rhs(wl, m)


def test_judge_rates_match_the_oracle_defect_correction():
    """rho of the plain cycles equals the oracle's defect-correction rate over the same cycles
    (one untimed, then `cycles` timed) in FP64; a network every judge rejects (zero output)
    leaves the rate unchanged, costs time, and is switched off."""
    wl, Ho, s, b = _judge_case("f64")
    L0 = Ho.levels[0]
    x = np.zeros(L0.N)
    x[L0.dn] = b[L0.dn]
    norms = []
    for _ in range(5):
        r = b - L0.A @ x
        norms.append(np.linalg.norm(r))
        x = x + Ho.vcycle(r)
    norms.append(np.linalg.norm(b - L0.A @ x))
    rho_ref = (norms[5] / norms[1]) ** (1.0 / 4)
    p = {k: np.zeros_like(v) for k, v in params(1).items()}
    s.learned_load(blob(p), enable=1)
    res = s.learned_judge(T64(b), cycles=4)
    print(f"[gpu] judge (zero network): {res}, oracle rho {rho_ref:.6f}", flush=True)
    assert abs(res["rho_plain"] - rho_ref) <= 1e-9 * rho_ref
    assert abs(res["rho_learned"] - res["rho_plain"]) <= 1e-12 * rho_ref
    assert res["ms_plain"] > 0 and res["ms_learned"] > 0
    assert res["enabled"] is False
    # the stage stays off: a solve rejects nothing
    s.solve(T64(b), tol=1e-10)
    assert B.sem_learned_skips(s.ctx) == 0
    s.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_judge_decision_follows_its_measurements(prec):
    """With a network that passes the scaled residual through (a Jacobi-like element step) the
    decision is the rule applied to the returned numbers, and the stage state follows it."""
    wl, Ho, s, b = _judge_case(prec)
    n = (wl.P + 1) ** 2
    pz = params_p(wl.P, 5, scale=0.0, bias=0.0)
    # GELU(u) - GELU(-u) = u: hidden pair (+u, -u) and output difference, per node
    W1 = np.zeros((5 * n, 128)); W2 = np.zeros((128, 128)); W3 = np.zeros((128, n))
    for j in range(min(n, 64)):
        W1[j, 2 * j], W1[j, 2 * j + 1] = 1.0, -1.0
        W2[2 * j, 2 * j], W2[2 * j + 1, 2 * j + 1] = 1.0, 1.0
        W3[2 * j, j], W3[2 * j + 1, j] = 1.0, -1.0
    pz.update(W1=W1, W2=W2, W3=W3)
    s.learned_load(B.blob_pack(5 * n, n, pz["W1"], pz["b1"], pz["W2"], pz["b2"], pz["W3"],
                               pz["b3"]), enable=1)
    res = s.learned_judge(T64(b), cycles=5)
    print(f"[gpu] judge ({prec}): {res}", flush=True)
    import math
    rule = (res["rho_learned"] < 1.0 and math.log(res["rho_learned"]) / res["ms_learned"]
            < math.log(res["rho_plain"]) / res["ms_plain"])
    assert res["enabled"] == rule
    assert 0.0 < res["rho_plain"] < 1.0 and 0.0 < res["rho_learned"] < 1.0
    # the decision holds for the next solve: skips are counted only with the stage on
    B.sem_learned_skips(s.ctx, reset=True)
    x, info, _ = s.solve(T64(b), tol=1e-10)
    assert info.rel_res <= 1e-10
    s.close()
