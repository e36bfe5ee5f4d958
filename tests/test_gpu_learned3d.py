"""GPU parity of the learned smoothing stage on hexahedra (3D) against the oracle.

The stage on a 3D fine level (P <= 6, n = (P+1)^3 nodes per element, 7n network inputs: the
residual, the five non-zero factor fields and the lumped mass) follows the same formulas as in
2D: r = b - A x, element corrections from the network (BF16 MFMA operands, FP32 accumulation),
their average over the up to eight hexahedra holding a node, q = A c, alpha = c.r / c.q, accepted
when finite and positive.  Bars: features and element-block targets 1e-6; one stage's update
within 1e-3 of the oracle's (BF16 emulation) with the same accept/reject decision; the V-cycle
with the stage in each placement within 1% (FP64) / 3% (FP32) of the stage's change of the cycle.
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
from paper_2411_14977_amd import cases  # noqa: E402

CASES = {
    # 32 hexahedra at P = 3 (two 16-element tiles), levels 3-2-1
    "h3": W.tank3d(4, 4, 2, 3, L=0.8, name="h3"),
    # the benchmark's order: 8 hexahedra at P = 6 (one ragged tile), levels 6-3-1
    "h6": W.tank3d(2, 2, 2, 6, L=0.8, orders=[6, 3, 1], name="h6"),
    # odd counts, P = 2
    "h2": W.tank3d(3, 2, 3, 2, L=0.6, name="h2"),
}
_hier = {}


def T64(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def frob(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def hier(name, gstore=None):
    key = (name, gstore)
    if key not in _hier:
        Hh = oc.hierarchy(CASES[name], gstore=gstore)
        pmg.estimate_lambdas(Hh)
        _hier[key] = Hh
    return _hier[key]


def solver(name, prec, Hh):
    s = cases.make_solver(CASES[name], prec=prec)
    for l, L in enumerate(Hh.levels[:-1]):
        s.set_lambda(l, L.lam)
    return s


def sizes(P):
    n = (P + 1) ** 3
    return 7 * n, n


def random_params(P, seed, scale=1.0, bias=0.1):
    nin, n = sizes(P)
    rng = np.random.default_rng(seed)
    p = mlp.init_params(nin, n, seed)
    for k in p:
        p[k] = p[k] * scale if k.startswith("W") else rng.standard_normal(p[k].shape) * bias
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def jacobi_like_params(P, seed, noise=0.05):
    """Close to a masked Jacobi correction on 64 of the element's nodes (GELU(u) - GELU(-u) = u
    passes r_e / s_e through both hidden layers), every weight and bias perturbed."""
    nin, n = sizes(P)
    nh = 128
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, min(n, nh // 2), replace=False))
    W1, W2, W3 = np.zeros((nin, nh)), np.zeros((nh, nh)), np.zeros((nh, n))
    for j, i in enumerate(idx):
        W1[i, 2 * j], W1[i, 2 * j + 1] = 1.0, -1.0
        W2[2 * j, 2 * j], W2[2 * j + 1, 2 * j] = 1.0, -1.0
        W2[2 * j, 2 * j + 1], W2[2 * j + 1, 2 * j + 1] = -1.0, 1.0
        W3[2 * j, i], W3[2 * j + 1, i] = 0.5, -0.5
    p = dict(W1=W1 + noise * rng.uniform(-1, 1, W1.shape) / np.sqrt(nin),
             b1=noise * rng.standard_normal(nh),
             W2=W2 + noise * rng.uniform(-1, 1, W2.shape) / np.sqrt(nh),
             b2=noise * rng.standard_normal(nh),
             W3=W3 + noise * rng.uniform(-1, 1, W3.shape) / np.sqrt(nh),
             b3=noise * rng.standard_normal(n))
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def blob(p, P):
    nin, n = sizes(P)
    return B.blob_pack(nin, n, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"])


@pytest.mark.parametrize("name", list(CASES))
def test_features3d_match_oracle(name):
    wl = CASES[name]
    Hh = hier(name)
    m = Hh.levels[0].mesh
    A = Hh.levels[0].A
    nin, n = sizes(wl.P)
    s = solver(name, "f64", Hh)
    rng = np.random.default_rng(6)
    r = rng.standard_normal(m.N)
    r[m.dirichlet_nodes()] = 0
    e = rng.standard_normal(m.N)
    X = torch.zeros(m.E, nin, dtype=torch.float32, device="cuda")
    Tt = torch.zeros(m.E, n, dtype=torch.float32, device="cuda")
    B.sem_learned_features(s.ctx, T64(r), T64(e), X, Tt)
    Xo, so = mlp.features(m, r)
    assert np.abs(H(X) - Xo).max() <= 1e-6 * np.abs(Xo).max()
    assert np.abs(H(Tt) - mlp.targets(m, e, so)).max() <= 1e-6 * np.abs(mlp.targets(m, e, so)).max()
    B.sem_learned_features(s.ctx, T64(r), None, X, Tt)
    Tl = mlp.local_targets(m, A, r, so)
    assert np.abs(H(Tt) - Tl).max() <= 1e-6 * np.abs(Tl).max()
    s.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("scale,seed", [(1.0, 7), (-1.0, 8), (0.3, 9)])
def test_learned_stage3d_matches_oracle(name, prec, scale, seed):
    print(f"[gpu] 3D stage {name} {prec} scale {scale}", flush=True)
    wl = CASES[name]
    Hh = hier(name)
    m = Hh.levels[0].mesh
    A = assemble.assemble_operator(m)
    p = random_params(wl.P, seed, scale=scale)
    rng = np.random.default_rng(seed)
    dn = m.dirichlet_nodes()
    b = W.random_vector(m.N, seed)
    b[dn] = 0.0
    x0 = 0.1 * rng.standard_normal(m.N)
    x0[dn] = 0.0
    s = solver(name, prec, Hh)
    s.learned_load(blob(p, wl.P), enable=True)
    x = T64(x0)
    acc = B.sem_learned_stage(s.ctx, T64(b), x)
    x1o, ok = mlp.stage(A, m, p, b, x0, emulate=True)
    assert acc == ok
    if ok:
        assert frob(H(x) - x0, x1o - x0) <= 1e-3, frob(H(x) - x0, x1o - x0)
    else:
        assert np.array_equal(H(x), x0) if prec == "f64" else frob(H(x), x0) <= 1e-6
    s.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_learned_vcycle3d_matches_oracle(name, prec, mode):
    print(f"[gpu] 3D learned vcycle {name} {prec} mode {mode}", flush=True)
    wl = CASES[name]
    Hh = hier(name, None if prec == "f64" else "f32")
    L0 = Hh.levels[0]
    sc = mlp.element_scales(L0.mesh)
    p = jacobi_like_params(wl.P, 30 + mode)
    s = solver(name, prec, Hh)
    r = W.random_vector(L0.N, 970 + mode)
    r[L0.dn] = 0.0
    z0 = H(s.vcycle(T64(r)))
    s.learned_load(blob(p, wl.P), enable=mode)
    B.sem_learned_skips(s.ctx, reset=True)
    z1 = H(s.vcycle(T64(r)))
    skips = B.sem_learned_skips(s.ctx)
    log = []

    def stage(l, b, x):
        if l != 0:
            return x
        xn, ok = mlp.stage(L0.A, L0.mesh, p, b, x, emulate=True, scales=sc)
        log.append(ok)
        return xn

    z0_ref = Hh.vcycle(r)
    z1_ref = Hh.vcycle(r, hook=stage if mode & 1 else None, hook_post=stage if mode & 2 else None)
    change = np.linalg.norm(z1_ref - z0_ref)
    err = np.linalg.norm(z1 - z1_ref) / change
    print(f"[gpu] 3D learned vcycle {name} {prec} mode {mode}: change "
          f"{change / np.linalg.norm(z0_ref):.2e}, error {err:.2e} of it, oracle {log}, skips {skips}",
          flush=True)
    assert skips == log.count(False) and all(log)
    assert np.linalg.norm(z0 - z0_ref) <= 1e-2 * change
    assert err <= (1e-2 if prec == "f64" else 3e-2), err
    s.close()


def test_harvest3d_rows_match_features():
    """sem_learned_harvest on a 3D context: with cycles = 0 the rows of b itself equal
    sem_learned_features (and so the oracle's)."""
    name = "h3"
    wl = CASES[name]
    Hh = hier(name)
    m = Hh.levels[0].mesh
    nin, n = sizes(wl.P)
    s = solver(name, "f64", Hh)
    b = W.random_vector(m.N, 12)
    b[m.dirichlet_nodes()] = 0.0
    X = torch.zeros(m.E, nin, dtype=torch.float32, device="cuda")
    Tt = torch.zeros(m.E, n, dtype=torch.float32, device="cuda")
    assert B.sem_learned_harvest(s.ctx, T64(b), 0, 0, 1, X, Tt) == m.E
    Xo, so = mlp.features(m, b)
    assert np.abs(H(X) - Xo).max() <= 1e-6 * np.abs(Xo).max()
    Tl = mlp.local_targets(m, Hh.levels[0].A, b, so)
    assert np.abs(H(Tt) - Tl).max() <= 1e-6 * np.abs(Tl).max()
    # cycles of the context's own p-multigrid: finite rows, sampled count
    Xs = torch.zeros(3 * 5, nin, dtype=torch.float32, device="cuda")
    Ts = torch.zeros(3 * 5, n, dtype=torch.float32, device="cuda")
    assert B.sem_learned_harvest(s.ctx, T64(b), 3, 5, 2, Xs, Ts) == 15
    assert torch.isfinite(Xs).all() and torch.isfinite(Ts).all()
    s.close()
