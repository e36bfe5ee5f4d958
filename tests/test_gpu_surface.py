"""GPU parity of the surface update (time series) against the CPU oracle.

After sem_mesh_update_surface the outer operator, the right-hand side (lumped mass, wall faces)
and the level-0 node coordinates must be those of the oracle's mesh on the new surface; with a
frozen preconditioner the coarser levels stay those of the set-up surface and the solve still
reaches the new operator's solution; with a refresh every level (operators, lambda_hat, V-cycle,
learned stage) is the oracle's on the new surface.  Bars as in the other parity tests.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble, mesh, mlp, pmg
from tests import oracle_cases as oc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_14977_amd import binding as B  # noqa: E402
from paper_2411_14977_amd import cases  # noqa: E402


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


WL3 = W.tank3d(4, 4, 2, 2, L=0.8, name="t3h")
CDM3 = 40


def eta3(wl, t):
    (X, Y), _, _ = oc.surface_samples(wl)
    return W.surface_3d(X, Y, t, wl.Lx, wl.surface_seed)


def args_with(wl, eta):
    a = oc.mesh_args(wl)
    a["eta"] = eta
    return a


def hierarchy_with(wl, eta, **kw):
    opts = dict(smoother=wl.smoother, nu_pre=wl.nu_pre, nu_post=wl.nu_post,
                cheb_degree=wl.cheb_degree, cheb_lo=wl.cheb_lo, cheb_hi=wl.cheb_hi,
                cheb_degree_coarse=wl.cheb_degree_coarse or None)
    opts.update(kw)
    return pmg.Hierarchy(args_with(wl, eta), wl.orders, **opts)


def source3(x, y, z, wl, t, eta_fn):
    return W.bumps_3d(x, y, z, t, wl.Lx, wl.rhs_seed,
                      lambda a, b: W.bar_depth_3d(a, b, wl.Lx, wl.surface_seed), eta_fn)


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_update_3d_frozen_preconditioner(prec):
    wl, t = WL3, 0.37
    e2 = eta3(wl, t)
    Ho = oc.hierarchy(wl, coarse_dense_max=CDM3)          # set-up surface
    Hn = hierarchy_with(wl, e2, coarse_dense_max=CDM3)    # new surface
    s = cases.make_solver(wl, prec=prec, coarse_dense_max=CDM3)
    s.update_surface(e2)
    m2 = Hn.levels[0].mesh
    x = W.random_vector(m2.N, 5)
    assert rel(H(s.apply(T(x))), Hn.levels[0].A @ x) < 1e-12
    # the V-cycle levels are those of the set-up surface
    x1 = W.random_vector(Ho.levels[1].N, 6)
    tol1 = 1e-12 if prec == "f64" else 1e-2
    assert rel(H(s.apply_level(1, T(x1))), Ho.levels[1].A @ x1) <= tol1
    # current node coordinates and right-hand side
    xg, yg, zg = s.coords(0)
    xo, yo, zo = m2.node_coords()
    assert np.abs(zg - zo).max() < 1e-13 and np.abs(xg - xo).max() < 1e-13
    eta_fn = lambda a, b: W.surface_3d(a, b, t, wl.Lx, wl.surface_seed)
    b_lib = H(s.assemble_rhs(f=T(source3(xg, yg, zg, wl, t, eta_fn))))
    b_ref = assemble.assemble_rhs(m2, f=source3(xo, yo, zo, wl, t, eta_fn))
    assert rel(b_lib, b_ref) < 1e-12
    xs, info, _ = s.solve(T(b_ref), tol=1e-10)
    xd = assemble.solve_direct(Hn.levels[0].A, b_ref)
    err = np.linalg.norm(H(xs) - xd) / np.linalg.norm(xd)
    print(f"[gpu] frozen 3D {prec}: {info.iters} iterations, error {err:.2e}", flush=True)
    assert err <= (1e-9 if prec == "f64" else 1e-8)
    s.close()


def test_update_3d_refresh():
    wl, t = WL3, 0.61
    e2 = eta3(wl, t)
    Hn = hierarchy_with(wl, e2, coarse_dense_max=CDM3)
    pmg.estimate_lambdas(Hn)
    s = cases.make_solver(wl, coarse_dense_max=CDM3)
    s.update_surface(e2, refresh=True)
    for l, L in enumerate(Hn.levels):
        x = W.random_vector(L.N, 40 + l)
        assert rel(H(s.apply_level(l, T(x))), L.A @ x) < 1e-12, l
        if l + 1 < len(Hn.levels):
            assert abs(s.level(l)[2] - L.lam) <= 1e-10 * L.lam, l
    r = W.random_vector(Hn.levels[0].N, 9)
    r[Hn.levels[0].dn] = 0.0
    assert rel(H(s.vcycle(T(r))), Hn.vcycle(r)) < 1e-12
    s.close()


def test_update_rejects_nonpositive_depth():
    wl = WL3
    s = cases.make_solver(wl, coarse_dense_max=CDM3)
    _, h, _ = oc.surface_samples(wl)
    with pytest.raises(B.SemError):
        s.update_surface(-h - 0.01)
    x = W.random_vector(s.n_global, 1)   # the context still works with its old surface
    Ho = oc.hierarchy(wl, coarse_dense_max=CDM3)
    assert rel(H(s.apply(T(x))), Ho.levels[0].A @ x) < 1e-12
    s.close()


def test_update_2d_frozen_and_refresh_with_learned_stage():
    wl = W.tank(16, 4, 8, Lx=1.6, name="tank8")
    xs_, h, _ = oc.surface_samples(wl)
    e2 = W.surface(xs_, wl.Lx, wl.surface_seed + 11)
    a2 = args_with(wl, e2)
    m2 = mesh.Mesh2D(a2["Nx"], a2["Nz"], wl.P, a2["Lx"], a2["h"], e2)
    A2 = assemble.assemble_operator(m2)
    s = cases.make_solver(wl, prec="f32")
    n = (wl.P + 1) ** 2
    rng = np.random.default_rng(3)
    p = mlp.init_params(5 * n, n, 3)
    p = {k: (v if k.startswith("W") else rng.standard_normal(v.shape) * 0.1).astype(np.float32)
         .astype(np.float64) for k, v in p.items()}
    s.learned_load(B.blob_pack(5 * n, n, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"]),
                   enable=True)
    s.update_surface(e2)
    x = W.random_vector(m2.N, 2)
    assert rel(H(s.apply(T(x))), A2 @ x) < 1e-12
    # refresh: the stage's geometry (features, element scales) follows the new surface
    s.update_surface(e2, refresh=True)
    b = W.random_vector(m2.N, 4)
    b[m2.dirichlet_nodes()] = 0.0
    x0 = 0.1 * rng.standard_normal(m2.N)
    x0[m2.dirichlet_nodes()] = 0.0
    xg = T(x0)
    acc = B.sem_learned_stage(s.ctx, T(b), xg)
    x1o, ok = mlp.stage(A2, m2, p, b, x0, emulate=True)
    assert acc == ok
    if ok:
        assert np.linalg.norm((H(xg) - x0) - (x1o - x0)) <= 1e-3 * np.linalg.norm(x1o - x0)
    s.close()
