"""GPU parity on 2D meshes whose x and sigma orders differ (semi-coarsened hierarchy, Sec. 5.1):
level orders, operator on every level (rectangular-element kernel and the equal-order kernels
below it), one-direction and two-direction transfers, smoothers, lambda_hat, V-cycle,
right-hand side and solves, each against the CPU oracle through the C ABI.

Bars as for equal orders: FP64 steps within 1e-12 (relative, max-norm) of the oracle, FP64
solves within 1e-9 of the oracle's direct solution, mixed precision within 1e-8 at a 1e-10
residual; inner-precision operators at 2e-6 (FP32) and 1e-2 (BF16 factors).
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble, pmg
from oracle.precision import with_stored_factors
from tests import oracle_cases as oc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - only on machines without a GPU
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


CASES = {
    # x order above sigma order, ragged column count: (6,3) -x-> (3,3) -> (2,2) -> (1,1)
    "semi_x": W.tank_semi(13, 3, 6, 3, Lx=1.3, name="semi_x"),
    # sigma order above x order: (2,7) -z-> (2,4) -z-> (2,2) -> (1,1)
    "semi_z": W.tank_semi(10, 2, 2, 7, Lx=1.0, name="semi_z"),
    # the largest order: (12,8) -x-> (8,8) (fused smoother steps) -> (4,4) -> (2,2) -> (1,1)
    "semi_wide": W.tank_semi(16, 2, 12, 8, Lx=4.0, name="semi_wide"),
    # linear in x: (1,4) -z-> (1,2) -z-> (1,1)
    "semi_px1": W.tank_semi(6, 2, 1, 4, Lx=0.6, name="semi_px1"),
    # the paper's order-sweep shape (N_x = 200, N_z = 2, P_z = 8) at P_x = 3
    "semi_sweep": W.tank_semi(200, 2, 3, 8, Lx=50.0, name="semi_sweep"),
}

_oracle = {}


def oracle_h(name):
    if name not in _oracle:
        H_ = oc.hierarchy(CASES[name])
        pmg.estimate_lambdas(H_)
        _oracle[name] = H_
    return _oracle[name]


def lib_solver(name, prec="f64", **kw):
    return cases.make_solver(CASES[name], prec=prec, **kw)


@pytest.mark.parametrize("name", list(CASES))
def test_semi_level_orders_and_sizes(name):
    wl = CASES[name]
    s = lib_solver(name)
    pairs = pmg.coarsen_orders_2d(wl.P, wl.pz)
    assert s.nlevels == len(pairs)
    H_ = oracle_h(name)
    for l, (px, pz) in enumerate(pairs):
        assert s.level_orders(l) == (px, pz), (name, l)
        assert s.level(l)[1] == H_.levels[l].N
    assert s.n_global == wl.n_global
    x, z = s.coords(0)
    xo, zo = H_.levels[0].mesh.node_coords()
    assert np.abs(x - xo).max() < 1e-13 and np.abs(z - zo).max() < 1e-13
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_semi_operator_fp64_all_levels(name):
    print(f"[gpu] semi operator parity {name}", flush=True)
    H_ = oracle_h(name)
    s = lib_solver(name)
    for l, L in enumerate(H_.levels):
        x = W.random_vector(L.N, 100 + l)
        y = H(s.apply_level(l, T(x)))
        assert rel(y, L.A @ x) < 1e-12, (name, l)
    x = W.random_vector(H_.levels[0].N, 7)
    assert rel(H(s.apply(T(x))), H_.levels[0].A @ x) < 1e-12
    s.close()


@pytest.mark.parametrize("name", ["semi_x", "semi_wide"])
@pytest.mark.parametrize("prec,bar", [("f32", 2e-6), ("bf16", 1e-2)])
def test_semi_operator_inner_precision(name, prec, bar):
    """Inner-precision operators against the oracle's operator with the factors rounded the
    same way (BF16) or exact (FP32: the bar covers the FP32 sums)."""
    H_ = oracle_h(name)
    s = lib_solver(name, prec=prec)
    for l, L in enumerate(H_.levels[:-1]):
        x = W.random_vector(L.N, 200 + l)
        y = H(s.apply_level(l, T(x)))
        ref = assemble.assemble_operator(with_stored_factors(L.mesh, prec)) @ x
        assert np.abs(y - ref).max() <= bar * np.abs(ref).max(), (name, prec, l)
    s.close()


def test_semi_pure_neumann_constant_nullspace():
    wl = CASES["semi_x"]
    s = cases.make_solver(wl, dirichlet=False)
    m = oc.fine_mesh(wl)
    A = assemble.assemble_operator(m, dirichlet=False)
    x = W.random_vector(m.N, 3)
    assert rel(H(s.apply(T(x))), A @ x) < 1e-12
    one = H(s.apply(T(np.ones(m.N))))
    assert np.abs(one).max() < 1e-12 * abs(A).max()
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_semi_transfers(name):
    H_ = oracle_h(name)
    s = lib_solver(name)
    for l in range(len(H_.levels) - 1):
        Lf, Lc = H_.levels[l], H_.levels[l + 1]
        b = W.random_vector(Lf.N, 300 + l)
        x = W.random_vector(Lf.N, 400 + l)
        b[Lf.dn] = 0.0
        rc = T(np.zeros(Lc.N))
        B.sem_restrict(s.ctx, l, T(b), T(x), rc)
        assert rel(H(rc), H_.restrict(l, b - Lf.A @ x)) < 1e-12, (name, l)
        B.sem_restrict(s.ctx, l, T(b), None, rc)
        assert rel(H(rc), H_.restrict(l, b)) < 1e-12, (name, l)
        ec = W.random_vector(Lc.N, 500 + l)
        ec[Lc.dn] = 0.0
        xf = T(x.copy())
        B.sem_prolong_add(s.ctx, l, T(ec), xf)
        assert rel(H(xf), x + H_.prolong(l, ec)) < 1e-12, (name, l)
    s.close()


@pytest.mark.parametrize("name", ["semi_x", "semi_z", "semi_wide"])
@pytest.mark.parametrize("smoother", ["jacobi", "chebyshev"])
def test_semi_smoothers(smoother, name):
    wl = CASES[name]
    H_ = oc.hierarchy(wl, smoother=smoother)
    pmg.estimate_lambdas(H_)
    s = cases.make_solver(wl, smoother=smoother)
    for l in range(len(H_.levels) - 1):
        L = H_.levels[l]
        s.set_lambda(l, L.lam)
        b = W.random_vector(L.N, 700 + l)
        b[L.dn] = 0.0
        x0 = W.random_vector(L.N, 800 + l)
        x0[L.dn] = 0.0
        x = T(np.zeros(L.N))
        B.sem_smooth(s.ctx, l, 1, T(b), x)
        assert rel(H(x), H_.smooth(l, b, np.zeros(L.N), pre=True)) < 1e-12, (name, l)
        x = T(x0)
        B.sem_smooth(s.ctx, l, 0, T(b), x)
        assert rel(H(x), H_.smooth(l, b, x0, pre=False)) < 1e-12, (name, l)
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_semi_lanczos_estimate(name):
    H_ = oracle_h(name)
    s = lib_solver(name)
    for l, L in enumerate(H_.levels[:-1]):
        assert abs(s.level(l)[2] - L.lam) < 1e-8 * L.lam, (name, l, s.level(l)[2], L.lam)
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_semi_vcycle(name):
    print(f"[gpu] semi vcycle parity {name}", flush=True)
    H_ = oracle_h(name)
    s = lib_solver(name)
    for l, L in enumerate(H_.levels[:-1]):
        s.set_lambda(l, L.lam)
    L0 = H_.levels[0]
    r = W.random_vector(L0.N, 900)
    r[L0.dn] = 0.0
    z = H(s.vcycle(T(r)))
    assert rel(z, H_.vcycle(r)) < 1e-12
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_semi_rhs_assembly(name):
    wl = CASES[name]
    s = lib_solver(name)
    ref = oc.rhs(wl, oc.fine_mesh(wl))
    got = H(cases.make_rhs(wl, s))
    assert rel(got, ref) < 1e-12
    s.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("outer", ["fpcg", "pdc", "gmres"])
def test_semi_solve_fp64_matches_direct(name, outer):
    print(f"[gpu] semi solve parity {name} {outer}", flush=True)
    wl = CASES[name]
    H_ = oracle_h(name)
    L0 = H_.levels[0]
    b = oc.rhs(wl, L0.mesh)
    xd = assemble.solve_direct(L0.A, b)
    s = lib_solver(name, outer=outer)
    x, info, st = s.solve(T(b), tol=1e-12)
    x = H(x)
    assert info.rel_res <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert np.linalg.norm(b - L0.A @ x) <= 2e-12 * np.linalg.norm(b)
    if outer == "fpcg":
        _, it_o, _ = pmg.fpcg(L0.A, b, np.zeros(L0.N), H_.vcycle, 1e-12)
        assert abs(info.iters - it_o) <= 1
    s.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_semi_mixed_precision_solve(prec):
    wl = CASES["semi_sweep"]
    H_ = oracle_h("semi_sweep")
    L0 = H_.levels[0]
    b = oc.rhs(wl, L0.mesh)
    xd = assemble.solve_direct(L0.A, b)
    s = lib_solver("semi_sweep", prec=prec)
    errs = {}
    for tol in (1e-6, 1e-8, 1e-10):
        x, info, st = s.solve(T(b), tol=tol)
        assert info.rel_res <= tol
        errs[tol] = np.linalg.norm(H(x) - xd) / np.linalg.norm(xd)
    print(f"[gpu] semi mixed {prec} errors {errs}", flush=True)
    assert errs[1e-10] <= 1e-8
    # deterministic: the same solve twice is bitwise equal
    x1, i1, _ = s.solve(T(b), tol=1e-10)
    x2, i2, _ = s.solve(T(b), tol=1e-10)
    assert i1.iters == i2.iters and torch.equal(x1, x2)
    s.close()


def test_semi_iterations_flat_in_px():
    """The paper's order sweep at N_x = 200, N_z = 2, P_z = 8, tolerance 1e-6: the library's
    FPCG iterations equal the oracle's (within one) and stay within a narrow band over P_x."""
    its = {}
    for Px in (2, 4, 6, 8, 10):
        wl = W.tank_semi(200, 2, Px, 8, Lx=50.0, name=f"sweep{Px}")
        s = cases.make_solver(wl, prec="bf16")
        b = cases.make_rhs(wl, s)
        x, info, _ = s.solve(b, tol=1e-6)
        its[Px] = info.iters
        s.close()
    print(f"[gpu] semi sweep iterations {its}", flush=True)
    assert max(its.values()) - min(its.values()) <= 2, its


def test_semi_rejects_schwarz_and_learned_stage():
    wl = CASES["semi_x"]
    with pytest.raises(B.SemError):
        cases.make_solver(wl, smoother="asm")
    s = lib_solver("semi_x", prec="f32")
    n = (wl.P + 1) * (wl.pz + 1)
    nin, nh = 5 * n, 128
    z = np.zeros
    blob = B.blob_pack(nin, n, z((nin, nh)), z(nh), z((nh, nh)), z(nh), z((nh, n)), z(n))
    with pytest.raises(B.SemError) as e:
        s.learned_load(blob, enable=1)
    assert "equal orders" in str(e.value)
    s.close()
