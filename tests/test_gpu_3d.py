"""GPU parity of the 3D path (sigma-mapped hexahedra) against the CPU oracle, through the C ABI.

Hierarchy: p-levels as in 2D, then levels coarsened by 2 in x and y at P = 1 until at most
``coarse_dense_max`` nodes remain (solved exactly); the oracle builds the same hierarchy.
Bars as in 2D: FP64 steps within 1e-12 (relative, max norm), FP32 operator 2e-6, BF16 factors
1e-2, solves within 1e-9 (FP64) and 1e-8 (mixed precision) of the oracle's direct solution.
The 64 x 64 x 8, P = 6 tank (7.26M nodes) is checked against the oracle's matrix-free product
and by the oracle's residual of a full solve.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble, pmg
from tests import oracle_cases as oc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_14977_amd import binding as B  # noqa: E402
from paper_2411_14977_amd import cases  # noqa: E402

# name -> (workload, coarse_dense_max)
CASES3 = {
    "t3a": (W.tank3d(4, 3, 2, 4, L=0.8, name="t3a"), 1200),           # Nx != Ny, 4-2-1
    "t3h": (W.tank3d(4, 4, 2, 2, L=0.8, name="t3h"), 40),             # one h-level below P = 1
    "t3hh": (W.tank3d(8, 4, 1, 2, L=0.8, name="t3hh"), 20),           # two h-levels
    "t3p6": (W.tank3d(2, 2, 2, 6, L=0.8, orders=[6, 3, 1], name="t3p6"), 1200),
    "t3odd": (W.tank3d(3, 2, 3, 3, L=0.8, name="t3odd"), 1200),       # odd P, odd counts
    # P = 8 -> 4: restriction rows of 17 entries take the general transfer kernel
    "t3p8": (W.tank3d(2, 1, 1, 8, L=0.8, name="t3p8"), 1200),
}

_oracle = {}


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_h(name):
    if name not in _oracle:
        wl, cdm = CASES3[name]
        Ho = oc.hierarchy(wl, coarse_dense_max=cdm)
        pmg.estimate_lambdas(Ho)
        _oracle[name] = Ho
    return _oracle[name]


def lib_solver(name, prec="f64", **kw):
    wl, cdm = CASES3[name]
    return cases.make_solver(wl, prec=prec, coarse_dense_max=cdm, **kw)


@pytest.mark.parametrize("name", list(CASES3))
def test_hierarchy_matches_oracle(name):
    Ho = oracle_h(name)
    s = lib_solver(name)
    assert s.nlevels == len(Ho.levels)
    for l, L in enumerate(Ho.levels):
        order, n, _ = s.level(l)
        assert (order, n) == (L.mesh.P, L.N), (name, l)
    s.close()


@pytest.mark.parametrize("name", list(CASES3))
def test_operator_3d_fp64_all_levels(name):
    print(f"[gpu] 3D operator parity {name}", flush=True)
    Ho = oracle_h(name)
    s = lib_solver(name)
    for l, L in enumerate(Ho.levels):
        x = W.random_vector(L.N, 100 + l)
        assert rel(H(s.apply_level(l, T(x))), L.A @ x) < 1e-12, (name, l)
    x = W.random_vector(Ho.levels[0].N, 7)
    assert rel(H(s.apply(T(x))), Ho.levels[0].A @ x) < 1e-12
    s.close()


@pytest.mark.parametrize("prec,bar", [("f32", 2e-6), ("bf16", 1e-2), ("col", 2e-6)])
def test_operator_3d_inner_precision(prec, bar):
    Ho = oracle_h("t3a")
    s = lib_solver("t3a", prec=prec)
    for l, L in enumerate(Ho.levels[:-1]):
        x = W.random_vector(L.N, 200 + l)
        ref = L.A @ x
        assert np.abs(H(s.apply_level(l, T(x))) - ref).max() <= bar * np.abs(ref).max(), (prec, l)
    s.close()


def test_pure_neumann_3d():
    wl, _ = CASES3["t3odd"]
    s = cases.make_solver(wl, dirichlet=False)
    m = oc.fine_mesh(wl)
    A = assemble.assemble_operator(m, dirichlet=False)
    x = W.random_vector(m.N, 3)
    assert rel(H(s.apply(T(x))), A @ x) < 1e-12
    assert np.abs(H(s.apply(T(np.ones(m.N))))).max() < 1e-12 * abs(A).max()
    s.close()


@pytest.mark.parametrize("name", list(CASES3))
def test_transfers_3d(name):
    Ho = oracle_h(name)
    s = lib_solver(name)
    for l in range(len(Ho.levels) - 1):
        Lf, Lc = Ho.levels[l], Ho.levels[l + 1]
        b = W.random_vector(Lf.N, 300 + l)
        x = W.random_vector(Lf.N, 400 + l)
        b[Lf.dn] = 0.0
        rc = T(np.zeros(Lc.N))
        B.sem_restrict(s.ctx, l, T(b), T(x), rc)
        assert rel(H(rc), Ho.restrict(l, b - Lf.A @ x)) < 1e-12, (name, l)
        B.sem_restrict(s.ctx, l, T(b), None, rc)
        assert rel(H(rc), Ho.restrict(l, b)) < 1e-12
        ec = W.random_vector(Lc.N, 500 + l)
        ec[Lc.dn] = 0.0
        xf = T(x.copy())
        B.sem_prolong_add(s.ctx, l, T(ec), xf)
        assert rel(H(xf), x + Ho.prolong(l, ec)) < 1e-12, (name, l)
    s.close()


@pytest.mark.parametrize("name", list(CASES3))
def test_coarse_solve_3d_exact(name):
    Ho = oracle_h(name)
    s = lib_solver(name)
    Lc = Ho.levels[-1]
    b = W.random_vector(Lc.N, 600)
    b[Lc.dn] = 0.0
    x = T(np.zeros(Lc.N))
    B.sem_coarse_solve(s.ctx, T(b), x)
    assert rel(H(x), Ho.coarse_solve(b)) < 1e-11
    s.close()


@pytest.mark.parametrize("name", list(CASES3))
def test_vcycle_3d(name):
    Ho = oracle_h(name)
    s = lib_solver(name)
    for l, L in enumerate(Ho.levels[:-1]):
        s.set_lambda(l, L.lam)
    L0 = Ho.levels[0]
    r = W.random_vector(L0.N, 900)
    r[L0.dn] = 0.0
    assert rel(H(s.vcycle(T(r))), Ho.vcycle(r)) < 1e-12
    s.close()


def test_lanczos_3d():
    Ho = oracle_h("t3h")
    s = lib_solver("t3h")
    for l, L in enumerate(Ho.levels[:-1]):
        lam = s.level(l)[2]
        assert abs(lam - L.lam) <= 1e-10 * L.lam, (l, lam, L.lam)
    s.close()


@pytest.mark.parametrize("name", ["t3a", "t3h", "t3p6"])
def test_rhs_assembly_3d(name):
    wl, _ = CASES3[name]
    s = lib_solver(name)
    m = oc.fine_mesh(wl)
    assert rel(H(cases.make_rhs(wl, s)), oc.rhs(wl, m)) < 1e-12
    s.close()


@pytest.mark.parametrize("name", ["t3a", "t3h", "t3hh", "t3p6"])
@pytest.mark.parametrize("prec,bar", [("f64", 1e-9), ("f32", 1e-8), ("bf16", 1e-8), ("col", 1e-8)])
def test_solve_3d_matches_direct(name, prec, bar):
    wl, _ = CASES3[name]
    Ho = oracle_h(name)
    A0 = Ho.levels[0].A
    b = oc.rhs(wl, Ho.levels[0].mesh)
    xd = assemble.solve_direct(A0, b)
    s = lib_solver(name, prec=prec)
    x, info, _ = s.solve(T(b), tol=1e-10)
    err = np.linalg.norm(H(x) - xd) / np.linalg.norm(xd)
    print(f"[gpu] 3D solve {name} {prec}: {info.iters} iterations, error {err:.2e}", flush=True)
    assert info.rel_res <= 1e-10 and err <= bar
    s.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "col"])
def test_operator_fullsize_c5(prec):
    wl = W.c5()
    print(f"[gpu] c5 operator {prec}", flush=True)
    s = cases.make_solver(wl, prec=prec)
    m = oc.fine_mesh(wl)
    x = W.random_vector(m.N, 11)
    ref = assemble.apply_matrix_free(m, x)
    bar = {"f64": 1e-12, "f32": 2e-6, "bf16": 1e-2, "col": 2e-6}[prec]
    assert rel(H(s.apply_level(0, T(x))), ref) <= bar
    assert rel(H(s.apply(T(x))), ref) <= 1e-12
    s.close()


def test_solve_fullsize_c5():
    wl = W.c5()
    m = oc.fine_mesh(wl)
    b = oc.rhs(wl, m)
    res = {}
    for prec in ("f64", "bf16"):
        s = cases.make_solver(wl, prec=prec)
        x, info, _ = s.solve(T(b), tol=1e-10)
        xh = H(x)
        r = b - assemble.apply_matrix_free(m, xh)
        res[prec] = (xh, float(np.linalg.norm(r) / np.linalg.norm(b)), info.iters)
        print(f"[gpu] c5 solve {prec}: {info.iters} iterations, oracle residual {res[prec][1]:.2e}",
              flush=True)
        s.close()
    assert res["f64"][1] <= 1.5e-10 and res["bf16"][1] <= 1.5e-10
    d = np.linalg.norm(res["bf16"][0] - res["f64"][0]) / np.linalg.norm(res["f64"][0])
    assert d <= 1e-8, d
