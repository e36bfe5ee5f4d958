"""GMRES-MG outer iteration (right-preconditioned, restarted) through the C ABI against the
oracle's GMRES with the same V-cycle (same lambda_hat): iteration counts, residual histories and
the solution.  The GPU orthogonalises by classical Gram-Schmidt applied twice, the oracle by
modified Gram-Schmidt: equal in exact arithmetic, so the histories agree to rounding."""
import numpy as np
import pytest

import workloads as W
from oracle import assemble, pmg
from tests import oracle_cases as oc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - only on machines without a GPU
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_14977_amd import cases  # noqa: E402

CASES = {
    "tank8": W.tank(16, 4, 8, Lx=1.6, name="tank8"),
    "ragged": W.tank(13, 3, 5, Lx=25.6 * 13 / 256, name="ragged"),
    "c2": W.c2(),
}


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name,restart", [("tank8", 30), ("ragged", 30), ("c2", 30),
                                          ("tank8", 3)])
def test_gmres_matches_oracle(name, restart):
    print(f"[gpu] GMRES {name} restart {restart}", flush=True)
    wl = CASES[name]
    Hh = oc.hierarchy(wl)
    pmg.estimate_lambdas(Hh)
    L0 = Hh.levels[0]
    s = cases.make_solver(wl, outer="gmres", gmres_restart=restart)
    for l, L in enumerate(Hh.levels[:-1]):
        s.set_lambda(l, L.lam)
    b = cases.make_rhs(wl, s)
    bh = H(b)
    x, info, st = s.solve(b, tol=1e-10)
    assert st == 0 and info.rel_res <= 1e-10
    xo, it_o, hist_o = pmg.gmres(L0.A, bh, np.zeros(L0.N), Hh.vcycle, 1e-10, restart=restart)
    assert info.iters == it_o, (info.iters, it_o)
    hist = np.array(info.hist[:info.nhist])
    ho = np.array(hist_o)
    assert len(hist) == len(ho)
    assert np.all(np.abs(hist - ho) <= 1e-6 * ho + 1e-13), (hist, ho)
    xd = assemble.solve_direct(L0.A, bh)
    assert np.linalg.norm(H(x) - xd) <= 1e-8 * np.linalg.norm(xd)
    s.close()


def test_gmres_mixed_precision_and_edge_cases():
    wl = CASES["c2"]
    s = cases.make_solver(wl, prec="bf16", outer="gmres")
    b = cases.make_rhs(wl, s)
    x, info, st = s.solve(b, tol=1e-10)
    assert st == 0 and info.rel_res <= 1e-10
    Hh = oc.hierarchy(wl)
    L0 = Hh.levels[0]
    xd = assemble.solve_direct(L0.A, H(b))
    assert np.linalg.norm(H(x) - xd) <= 1e-8 * np.linalg.norm(xd)
    # converged initial guess: no iteration; maxit reached: status 4 with the last iterate
    x2, info2, _ = s.solve(b, x=x.clone(), tol=1e-8)
    assert info2.iters == 0
    s.close()
    s2 = cases.make_solver(wl, outer="gmres", maxit=2)
    _, info3, st3 = s2.solve(b, tol=1e-14, check=False)
    assert st3 == 4 and info3.iters == 2
    s2.close()
    with pytest.raises(Exception):
        cases.make_solver(wl, outer="gmres", gmres_restart=65)


@pytest.mark.parametrize("name,cdm", [("t3a", 1200), ("t3h", 40)])
def test_gmres_3d_matches_oracle(name, cdm):
    """3D (p-levels, and an h-level below P = 1): the same parity as in 2D."""
    print(f"[gpu] GMRES 3D {name}", flush=True)
    wl = {"t3a": W.tank3d(4, 3, 2, 4, L=0.8, name="t3a"),
          "t3h": W.tank3d(4, 4, 2, 2, L=0.8, name="t3h")}[name]
    Hh = oc.hierarchy(wl, coarse_dense_max=cdm)
    pmg.estimate_lambdas(Hh)
    L0 = Hh.levels[0]
    s = cases.make_solver(wl, coarse_dense_max=cdm, outer="gmres", gmres_restart=30)
    for l, L in enumerate(Hh.levels[:-1]):
        s.set_lambda(l, L.lam)
    b = cases.make_rhs(wl, s)
    bh = H(b)
    x, info, st = s.solve(b, tol=1e-10)
    assert st == 0 and info.rel_res <= 1e-10
    xo, it_o, hist_o = pmg.gmres(L0.A, bh, np.zeros(L0.N), Hh.vcycle, 1e-10, restart=30)
    assert info.iters == it_o, (info.iters, it_o)
    hist = np.array(info.hist[:info.nhist])
    ho = np.array(hist_o)
    assert np.all(np.abs(hist - ho) <= 1e-6 * ho + 1e-13), (hist, ho)
    xd = assemble.solve_direct(L0.A, bh)
    assert np.linalg.norm(H(x) - xd) <= 1e-8 * np.linalg.norm(xd)
    s.close()
