"""GPU parity of the mixed-stage outer operator (Sec. 3.1 eq. poissonp, eq. weak4: stage k's
divergence of stage k-1's gradient) against the oracle, through the C ABI: the operator (FP64,
1e-12), GMRES and PDC solves against the oracle's direct solve of the non-symmetric system
(1e-9), FPCG refused, and the return to the same-stage operator."""
import math

import numpy as np
import pytest

from oracle import assemble, mesh, mixed

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_14977_amd import binding as B  # noqa: E402


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = {"p6": (9, 2, 6, None), "semi": (7, 3, 6, 3)}


def setup(name, outer="gmres", prec="f64"):
    Nx, Nz, P, Pz = CASES[name]
    Lx = 0.2 * Nx
    x = B.fine_x_nodes(Nx, P, Lx)
    h = 0.45 - 0.1 * np.sin(math.pi * x / Lx)
    ek = 0.04 * np.sin(2 * math.pi * x / Lx + 0.3)
    ep = 0.03 * np.cos(2 * math.pi * x / Lx - 0.2)
    s = B.Solver(2, (Nx, 1, Nz), P, (Lx,), h, ek, prec=prec, outer=outer, order_z=Pz)
    mk = mesh.Mesh2D(Nx, Nz, P, Lx, h, ek, Pz=Pz)
    mp = mesh.Mesh2D(Nx, Nz, P, Lx, h, ep, Pz=Pz)
    return s, mk, mp, ep


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_operator_matches_oracle(name):
    s, mk, mp, ep = setup(name)
    s.mixed_stage(ep)
    A = mixed.assemble_operator(mk, mp)
    x = np.random.default_rng(5).standard_normal(mk.N)
    assert rel(H(s.apply(T(x))), A @ x) < 1e-12
    # back to the same-stage operator
    s.mixed_stage(None)
    assert rel(H(s.apply(T(x))), assemble.assemble_operator(mk) @ x) < 1e-12
    s.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("outer,prec", [("gmres", "f64"), ("gmres", "bf16"), ("pdc", "f64")])
def test_mixed_solve_matches_direct(name, outer, prec):
    s, mk, mp, ep = setup(name, outer=outer, prec=prec)
    s.mixed_stage(ep)
    A = mixed.assemble_operator(mk, mp)
    b = np.random.default_rng(7).standard_normal(mk.N)
    b[mk.dirichlet_nodes()] = 0.0
    x, info, st = s.solve(T(b), tol=1e-11)
    xd = assemble.solve_direct(A, b)
    print(f"[gpu] mixed-stage {name} {outer} {prec}: {info.iters} iterations", flush=True)
    assert info.rel_res <= 1e-11
    assert np.linalg.norm(H(x) - xd) <= 1e-9 * np.linalg.norm(xd)
    s.close()


def test_mixed_refuses_fpcg_and_ends_with_a_new_surface():
    s, mk, mp, ep = setup("p6", outer="fpcg")
    s.mixed_stage(ep)
    b = np.zeros(mk.N)
    b[3] = 1.0
    x, info, st = s.solve(T(b), tol=1e-10, check=False)
    assert st == 6
    # a surface update returns to the same-stage operator of the new surface
    s.update_surface(ep)
    x_ = np.random.default_rng(9).standard_normal(mk.N)
    assert rel(H(s.apply(T(x_))), assemble.assemble_operator(mp) @ x_) < 1e-12
    x, info, st = s.solve(T(b), tol=1e-10)
    assert st == 0
    s.close()
