"""GPU parity at the benchmark sizes, in the launch configuration the benchmark times.

The 1024 x 16 and 2048 x 16 element tanks at P = 8 (1.06M and 2.11M nodes) are where the
operator runs two element columns per workgroup in the XCD-aware order; the small parity meshes
run one.  The oracle side is its matrix-free FP64 product (the assembled matrix would not fit a
test), checked against the assembled matrix by the oracle's own tests.  Bars as in
test_gpu_parity: FP64 1e-12, FP32 2e-6, BF16 factors 1e-2 (relative, max norm); the solve is
judged by the oracle's residual of the returned pressure and by its distance to the FP64 solve.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble
from tests import oracle_cases as oc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_14977_amd import cases  # noqa: E402

SIZES = {"c4": W.c4(0), "c3": W.c3()}
BARS = {"f64": 1e-12, "f32": 2e-6, "bf16": 1e-2, "col": 2e-6}


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(SIZES))
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "col"])
def test_operator_fullsize_all_levels(name, prec):
    wl = SIZES[name]
    print(f"[gpu] full-size operator {name} {prec}", flush=True)
    s = cases.make_solver(wl, prec=prec)
    for l, p in enumerate(wl.orders):
        m = oc.fine_mesh(wl, P=p)
        x = W.random_vector(m.N, 300 + l)
        ref = assemble.apply_matrix_free(m, x)
        y = H(s.apply_level(l, T(x)))
        bar = BARS["f64"] if l == len(wl.orders) - 1 else BARS[prec]
        assert rel(y, ref) <= bar, (name, prec, l, rel(y, ref))
        if l == 0:
            assert rel(H(s.apply(T(x))), ref) <= BARS["f64"]  # the FP64 outer operator
    s.close()


def test_mixed_solve_fullsize_c4():
    wl = SIZES["c4"]
    print("[gpu] full-size solve c4", flush=True)
    res = {}
    m = oc.fine_mesh(wl)
    bh = oc.rhs(wl, m)  # the oracle's right-hand side, fed to both solves
    for prec in ("f64", "bf16"):
        s = cases.make_solver(wl, prec=prec)
        x, info, _ = s.solve(T(bh), tol=1e-10)
        xh = H(x)
        r = bh - assemble.apply_matrix_free(m, xh)
        res[prec] = (xh, float(np.linalg.norm(r) / np.linalg.norm(bh)), info.iters)
        s.close()
    print(f"[gpu] oracle residuals {res['f64'][1]:.2e} (fp64), {res['bf16'][1]:.2e} (bf16), "
          f"iterations {res['f64'][2]}, {res['bf16'][2]}", flush=True)
    assert res["f64"][1] <= 1.5e-10 and res["bf16"][1] <= 1.5e-10
    d = np.linalg.norm(res["bf16"][0] - res["f64"][0]) / np.linalg.norm(res["f64"][0])
    assert d <= 1e-8, d
