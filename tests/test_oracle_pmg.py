"""Pins of the oracle's p-multigrid pieces: transfers, smoothers, V-cycle, outer iterations."""
import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import assemble, pmg
from tests import oracle_cases as oc


def _tank(Nx=4, Nz=2, P=4, **kw):
    wl = W.tank(Nx, Nz, P, Lx=25.6 * Nx / 256)
    return wl, oc.hierarchy(wl, **kw)


def dense_B(H):
    n = H.levels[0].N
    B = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        B[:, k] = H.vcycle(e)
    return B


def test_orders():
    assert pmg.coarsen_orders(8) == [8, 4, 2, 1]
    assert pmg.coarsen_orders(6) == [6, 3, 2, 1]
    assert pmg.coarsen_orders(4) == [4, 2, 1]
    assert pmg.coarsen_orders(1) == [1]


def test_prolongation_reproduces_polynomials_in_reference_coordinates():
    wl, H = _tank(Nx=3, Nz=2, P=6, smoother="jacobi")
    for l in range(len(H.orders) - 1):
        mf, mc = H.levels[l].mesh, H.levels[l + 1].mesh
        pc = H.orders[l + 1]

        def glob(m, F):
            out = np.zeros(m.N)
            out[m.l2g.ravel()] = F.reshape(m.E, -1).ravel()
            return out

        for a in range(pc + 1):
            for b in range(pc + 1 - a if pc > 1 else 2):
                fc = glob(mc, mc.X ** a * mc.SIG ** b)
                ff = glob(mf, mf.X ** a * mf.SIG ** b)
                assert np.abs(H.prolong(l, fc) - ff).max() < 1e-11 * max(1.0, np.abs(ff).max())


def test_single_level_is_exact_inverse():
    wl = W.tank(4, 2, 1, Lx=0.4)
    H = oc.hierarchy(wl)
    A = H.levels[0].A.toarray()
    B = dense_B(H)
    assert np.abs(B @ A - np.eye(A.shape[0])).max() < 1e-10


def test_no_smoothing_is_coarse_galerkin_correction():
    wl, H = _tank(Nx=3, Nz=2, P=2, smoother="jacobi", nu_pre=0, nu_post=0)
    P = H.P[0].toarray()
    Ac = H.levels[1].A.toarray()
    Z = np.eye(Ac.shape[0])
    Z[H.levels[1].dn, H.levels[1].dn] = 0.0
    B_ref = P @ np.linalg.solve(Ac, Z @ P.T)
    assert np.abs(dense_B(H) - B_ref).max() < 1e-12 * np.abs(B_ref).max()


@pytest.mark.parametrize("smoother", ["jacobi", "chebyshev"])
def test_vcycle_symmetric(smoother):
    wl, H = _tank(Nx=3, Nz=2, P=4, smoother=smoother)
    pmg.estimate_lambdas(H)
    B = dense_B(H)
    assert np.abs(B - B.T).max() < 1e-10 * np.abs(B).max()
    # and positive definite on the free space
    free = np.setdiff1d(np.arange(B.shape[0]), H.levels[0].dn)
    np.linalg.cholesky(0.5 * (B + B.T)[np.ix_(free, free)])


def _smoother_matrix(H, fn, level=0):
    """Error propagation of a smoother: x_out = E x_in for b = 0."""
    n = H.levels[level].N
    E = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        E[:, k] = fn(np.zeros(n), e)
    return E


def test_chebyshev_is_the_scaled_chebyshev_polynomial():
    """On each eigenvector of D^{-1}A with eigenvalue lam the Chebyshev smoother multiplies
    the error by T_k((theta - lam)/delta) / T_k(theta/delta) exactly."""
    wl, H = _tank(Nx=2, Nz=2, P=3)
    L = H.levels[0]
    L.lam = 2.3
    k = 3
    E = _smoother_matrix(H, lambda b, x: H.chebyshev(0, b, x, k))
    A = L.A.toarray()
    Dm = np.diag(L.dinv)
    lam, V = np.linalg.eig(Dm @ A)
    lam, V = lam.real, V.real
    a, b = H.cheb_lo * L.lam, H.cheb_hi * L.lam
    theta, delta = (a + b) / 2, (b - a) / 2
    Tk = npcheb.Chebyshev.basis(k)
    for j in range(lam.size):
        expect = Tk((theta - lam[j]) / delta) / Tk(theta / delta)
        assert np.abs(E @ V[:, j] - expect * V[:, j]).max() < 1e-9


def test_level_degrees_in_the_smoother():
    """With a coarse degree set, the smoother of every level between the finest and the
    coarsest is that degree's scaled Chebyshev polynomial on each eigenvector (the finest keeps
    its own degree)."""
    wl, H = _tank(Nx=4, Nz=2, P=4, cheb_degree=5, cheb_degree_coarse=2)
    for l, k in ((0, 5), (1, 2)):
        L = H.levels[l]
        L.lam = 2.1
        E = _smoother_matrix(H, lambda b, x: H.smooth(l, b, x, pre=True), level=l)
        lam, V = np.linalg.eig(np.diag(L.dinv) @ L.A.toarray())
        lam, V = lam.real, V.real
        a, b = H.cheb_lo * L.lam, H.cheb_hi * L.lam
        theta, delta = (a + b) / 2, (b - a) / 2
        Tk = npcheb.Chebyshev.basis(k)
        for j in range(lam.size):
            expect = Tk((theta - lam[j]) / delta) / Tk(theta / delta)
            assert np.abs(E @ V[:, j] - expect * V[:, j]).max() < 1e-9, (l, j)


def test_jacobi_error_propagation():
    wl, H = _tank(Nx=2, Nz=2, P=3, smoother="jacobi")
    L = H.levels[0]
    E = _smoother_matrix(H, lambda b, x: H.jacobi(0, b, x, 2))
    M = np.eye(L.N) - H.omega * np.diag(L.dinv) @ L.A.toarray()
    assert np.abs(E - M @ M).max() < 1e-12


def test_fpcg_equals_pcg_for_linear_preconditioner():
    wl, H = _tank(Nx=4, Nz=2, P=4)
    pmg.estimate_lambdas(H)
    L = H.levels[0]
    b = W.random_vector(L.N, 1)
    b[L.dn] = 0.0
    x1, it1, h1 = pmg.pcg(L.A, b, np.zeros(L.N), H.vcycle, 1e-10)
    x2, it2, h2 = pmg.fpcg(L.A, b, np.zeros(L.N), H.vcycle, 1e-10)
    assert it1 == it2
    assert np.abs(np.array(h1) - np.array(h2)).max() < 1e-9
    assert np.abs(x1 - x2).max() < 1e-10 * np.abs(x1).max()


def test_lanczos_estimate_vs_dense_eigenvalue():
    wl, H = _tank(Nx=3, Nz=2, P=4)
    L = H.levels[0]
    lam_true = np.linalg.eigvals(np.diag(L.dinv) @ L.A.toarray()).real.max()
    v0 = pmg.splitmix64_uniform(L.N, 12345)
    v0[L.dn] = 0.0
    lam = pmg.lanczos_lambda_max(L.A, L.dinv, v0, steps=20)
    assert lam <= lam_true * (1 + 1e-12)
    assert lam > 0.97 * lam_true


def test_splitmix64_reference_values():
    # SplitMix64 with state 0: first outputs 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4
    # (published reference sequence); our mapping uses the top 53 bits.
    v = pmg.splitmix64_uniform(2, 0)
    ref = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]
    for got, r in zip(v, ref):
        assert got == (r >> 11) * (1.0 / (1 << 53)) * 2.0 - 1.0


def test_solve_to_tolerance_matches_direct_and_flat_iterations():
    its = []
    for Nx in (8, 16, 32):
        wl = W.tank(Nx, 2, 4, Lx=25.6 * Nx / 64)
        H = oc.hierarchy(wl)
        pmg.estimate_lambdas(H)
        L = H.levels[0]
        b = oc.rhs(wl, L.mesh)
        x, it, hist = pmg.fpcg(L.A, b, np.zeros(L.N), H.vcycle, 1e-10)
        xd = assemble.solve_direct(L.A, b)
        assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
        its.append(it)
    assert max(its) - min(its) <= 4


def test_pdc_converges():
    wl = W.c1(4)
    H = oc.hierarchy(wl)
    L = H.levels[0]
    b = oc.rhs(wl, L.mesh)
    x, it, hist = pmg.pdc(L.A, b, np.zeros(L.N), H.vcycle, 1e-10)
    assert hist[-1] <= 1e-10 and it < 60
    assert np.linalg.norm(x - assemble.solve_direct(L.A, b)) < 1e-8 * np.linalg.norm(x)


# ---- 3D: levels below P = 1 (mesh coarsened in x and y) --------------------------------------
def _tank3d(Nx=4, Ny=4, Nz=2, P=2, **kw):
    wl = W.tank3d(Nx, Ny, Nz, P, L=0.8)
    return wl, oc.hierarchy(wl, **kw)


def test_linear_prolongation_reproduces_linear_functions():
    for Nc in (1, 2, 5):
        Pl = pmg.prolongation_1d_linear(Nc).toarray()
        xc = np.linspace(0.0, 1.0, Nc + 1)
        xf = np.linspace(0.0, 1.0, 2 * Nc + 1)
        for f in (np.ones_like, lambda t: t, lambda t: 3.0 * t - 1.0):
            assert np.abs(Pl @ f(xc) - f(xf)).max() < 1e-15
        # exactly one unit entry per even row, two halves per odd row
        assert np.allclose(Pl.sum(axis=1), 1.0)


def test_h_levels_3d_structure_and_linear_reproduction():
    wl, H = _tank3d(coarse_dense_max=40, smoother="jacobi")
    # P = 2 (405 nodes), P = 1 (75 > 40) -> one h-level 2 x 2 x 2 at P = 1 (27 nodes)
    assert [L.mesh.P for L in H.levels] == [2, 1, 1]
    assert [L.N for L in H.levels] == [405, 75, 27]
    mf, mc = H.levels[1].mesh, H.levels[2].mesh
    # the coarse vertices are fine vertices: same coordinates there
    xf, yf, zf = mf.node_coords()
    xc, yc, zc = mc.node_coords()
    sel = np.array([((2 * ix) * mf.ny_nodes + 2 * iy) * mf.nz_nodes + iz
                    for ix in range(mc.nx_nodes) for iy in range(mc.ny_nodes)
                    for iz in range(mc.nz_nodes)])
    assert np.abs(xf[sel] - xc).max() < 1e-14 and np.abs(yf[sel] - yc).max() < 1e-14
    assert np.abs(zf[sel] - zc).max() < 1e-14
    # prolongation of a function linear in (x, y) and arbitrary in sigma-level index is exact
    for a, b in ((1.0, 0.0), (0.3, -2.0)):
        kz = np.arange(mc.nz_nodes)
        fc = (a * xc + b * yc) * (1 + kz[np.arange(mc.N) % mc.nz_nodes])
        kf = np.arange(mf.N) % mf.nz_nodes
        ff = (a * xf + b * yf) * (1 + kf)
        assert np.abs(H.prolong(1, fc) - ff).max() < 1e-13


def test_h_levels_3d_no_smoothing_is_composed_coarse_correction():
    wl, H = _tank3d(Nx=2, Ny=2, Nz=1, P=2, coarse_dense_max=10, smoother="jacobi", nu_pre=0,
                    nu_post=0)
    assert len(H.levels) == 3
    P0, P1 = H.P[0].toarray(), H.P[1].toarray()
    Ac = H.levels[2].A.toarray()
    Z1 = np.eye(H.levels[1].N)
    Z1[H.levels[1].dn, H.levels[1].dn] = 0.0
    Z2 = np.eye(Ac.shape[0])
    Z2[H.levels[2].dn, H.levels[2].dn] = 0.0
    B_ref = P0 @ P1 @ np.linalg.solve(Ac, Z2 @ P1.T @ Z1 @ P0.T)
    assert np.abs(dense_B(H) - B_ref).max() < 1e-12 * np.abs(B_ref).max()


def test_h_levels_3d_vcycle_symmetric_and_solve_matches_direct():
    wl, H = _tank3d(coarse_dense_max=40)
    pmg.estimate_lambdas(H)
    B = dense_B(H)
    assert np.abs(B - B.T).max() < 1e-10 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    m = H.levels[0].mesh
    b = oc.rhs(wl, m)
    x, it, _ = pmg.fpcg(H.levels[0].A, b, np.zeros(m.N), H.vcycle, 1e-12)
    xd = assemble.solve_direct(H.levels[0].A, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


# ---- additive Schwarz smoother (Sec. 5.3) -----------------------------------------------
def test_schwarz_one_element_is_the_exact_solve():
    # a single element block holds every node and W = 1: one sweep solves A x = b exactly
    wl = W.tank(1, 1, 4, Lx=0.1)
    H = oc.hierarchy(wl, smoother="asm", nu_pre=1, nu_post=1)
    L = H.levels[0]
    b = W.random_vector(L.N, 3)
    b[L.dn] = 0.0
    x = H.schwarz_sweeps(0, b, np.zeros(L.N), 1)
    xd = np.linalg.solve(L.A.toarray(), b)
    assert np.abs(x - xd).max() < 1e-11 * np.abs(xd).max()


def test_schwarz_unweighted_sum_is_symmetric_and_weights_partition_unity():
    wl, H = _tank(Nx=3, Nz=2, P=3, smoother="asm")
    L = H.levels[0]
    n = L.N
    S0 = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        S0[:, k] = L.schwarz(e, weighted=False)
    assert np.abs(S0 - S0.T).max() < 1e-11 * np.abs(S0).max()
    inv, w = L.schwarz_blocks()[:2]
    counts = np.zeros(n)
    for idx in L.mesh.l2g:
        counts[idx] += 1.0
    assert np.array_equal(w * counts, np.ones(n))
    assert set(np.unique(counts)) <= {1.0, 2.0, 4.0}


def test_schwarz_matches_dense_construction_with_explicit_restrictions():
    # S^{-1} = W sum_i R_i^T (R_i A R_i^T)^{-1} R_i with R_i as 0/1 matrices and W as a dense
    # inverse (cross-check of the index bookkeeping, not of the formula)
    wl, H = _tank(Nx=2, Nz=2, P=2, smoother="asm")
    L = H.levels[0]
    A = L.A.toarray()
    n = L.N
    Rs = []
    for idx in L.mesh.l2g:
        R = np.zeros((len(idx), n))
        R[np.arange(len(idx)), idx] = 1.0
        Rs.append(R)
    Wd = np.linalg.inv(sum(R @ R.T for R in [r.T for r in Rs]))
    S = Wd @ sum(R.T @ np.linalg.inv(R @ A @ R.T) @ R for R in Rs)
    r = W.random_vector(n, 5)
    assert np.abs(L.schwarz(r) - S @ r).max() < 1e-12 * np.abs(S @ r).max()


def test_schwarz_preconditioned_solve_matches_direct():
    wl, H = _tank(Nx=6, Nz=2, P=4, smoother="asm", nu_pre=1, nu_post=1)
    L = H.levels[0]
    b = W.random_vector(L.N, 7)
    b[L.dn] = 0.0
    x, it, hist = pmg.fpcg(L.A, b, np.zeros(L.N), H.vcycle, 1e-10)
    xd = assemble.solve_direct(L.A, b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    assert it <= 30


def _small_system(n=40, seed=3):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)          # SPD
    N = rng.standard_normal((n, n))
    Bm = np.diag(1.0 / np.diag(A)) + 0.01 * (N + N.T) / n   # a fixed linear preconditioner
    b = rng.standard_normal(n)
    return A, Bm, b


def test_gmres_minimises_residual_over_krylov_space():
    """Pin (definition): the k-th GMRES iterate is the minimum-residual point of
    x0 + span{B r0, (B A) B r0, ..} = x0 + B K_k(A B, r0), here built explicitly and solved by
    least squares."""
    A, Bm, b = _small_system()
    x0 = np.zeros_like(b)
    r0 = b - A @ x0
    for k in range(1, 7):
        xg, it, _ = pmg.gmres(A, b, x0, lambda v: Bm @ v, 1e-30, restart=30, maxit=k)
        assert it == k
        K = [r0]
        for _ in range(k - 1):
            K.append(A @ (Bm @ K[-1]))
        Zk = Bm @ np.column_stack(K)
        y = np.linalg.lstsq(A @ Zk, r0, rcond=None)[0]
        xb = x0 + Zk @ y
        assert np.linalg.norm(xg - xb) <= 1e-9 * np.linalg.norm(xb)


def test_gmres_exact_preconditioner_and_restart():
    """With B = A^-1 one step is exact; restarted GMRES(2) never increases the residual and
    converges; zero initial residual returns at once."""
    A, Bm, b = _small_system()
    Ainv = np.linalg.inv(A)
    x, it, hist = pmg.gmres(A, b, np.zeros_like(b), lambda v: Ainv @ v, 1e-12)
    assert it == 1 and hist[-1] <= 1e-12
    x, it, hist = pmg.gmres(A, b, np.zeros_like(b), lambda v: Bm @ v, 1e-10, restart=2, maxit=400)
    assert hist[-1] <= 1e-10
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    x, it, hist = pmg.gmres(A, b, xs, lambda v: Bm @ v, 1e-8)
    assert it == 0


def test_gmres_with_vcycle_on_tank():
    """GMRES-MG on a small sigma-mapped tank reaches the direct solution; with the same V-cycle
    it needs no more iterations than flexible CG (GMRES minimises the residual norm)."""
    wl = W.tank(16, 4, 4, Lx=1.6, name="gm")
    H_ = oc.hierarchy(wl)
    pmg.estimate_lambdas(H_)
    L0 = H_.levels[0]
    b = W.random_vector(L0.N, 77)
    b[L0.dn] = 0.0
    xs = spla.spsolve(L0.A.tocsc(), b)
    xg, itg, hg = pmg.gmres(L0.A, b, np.zeros(L0.N), H_.vcycle, 1e-10)
    xc, itc, hc = pmg.fpcg(L0.A, b, np.zeros(L0.N), H_.vcycle, 1e-10)
    assert hg[-1] <= 1e-10
    assert np.linalg.norm(xg - xs) <= 1e-8 * np.linalg.norm(xs)
    assert itg <= itc


def test_vcycle_stage_placements():
    """The two stage positions of the V-cycle (used by the learned stage): ``hook`` acts after the
    finest pre-smoothing, before the residual that is restricted; ``hook_post`` after the coarse
    correction is added, before the post-smoothing.  Checked through the V-cycle's affine
    structure: a stage that adds a fixed vector v changes the result by the post-smoothing's error
    propagation applied to v (after the post position), or to v minus its coarse-grid correction
    (after the pre position); a stage that returns the exact solution makes B = A^-1."""
    wl, H = _tank(Nx=3, Nz=2, P=4)
    pmg.estimate_lambdas(H)
    L0 = H.levels[0]
    rng = np.random.default_rng(3)
    b = rng.standard_normal(L0.N)
    b[L0.dn] = 0.0
    v = rng.standard_normal(L0.N)
    v[L0.dn] = 0.0
    z0 = H.vcycle(b)
    zero = np.zeros(L0.N)

    def post_smooth_error(e):          # post-smoothing of x = e with b = 0
        return H.smooth(0, zero, e, pre=False)

    seen = {}

    def add_pre(l, bb, x):
        if l == 0:
            seen["pre"] = x.copy()
            return x + v
        return x

    def add_post(l, bb, x):
        if l == 0:
            seen["post"] = x.copy()
            return x + v
        return x

    z_post = H.vcycle(b, hook_post=add_post)
    assert np.abs(z_post - (z0 + post_smooth_error(v))).max() < 1e-12 * np.abs(z0).max()
    z_pre = H.vcycle(b, hook=add_pre)
    ec = H.vcycle(H.restrict(0, L0.A @ v), 1)
    ref = z0 + post_smooth_error(v - H.prolong(0, ec))
    assert np.abs(z_pre - ref).max() < 1e-12 * np.abs(z0).max()
    assert np.abs(seen["pre"] - H.smooth(0, b, zero, pre=True)).max() < 1e-14 * np.abs(b).max()
    # the post position sees the pre-smoothed iterate plus the prolonged coarse correction
    xpre = H.smooth(0, b, zero, pre=True)
    ecb = H.vcycle(H.restrict(0, b - L0.A @ xpre), 1)
    assert np.abs(seen["post"] - (xpre + H.prolong(0, ecb))).max() < 1e-12 * np.abs(z0).max()
    xs = spla.spsolve(L0.A.tocsc(), b)
    for kw in ("hook", "hook_post"):
        z = H.vcycle(b, **{kw: (lambda l, bb, x: xs if l == 0 else x)})
        assert np.abs(z - xs).max() < 1e-10 * np.abs(xs).max(), kw
    # identity stages leave the V-cycle unchanged
    ident = (lambda l, bb, x: x)
    assert np.array_equal(H.vcycle(b, hook=ident, hook_post=ident), z0)


def test_stored_factor_rounding_levels():
    """gstore rounds the factors of every level above the coarsest (the coarsest stays exact), and
    the operator built from them differs from the exact one by the rounding's relative size."""
    from oracle import precision
    wl = W.tank(4, 2, 4, Lx=0.4)
    He = oc.hierarchy(wl)
    Hb = oc.hierarchy(wl, gstore="bf16")
    Hf = oc.hierarchy(wl, gstore="f32")
    for l in range(len(He.levels)):
        Ae, Ab, Af = He.levels[l].A, Hb.levels[l].A, Hf.levels[l].A
        d = abs(Ab - Ae).max() / abs(Ae).max()
        df = abs(Af - Ae).max() / abs(Ae).max()
        if l == len(He.levels) - 1:
            assert d == 0 and df == 0
        else:
            assert 1e-5 < d < 2 ** -7 * 4 and 0 < df < 1e-6
    m = Hb.levels[0].mesh
    mb = precision.with_stored_factors(m, "bf16")
    assert np.array_equal(mb.Grs, precision.bf16(m.Grs)) and mb.Grs is not m.Grs
    assert mb.mass is m.mass and np.array_equal(m.Grs, He.levels[0].mesh.Grs)
