"""Pins of the oracle on 2D meshes whose x and sigma orders differ (semi-coarsening, Sec. 5.1).

Independent checks: geometric factors from the isoparametric map of the nodal coordinates, a
brute-force quadrature assembly, the Kronecker closed form on rectangles (1D stiffness from
Gauss-Legendre quadrature of the Lagrange basis), exact reproduction of harmonic polynomials,
spectral convergence in each direction separately, exact polynomial reproduction of the
semi-coarsened prolongations, and the V-cycle's algebraic properties (symmetry, the coarse
Galerkin correction without smoothing, solves that match a direct solve).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import assemble, gll, mesh, pmg
from tests import oracle_cases as oc


def test_semi_coarsened_orders():
    assert pmg.coarsen_orders_2d(16, 8) == [(16, 8), (8, 8), (4, 4), (2, 2), (1, 1)]
    assert pmg.coarsen_orders_2d(12, 8) == [(12, 8), (8, 8), (4, 4), (2, 2), (1, 1)]
    assert pmg.coarsen_orders_2d(2, 8) == [(2, 8), (2, 4), (2, 2), (1, 1)]
    assert pmg.coarsen_orders_2d(3, 8) == [(3, 8), (3, 4), (3, 3), (2, 2), (1, 1)]
    assert pmg.coarsen_orders_2d(5, 8) == [(5, 8), (5, 5), (3, 3), (2, 2), (1, 1)]
    assert pmg.coarsen_orders_2d(1, 4) == [(1, 4), (1, 2), (1, 1)]
    for P in (1, 4, 6, 8):
        assert pmg.coarsen_orders_2d(P, P) == [(p, p) for p in pmg.coarsen_orders(P)]


def _tank_mesh(Nx, Nz, Px, Pz, seed=7):
    wl = W.tank_semi(Nx, Nz, Px, Pz, Lx=25.6 * Nx / 64, surface_seed=seed)
    return oc.fine_mesh(wl)


def _iso_factors(m):
    """w_x w_sigma |J| J^{-1} J^{-T} from the nodal (x, z) by differentiating with each
    direction's own GLL differentiation matrix."""
    NP, NPz = m.NP, m.NPz
    X = m.X.reshape(m.E, NP, NPz)
    Z = m.Z.reshape(m.E, NP, NPz)
    Dx = gll.diff_matrix(m.P)
    Dz = gll.diff_matrix(m.Pz)
    xr = np.einsum("ik,ekj->eij", Dx, X)
    xs = np.einsum("jk,eik->eij", Dz, X)
    zr = np.einsum("ik,ekj->eij", Dx, Z)
    zs = np.einsum("jk,eik->eij", Dz, Z)
    J = xr * zs - xs * zr
    rx, rz = zs / J, -xs / J
    sx, sz = -zr / J, xr / J
    ww = np.outer(gll.gll_weights(m.P), gll.gll_weights(m.Pz))[None]
    return (ww * J * (rx * rx + rz * rz), ww * J * (rx * sx + rz * sz),
            ww * J * (sx * sx + sz * sz), ww * J)


@pytest.mark.parametrize("Px,Pz", [(2, 5), (6, 3), (8, 4), (3, 8)])
def test_unequal_orders_factors_match_isoparametric(Px, Pz):
    m = _tank_mesh(4, 3, Px, Pz)
    Grr, Grs, Gss, WJ = _iso_factors(m)
    sc = np.abs(Gss).max()
    assert np.abs(Grr - m.Grr).max() < 1e-12 * sc
    assert np.abs(Grs - m.Grs).max() < 1e-12 * sc
    assert np.abs(Gss - m.Gss).max() < 1e-12 * sc
    assert np.abs(WJ - m.mass).max() < 1e-14


def _brute_force_stiffness(m):
    """Dense stiffness by loops over elements, quadrature points and basis pairs, with the
    x rule of order P and the sigma rule of order Pz."""
    NP, NPz = m.NP, m.NPz
    Dx, Dz = gll.diff_matrix(m.P), gll.diff_matrix(m.Pz)
    wx, wz = gll.gll_weights(m.P), gll.gll_weights(m.Pz)
    K = np.zeros((m.N, m.N))
    X = m.X.reshape(m.E, NP, NPz)
    Z = m.Z.reshape(m.E, NP, NPz)
    for e in range(m.E):
        g = m.l2g[e].reshape(NP, NPz)
        for qi in range(NP):
            for qj in range(NPz):
                xr = sum(Dx[qi, k] * X[e, k, qj] for k in range(NP))
                xs = sum(Dz[qj, k] * X[e, qi, k] for k in range(NPz))
                zr = sum(Dx[qi, k] * Z[e, k, qj] for k in range(NP))
                zs = sum(Dz[qj, k] * Z[e, qi, k] for k in range(NPz))
                J = np.array([[xr, xs], [zr, zs]])
                Jit = np.linalg.inv(J).T
                wq = wx[qi] * wz[qj] * abs(np.linalg.det(J))
                grads = {}
                for a in range(NP):
                    for b in range(NPz):
                        dr = Dx[qi, a] if b == qj else 0.0
                        ds = Dz[qj, b] if a == qi else 0.0
                        if dr or ds:
                            grads[(a, b)] = Jit @ np.array([dr, ds])
                for (a, b), ga in grads.items():
                    for (c, d), gc in grads.items():
                        K[g[a, b], g[c, d]] += wq * ga @ gc
    return K


@pytest.mark.parametrize("Px,Pz", [(2, 4), (5, 2)])
def test_unequal_orders_bruteforce_assembly(Px, Pz):
    m = _tank_mesh(2, 2, Px, Pz)
    K = _brute_force_stiffness(m)
    A = assemble.assemble_stiffness(m).toarray()
    assert np.abs(K - A).max() < 1e-12 * np.abs(A).max()
    # symmetric, constants in the null space, masked operator SPD
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    assert np.abs(A @ np.ones(m.N)).max() < 1e-12 * np.abs(A).max()
    np.linalg.cholesky(assemble.masked(assemble.assemble_stiffness(m),
                                       m.dirichlet_nodes()).toarray())


def _khat(P):
    """1D reference stiffness int l_a' l_b' on [-1, 1] by Gauss-Legendre quadrature of the
    Lagrange basis through the GLL nodes (exact for polynomials of this degree)."""
    r = gll.gll_nodes(P)
    xg, wg = np.polynomial.legendre.leggauss(P + 2)
    L = np.zeros((P + 1, xg.size))
    for i in range(P + 1):
        c = np.polynomial.polynomial.polyfromroots(np.delete(r, i))
        c = c / np.polynomial.polynomial.polyval(r[i], c)
        L[i] = np.polynomial.polynomial.polyval(xg, np.polynomial.polynomial.polyder(c))
    return (L * wg) @ L.T


@pytest.mark.parametrize("Px,Pz", [(3, 6), (7, 2), (4, 4)])
def test_unequal_orders_rectangle_kronecker(Px, Pz):
    Nx, Nz, Lx, H = 3, 2, 3.0, 0.8
    m = oc.affine_mesh(Nx, Nz, Px, Lx, H, Pz=Pz)
    dx, dz = Lx / Nx, H / Nz
    Wx = np.diag(gll.gll_weights(Px))
    Wz = np.diag(gll.gll_weights(Pz))
    Ae_ref = (dz / dx) * np.kron(_khat(Px), Wz) + (dx / dz) * np.kron(Wx, _khat(Pz))
    Ae = assemble.element_matrices(m)
    assert Ae.shape == (Nx * Nz, (Px + 1) * (Pz + 1), (Px + 1) * (Pz + 1))
    assert np.abs(Ae - Ae_ref[None]).max() < 1e-12 * np.abs(Ae_ref).max()
    # the assembled 2D stiffness is the Kronecker sum of the assembled 1D matrices
    def assemble_1d(Ne, P, M):
        n = Ne * P + 1
        out = np.zeros((n, n))
        for e in range(Ne):
            out[e * P:e * P + P + 1, e * P:e * P + P + 1] += M
        return out
    K = (dz / dx) * np.kron(assemble_1d(Nx, Px, _khat(Px)), assemble_1d(Nz, Pz, Wz)) + \
        (dx / dz) * np.kron(assemble_1d(Nx, Px, Wx), assemble_1d(Nz, Pz, _khat(Pz)))
    A = assemble.assemble_stiffness(m).toarray()
    assert np.abs(A - K).max() < 1e-12 * np.abs(K).max()


@pytest.mark.parametrize("Px,Pz", [(2, 4), (4, 2), (3, 5)])
def test_unequal_orders_harmonic_polynomials_reproduced(Px, Pz):
    cases = [
        (lambda x, z: x * x - z * z, lambda x, z: 2 * x, lambda x, z: -2 * z),
        (lambda x, z: x * z, lambda x, z: z, lambda x, z: x),
        (lambda x, z: 3 * x - 2 * z + 1, lambda x, z: 3 + 0 * x, lambda x, z: -2 + 0 * x),
    ]
    m = oc.affine_mesh(3, 2, Px, 2.0, 1.0, Pz=Pz)
    A_full = assemble.assemble_stiffness(m)
    A = assemble.masked(A_full, m.dirichlet_nodes())
    x, z = m.node_coords()
    fw = m.face_weights()
    il, ir, ib = fw["left"][0], fw["right"][0], fw["bottom"][0]
    dn = m.dirichlet_nodes()
    for u, ux, uz in cases:
        gN = {"left": -ux(x[il], z[il]), "right": ux(x[ir], z[ir]), "bottom": -uz(x[ib], z[ib])}
        b = assemble.assemble_rhs(m, f=np.zeros(m.N), gN=gN, gD=u(x[dn], z[dn]), A_full=A_full)
        assert np.abs(assemble.solve_direct(A, b) - u(x, z)).max() < 1e-12


def _wave_error(Px, Pz):
    """Nodal error of the discrete solution of u = cos(kx) cosh(k(z + h0)) under a wavy free
    surface (Dirichlet on the surface, zero normal derivative on walls and flat bottom)."""
    Lx, h0, k = 4.0, 0.5, 2 * math.pi / 4.0 * 2
    x = oc.fine_x_nodes(6, Px, Lx)
    eta = 0.05 * np.sin(2 * math.pi * x / Lx + 0.3)
    m = mesh.Mesh2D(6, 1, Px, Lx, np.full_like(x, h0), eta, Pz=Pz)
    A_full = assemble.assemble_stiffness(m)
    A = assemble.masked(A_full, m.dirichlet_nodes())
    X, Z = m.node_coords()
    dn = m.dirichlet_nodes()
    b = assemble.assemble_rhs(m, f=np.zeros(m.N), gD=W.mms_wave(X[dn], Z[dn], k, h0),
                              A_full=A_full)
    return np.abs(assemble.solve_direct(A, b) - W.mms_wave(X, Z, k, h0)).max()


def test_unequal_orders_converge_in_each_direction():
    """With one order high, raising the other drives the error down spectrally: the x and sigma
    rules enter the right directions (a swap would stall one of the two sequences)."""
    ex = [_wave_error(Px, 12) for Px in (3, 5, 7, 9)]
    ez = [_wave_error(12, Pz) for Pz in (2, 4, 6, 8)]
    assert all(ex[i + 1] < 0.1 * ex[i] for i in range(3)), ex
    assert all(ez[i + 1] < 0.1 * ez[i] for i in range(3)), ez
    assert ex[-1] < 1e-6 and ez[-1] < 1e-7


def _semi_hierarchy(Nx=3, Nz=2, Px=6, Pz=2, **kw):
    wl = W.tank_semi(Nx, Nz, Px, Pz, Lx=25.6 * Nx / 64)
    return wl, oc.hierarchy(wl, **kw)


@pytest.mark.parametrize("Px,Pz", [(6, 2), (2, 5), (7, 4)])
def test_semi_prolongation_reproduces_polynomials(Px, Pz):
    wl, H = _semi_hierarchy(Px=Px, Pz=Pz, smoother="jacobi")
    pairs = pmg.level_orders_2d(H.orders)
    for l in range(len(pairs) - 1):
        mf, mc = H.levels[l].mesh, H.levels[l + 1].mesh
        pcx, pcz = pairs[l + 1]
        assert (mc.P, mc.Pz) == (pcx, pcz)

        def glob(m, F):
            out = np.zeros(m.N)
            out[m.l2g.ravel()] = F.reshape(m.E, -1).ravel()
            return out

        # x^a sigma^b with a <= pcx, b <= pcz lies in the coarse space and is interpolated exactly
        for a in range(pcx + 1):
            for b in range(pcz + 1):
                fc = glob(mc, mc.X ** a * mc.SIG ** b)
                ff = glob(mf, mf.X ** a * mf.SIG ** b)
                assert np.abs(H.prolong(l, fc) - ff).max() < 1e-10 * max(1.0, np.abs(ff).max())


def _dense_B(H):
    n = H.levels[0].N
    B = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        B[:, k] = H.vcycle(e)
    return B


def test_semi_no_smoothing_is_coarse_galerkin_correction():
    wl = W.tank_semi(3, 2, 2, 1, Lx=1.2)
    H = pmg.Hierarchy(oc.mesh_args(wl), [(2, 1), (1, 1)], smoother="jacobi", nu_pre=0,
                      nu_post=0)
    P = H.P[0].toarray()
    assert P.shape == (H.levels[0].N, H.levels[1].N)
    Ac = H.levels[1].A.toarray()
    Z = np.eye(Ac.shape[0])
    Z[H.levels[1].dn, H.levels[1].dn] = 0.0
    B_ref = P @ np.linalg.solve(Ac, Z @ P.T)
    assert np.abs(_dense_B(H) - B_ref).max() < 1e-12 * np.abs(B_ref).max()


@pytest.mark.parametrize("Px,Pz", [(6, 2), (2, 4)])
def test_semi_vcycle_symmetric_positive(Px, Pz):
    wl, H = _semi_hierarchy(Px=Px, Pz=Pz)
    pmg.estimate_lambdas(H)
    B = _dense_B(H)
    assert np.abs(B - B.T).max() < 1e-10 * np.abs(B).max()
    free = np.setdiff1d(np.arange(B.shape[0]), H.levels[0].dn)
    np.linalg.cholesky(0.5 * (B + B.T)[np.ix_(free, free)])


@pytest.mark.parametrize("Px", [3, 10])
def test_semi_solve_matches_direct(Px):
    wl = W.tank_semi(16, 2, Px, 8, Lx=4.0)
    H = oc.hierarchy(wl)
    pmg.estimate_lambdas(H)
    L = H.levels[0]
    b = oc.rhs(wl, L.mesh)
    x, it, hist = pmg.fpcg(L.A, b, np.zeros(L.N), H.vcycle, 1e-10)
    xd = assemble.solve_direct(L.A, b)
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_semi_iterations_flat_in_px():
    """The paper's order sweep (Sec. 6): N_x = 200, N_z = 2, P_z = 8, tolerance 1e-6, P_x from
    2 to 10; FPCG with the semi-coarsened V-cycle takes nearly the same number of iterations
    at every P_x."""
    its = {}
    for Px in (2, 3, 4, 6, 8, 10):
        wl = W.tank_semi(200, 2, Px, 8, Lx=50.0)
        H = oc.hierarchy(wl)
        pmg.estimate_lambdas(H)
        L = H.levels[0]
        b = oc.rhs(wl, L.mesh)
        x, it, hist = pmg.fpcg(L.A, b, np.zeros(L.N), H.vcycle, 1e-6)
        assert hist[-1] <= 1e-6
        its[Px] = it
    assert max(its.values()) - min(its.values()) <= 2, its
