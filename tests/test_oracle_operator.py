"""Pins of the oracle's geometry, operator, right-hand side and discrete solution.

Each check is independent of the oracle's own formulas: isoparametric geometric factors from
nodal coordinates, a brute-force quadrature assembly, the Kronecker closed form on rectangles,
exact reproduction of harmonic polynomials, spectral convergence to harmonic functions, and
dense LAPACK solves.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import assemble, gll, mesh
from tests import oracle_cases as oc


def iso_factors_2d(m):
    """G from the isoparametric map of the nodal (x, z): w |J| J^{-1} J^{-T}."""
    NP = m.NP
    D = m.D
    X = m.X.reshape(m.E, NP, NP)
    Z = m.Z.reshape(m.E, NP, NP)
    xr = np.einsum("ik,ekj->eij", D, X)
    xs = np.einsum("jk,eik->eij", D, X)
    zr = np.einsum("ik,ekj->eij", D, Z)
    zs = np.einsum("jk,eik->eij", D, Z)
    J = xr * zs - xs * zr
    rx, rz = zs / J, -xs / J
    sx, sz = -zr / J, xr / J
    ww = np.outer(m.w, m.w)[None]
    return (ww * J * (rx * rx + rz * rz), ww * J * (rx * sx + rz * sz),
            ww * J * (sx * sx + sz * sz), ww * J)


def tank_mesh(Nx=6, Nz=3, P=5, seed=7):
    wl = W.tank(Nx, Nz, P, surface_seed=seed)
    return oc.fine_mesh(wl)


def test_geometric_factors_match_isoparametric():
    for P in (2, 5, 8):
        m = tank_mesh(P=P)
        Grr, Grs, Gss, WJ = iso_factors_2d(m)
        sc = np.abs(Gss).max()
        assert np.abs(Grr - m.Grr).max() < 1e-12 * sc
        assert np.abs(Grs - m.Grs).max() < 1e-12 * sc
        assert np.abs(Gss - m.Gss).max() < 1e-12 * sc
        assert np.abs(WJ - m.mass).max() < 1e-14


def brute_force_stiffness(m):
    """Dense global stiffness by explicit quadrature loops over elements and node pairs."""
    NP, D, w = m.NP, m.D, m.w
    K = np.zeros((m.N, m.N))
    X = m.X.reshape(m.E, NP, NP)
    Z = m.Z.reshape(m.E, NP, NP)
    for e in range(m.E):
        g = m.l2g[e].reshape(NP, NP)
        for qi in range(NP):
            for qj in range(NP):
                xr = sum(D[qi, k] * X[e, k, qj] for k in range(NP))
                xs = sum(D[qj, k] * X[e, qi, k] for k in range(NP))
                zr = sum(D[qi, k] * Z[e, k, qj] for k in range(NP))
                zs = sum(D[qj, k] * Z[e, qi, k] for k in range(NP))
                J = np.array([[xr, xs], [zr, zs]])
                Jit = np.linalg.inv(J).T
                wq = w[qi] * w[qj] * abs(np.linalg.det(J))
                grads = {}
                for a in range(NP):
                    for b in range(NP):
                        dr = D[qi, a] if b == qj else 0.0
                        ds = D[qj, b] if a == qi else 0.0
                        if dr or ds:
                            grads[(a, b)] = Jit @ np.array([dr, ds])
                for (a, b), ga in grads.items():
                    for (c, d), gc in grads.items():
                        K[g[a, b], g[c, d]] += wq * ga @ gc
    return K


def test_bruteforce_assembly_equals_csr():
    m = tank_mesh(Nx=2, Nz=2, P=3)
    K = brute_force_stiffness(m)
    A = assemble.assemble_stiffness(m).toarray()
    assert np.abs(K - A).max() < 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("P", [2, 4, 6])
def test_symmetry_and_constant_nullspace(P):
    m = tank_mesh(P=P)
    A = assemble.assemble_stiffness(m)
    sc = abs(A).max()
    assert abs(A - A.T).max() < 1e-14 * sc * 10
    assert np.abs(A @ np.ones(m.N)).max() < 1e-13 * sc
    # masked (Dirichlet top) operator is SPD: dense Cholesky succeeds
    Am = assemble.masked(A, m.dirichlet_nodes()).toarray()
    np.linalg.cholesky(Am)


def test_rectangle_kronecker_closed_form():
    Nx, Nz, P, Lx, H = 3, 2, 4, 3.0, 0.8
    m = oc.affine_mesh(Nx, Nz, P, Lx, H)
    dx, dz = Lx / Nx, H / Nz
    # 1D stiffness from Gauss-Legendre quadrature of the Lagrange basis (exact)
    r = gll.gll_nodes(P)
    xg, wg = np.polynomial.legendre.leggauss(P + 2)
    L = np.zeros((P + 1, xg.size))
    for i in range(P + 1):
        c = np.polynomial.polynomial.polyfromroots(np.delete(r, i))
        c = c / np.polynomial.polynomial.polyval(r[i], c)
        L[i] = np.polynomial.polynomial.polyval(xg, np.polynomial.polynomial.polyder(c))
    Khat = (L * wg) @ L.T
    What = np.diag(gll.gll_weights(P))
    Ae_ref = (dz / dx) * np.kron(Khat, What) + (dx / dz) * np.kron(What, Khat)
    Ae = assemble.element_matrices(m)
    assert np.abs(Ae - Ae_ref[None]).max() < 1e-12 * np.abs(Ae_ref).max()


def _solve_affine(u, dudx, dudz, Nx=3, Nz=2, P=3, Lx=2.0, H=1.0):
    m = oc.affine_mesh(Nx, Nz, P, Lx, H)
    A_full = assemble.assemble_stiffness(m)
    A = assemble.masked(A_full, m.dirichlet_nodes())
    x, z = m.node_coords()
    fw = m.face_weights()
    il, ir, ib = fw["left"][0], fw["right"][0], fw["bottom"][0]
    gN = {"left": -dudx(x[il], z[il]), "right": dudx(x[ir], z[ir]), "bottom": -dudz(x[ib], z[ib])}
    dn = m.dirichlet_nodes()
    b = assemble.assemble_rhs(m, f=np.zeros(m.N), gN=gN, gD=u(x[dn], z[dn]), A_full=A_full)
    return assemble.solve_direct(A, b), u(x, z)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_harmonic_polynomials_reproduced(P):
    cases = [
        (lambda x, z: x * x - z * z, lambda x, z: 2 * x, lambda x, z: -2 * z),
        (lambda x, z: x * z, lambda x, z: z, lambda x, z: x),
        (lambda x, z: 3 * x - 2 * z + 1, lambda x, z: 3 + 0 * x, lambda x, z: -2 + 0 * x),
    ]
    for u, ux, uz in cases:
        uh, ue = _solve_affine(u, ux, uz, P=P)
        assert np.abs(uh - ue).max() < 1e-12


def test_manufactured_c1_spectral_convergence():
    errs = {}
    for P in (2, 4, 6, 8):
        wl = W.c1(P)
        m = oc.fine_mesh(wl)
        A_full = assemble.assemble_stiffness(m)
        A = assemble.masked(A_full, m.dirichlet_nodes())
        b = oc.rhs(wl, m, A_full)
        u = assemble.solve_direct(A, b)
        x, z = m.node_coords()
        errs[P] = np.abs(u - W.mms_c1(x, z)).max()
    assert errs[2] < 1e-3 and errs[4] < 1e-6 and errs[6] < 1e-9 and errs[8] < 1e-12
    assert errs[4] < 1e-2 * errs[2] and errs[6] < 1e-2 * errs[4]


def test_sigma_mapped_manufactured_convergence():
    """u = cos(kx) cosh(k(z+h0)) under a wavy free surface; Dirichlet on the surface, zero
    normal derivative on the walls and flat bottom; spectral decay of the nodal error."""
    Lx, h0, k = 4.0, 0.5, 2 * math.pi / 4.0
    errs = []
    for P in (3, 5, 7, 9):
        x = oc.fine_x_nodes(8, P, Lx)
        eta = 0.05 * np.sin(2 * math.pi * x / Lx + 0.3) + 0.02 * np.cos(6 * math.pi * x / Lx)
        m = mesh.Mesh2D(8, 2, P, Lx, np.full_like(x, h0), eta)
        A_full = assemble.assemble_stiffness(m)
        A = assemble.masked(A_full, m.dirichlet_nodes())
        X, Z = m.node_coords()
        dn = m.dirichlet_nodes()
        b = assemble.assemble_rhs(m, f=np.zeros(m.N), gD=W.mms_wave(X[dn], Z[dn], k, h0),
                                  A_full=A_full)
        u = assemble.solve_direct(A, b)
        errs.append(np.abs(u - W.mms_wave(X, Z, k, h0)).max())
    assert errs[-1] < 1e-9
    assert all(errs[i + 1] < 0.05 * errs[i] for i in range(len(errs) - 1))


def test_direct_equals_dense_solve():
    m = tank_mesh(Nx=2, Nz=1, P=3)
    A = assemble.assemble_operator(m)
    b = W.random_vector(m.N, 3)
    b[m.dirichlet_nodes()] = 0.0
    assert np.abs(assemble.solve_direct(A, b) - np.linalg.solve(A.toarray(), b)).max() < 1e-11


def test_matrix_free_equals_csr():
    m = tank_mesh(Nx=5, Nz=3, P=4)
    x = W.random_vector(m.N, 5)
    for dirichlet in (True, False):
        A = assemble.assemble_operator(m, dirichlet=dirichlet)
        y = assemble.apply_matrix_free(m, x, dirichlet=dirichlet)
        assert np.abs(y - A @ x).max() < 1e-12 * np.abs(y).max()


def test_mass_and_face_measures():
    # lumped mass integrates 1 exactly on the affine c1 domain: area 2 pi
    m = oc.fine_mesh(W.c1(4))
    assert abs(assemble.lumped_mass(m).sum() - 2 * math.pi) < 1e-12
    fw = m.face_weights()
    assert abs(fw["bottom"][1].sum() - 2 * math.pi) < 1e-12
    assert abs(fw["left"][1].sum() - 1.0) < 1e-14
    # sigma-mapped tank: area = int_0^L d(x) dx, exact for the element polynomial d
    mt = tank_mesh(Nx=4, Nz=2, P=6)
    xg, wg = np.polynomial.legendre.leggauss(12)
    area = 0.0
    for ex in range(mt.Nx):
        # integrate the degree-P interpolant of d with Gauss-Legendre
        c = np.polynomial.polynomial.polyfit(mt.r, mt.d[ex], mt.P)
        area += (mt.dx / 2) * (wg * np.polynomial.polynomial.polyval(xg, c)).sum()
    assert abs(assemble.lumped_mass(mt).sum() - area) < 1e-12


def test_3d_operator_properties():
    wl = W.tank3d(2, 2, 2, 3, L=1.6)
    m = oc.fine_mesh(wl)
    A = assemble.assemble_stiffness(m)
    sc = abs(A).max()
    assert abs(A - A.T).max() < 1e-13 * sc
    assert np.abs(A @ np.ones(m.N)).max() < 1e-12 * sc
    x = W.random_vector(m.N, 11)
    y = assemble.apply_matrix_free(m, x)
    assert np.abs(y - assemble.assemble_operator(m) @ x).max() < 1e-12 * np.abs(y).max()


def test_3d_harmonic_reproduction():
    """u = x^2 - z^2 + x y - y^2/2 ... (harmonic) reproduced on an affine box, P = 2."""
    Nx = Ny = 2
    Nz, P, L, H = 2, 2, 1.0, 0.5
    x = oc.fine_x_nodes(Nx, P, L)
    Xh, Yh = np.meshgrid(x, x, indexing="ij")
    m = mesh.Mesh3D(Nx, Ny, Nz, P, L, L, np.full_like(Xh, H), np.zeros_like(Xh))

    def u(x, y, z):
        return x * x - z * z + x * y + 0.5 * (y * y - x * x) - 0.5 * (y * y - z * z)

    def grad(x, y, z):
        return (2 * x + y - x, x + y - y, -2 * z + z)

    A_full = assemble.assemble_stiffness(m)
    A = assemble.masked(A_full, m.dirichlet_nodes())
    X, Y, Z = m.node_coords()
    fw = m.face_weights()
    gN = {}
    for name, comp, sgn in (("xlo", 0, -1), ("xhi", 0, 1), ("ylo", 1, -1), ("yhi", 1, 1),
                            ("bottom", 2, -1)):
        idx = fw[name][0]
        gN[name] = sgn * grad(X[idx], Y[idx], Z[idx])[comp]
    dn = m.dirichlet_nodes()
    b = assemble.assemble_rhs(m, f=np.zeros(m.N), gN=gN, gD=u(X[dn], Y[dn], Z[dn]), A_full=A_full)
    uh = assemble.solve_direct(A, b)
    assert np.abs(uh - u(X, Y, Z)).max() < 1e-12


# ---- 3D sigma-mapped geometry --------------------------------------------------------------
def _wavy_3d(Nx, Ny, Nz, P, Lx=1.7, Ly=1.3, swap=False):
    """A sigma-mapped 3D mesh whose depth and surface vary along x and y (non-zero h_x, h_y,
    eta_x, eta_y).  swap=True builds the mirror mesh with the roles of x and y exchanged."""
    def h(x, y):
        return 0.6 + 0.15 * np.sin(1.3 * x + 0.4) * np.cos(0.9 * y - 0.2) + 0.05 * y

    def eta(x, y):
        return 0.04 * np.sin(2.1 * x - 1.7 * y + 0.3) + 0.02 * np.cos(3.0 * y)

    if swap:
        Nx, Ny, Lx, Ly = Ny, Nx, Ly, Lx
        hf, ef = (lambda x, y: h(y, x)), (lambda x, y: eta(y, x))
    else:
        hf, ef = h, eta
    xs = oc.fine_x_nodes(Nx, P, Lx)
    ys = oc.fine_x_nodes(Ny, P, Ly)
    Xh, Yh = np.meshgrid(xs, ys, indexing="ij")
    return mesh.Mesh3D(Nx, Ny, Nz, P, Lx, Ly, hf(Xh, Yh), ef(Xh, Yh))


def iso_factors_3d(m):
    """w |J| (grad a . grad b) for a, b in (r, t, s) from the isoparametric map of the nodal
    (x, y, z): the Jacobian from differentiating the nodal coordinates with D, inverted per
    node (its rows are grad r, grad t, grad s)."""
    D = m.D
    sh = (m.E, m.NP, m.NP, m.NP)
    crd = [m.X.reshape(sh), m.Y.reshape(sh), m.Z.reshape(sh)]
    J = np.empty(sh + (3, 3))
    for c, F in enumerate(crd):
        J[..., c, 0] = np.einsum("ia,eamj->eimj", D, F)   # d/dr (element-local axis i)
        J[..., c, 1] = np.einsum("ma,eiaj->eimj", D, F)   # d/dt (axis m)
        J[..., c, 2] = np.einsum("ja,eima->eimj", D, F)   # d/ds (axis j)
    det = np.linalg.det(J)
    Ji = np.linalg.inv(J)            # Ji[..., a, :] = grad of reference coordinate a
    w3 = m.w[:, None, None] * m.w[None, :, None] * m.w[None, None, :]
    wj = w3[None] * det
    G = {}
    names = "rts"
    for a in range(3):
        for b in range(a, 3):
            G[names[a] + names[b]] = wj * np.einsum("...k,...k->...", Ji[..., a, :], Ji[..., b, :])
    return G, wj


@pytest.mark.parametrize("P", [2, 4, 6])
def test_3d_geometric_factors_match_isoparametric(P):
    m = _wavy_3d(3, 2, 2, P)
    # the mesh really is sigma-mapped along both horizontal directions
    assert np.abs(m.hx).max() > 0.05 and np.abs(m.hy).max() > 0.05
    assert np.abs(m.dxd - m.hx).max() > 0.01 and np.abs(m.dyd - m.hy).max() > 0.01
    G, wj = iso_factors_3d(m)
    sc = max(np.abs(m.Gss).max(), np.abs(m.Grr).max())
    for nm, ours in (("rr", m.Grr), ("tt", m.Gtt), ("rs", m.Grs), ("ts", m.Gts), ("ss", m.Gss)):
        assert np.abs(G[nm] - ours).max() < 1e-12 * sc, nm
    assert np.abs(G["rt"]).max() < 1e-12 * sc          # x and y affine: no r-t coupling
    assert np.abs(wj - m.mass).max() < 1e-14 * np.abs(m.mass).max() * 100


def test_3d_operator_invariant_under_xy_transposition():
    """Exchanging the roles of x and y (depth and surface mirrored) permutes the nodes and must
    leave the operator unchanged: catches an h_x / h_y or eta_x / eta_y mix-up."""
    Nx, Ny, Nz, P = 3, 2, 2, 3
    a = _wavy_3d(Nx, Ny, Nz, P)
    b = _wavy_3d(Nx, Ny, Nz, P, swap=True)
    Aa = assemble.assemble_operator(a).toarray()
    Ab = assemble.assemble_operator(b).toarray()
    nx, ny, nz = a.nx_nodes, a.ny_nodes, a.nz_nodes
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ga = ((ix * ny + iy) * nz + iz).ravel()
    gb = ((iy * nx + ix) * nz + iz).ravel()           # the same physical node in mesh b
    perm = np.empty(a.N, dtype=np.int64)
    perm[ga] = gb
    assert np.abs(Aa - Ab[np.ix_(perm, perm)]).max() < 1e-12 * np.abs(Aa).max()


def test_3d_y_uniform_reduces_to_2d():
    """With depth and surface independent of y, every x-sigma section of the 3D factors is the
    2D mesh's factor times the y quadrature weight w_m dy/2 (and the y couplings vanish)."""
    Nx, Ny, Nz, P, Lx, Ly = 3, 2, 2, 5, 1.9, 0.8

    def h(x):
        return 0.5 + 0.2 * np.sin(1.7 * x)

    def eta(x):
        return 0.03 * np.cos(2.3 * x + 0.1)

    xs = oc.fine_x_nodes(Nx, P, Lx)
    ys = oc.fine_x_nodes(Ny, P, Ly)
    Xh, _ = np.meshgrid(xs, ys, indexing="ij")
    m3 = mesh.Mesh3D(Nx, Ny, Nz, P, Lx, Ly, h(Xh), eta(Xh))
    m2 = mesh.Mesh2D(Nx, Nz, P, Lx, h(xs), eta(xs))
    NP = P + 1
    s3 = (Nx, Ny, Nz, NP, NP, NP)
    wy = (m3.w * Ly / Ny / 2.0)[None, None, None, None, :, None]

    def as3(g2):   # (E2, NP, NP) -> (Nx, 1, Nz, NP, 1, NP)
        return g2.reshape(Nx, Nz, NP, NP)[:, None, :, :, None, :]

    for f3, f2 in ((m3.Grr, m2.Grr), (m3.Grs, m2.Grs), (m3.Gss, m2.Gss), (m3.mass, m2.mass)):
        ref = as3(f2) * wy
        assert np.abs(f3.reshape(s3) - ref).max() < 1e-13 * np.abs(ref).max()
    assert np.abs(m3.Gts).max() < 1e-14 * np.abs(m3.Gss).max()


def test_3d_sigma_mapped_manufactured_convergence():
    """u = cos(kx x) cos(ky y) cosh(k (z + h0)), k^2 = kx^2 + ky^2 (harmonic), on a flat-bottomed
    box under a free surface that varies in x and y: Dirichlet data on the surface, zero normal
    derivative on the walls (kx = pi / Lx, ky = pi / Ly) and on the bottom z = -h0; the nodal
    error must decay geometrically in P (a wrong sigma_x or sigma_y term leaves an O(eta) error
    that does not decay)."""
    Lx, Ly, h0 = 2.0, 1.5, 0.5
    kx, ky = math.pi / Lx, math.pi / Ly
    k = math.hypot(kx, ky)

    def u(x, y, z):
        return np.cos(kx * x) * np.cos(ky * y) * np.cosh(k * (z + h0))

    errs = []
    for P in (2, 3, 4, 5, 6):
        xs = oc.fine_x_nodes(2, P, Lx)
        ys = oc.fine_x_nodes(2, P, Ly)
        Xh, Yh = np.meshgrid(xs, ys, indexing="ij")
        eta = 0.04 * np.sin(2 * math.pi * Xh / Lx + 0.3) * np.cos(2 * math.pi * Yh / Ly - 0.5)
        m = mesh.Mesh3D(2, 2, 1, P, Lx, Ly, np.full_like(Xh, h0), eta)
        assert np.abs(m.dxd).max() > 0.05 and np.abs(m.dyd).max() > 0.05
        A_full = assemble.assemble_stiffness(m)
        A = assemble.masked(A_full, m.dirichlet_nodes())
        X, Y, Z = m.node_coords()
        dn = m.dirichlet_nodes()
        b = assemble.assemble_rhs(m, f=np.zeros(m.N), gD=u(X[dn], Y[dn], Z[dn]), A_full=A_full)
        uh = assemble.solve_direct(A, b)
        errs.append(np.abs(uh - u(X, Y, Z)).max())
    # measured: 2.8e-2, 2.7e-3, 3.8e-4, 8.2e-5, 1.3e-5
    assert errs[-1] < 3e-5, errs
    assert all(errs[i + 1] < 0.3 * errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-3 * errs[0], errs
