"""Oracle: element matrices, global assembly, right-hand side, direct solve (test infrastructure only).

Global sparse matrices are the sum of the local dense element matrices (Sec. 4.2, eqs.
flocal / globallocal).  The element stiffness (the L^b matrices of eq. flocal2, read with the
missing transpose as D^T M D and with GLL collocation for the quadrature) is, per element,
    A_e = sum_{a,b} D_a^T diag(G_ab) D_b,   a, b in {r, s} (2D) or {r, t, s} (3D),
with D_r = D (x) I, D_s = I (x) D in the element-local ordering (i slow, j fast); on 2D meshes
with different orders along x and sigma, D_r = D_x (x) I and D_s = I (x) D_sigma.

Boundary value problem (Sec. 3.2): p = g_D on the free surface (top, eq. bcpd), n . grad p =
g_N on walls and bottom (eq. bcpdneu), -lap p = f inside.  The discrete system solved is
    [A_ff 0; 0 I] [p_f; p_D] = [M f + B g_N - A_fD g_D ; g_D]
("masked" operator: the free block on free rows, identity on Dirichlet rows), M the assembled
GLL-lumped mass and B g_N the GLL surface quadrature of the Neumann data.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _kron_ops(mesh):
    NP = mesh.NP
    I = np.eye(NP)
    D = mesh.D
    if mesh.dim == 2:  # x rule of order P, sigma rule of order Pz
        return {"r": np.kron(D, np.eye(mesh.NPz)), "s": np.kron(I, mesh.Dz)}
    return {"r": np.kron(np.kron(D, I), I), "t": np.kron(np.kron(I, D), I),
            "s": np.kron(np.kron(I, I), D)}


def _field_pairs(mesh):
    """(a, b, G_ab) for every ordered pair with non-zero geometric factor."""
    E = mesh.E
    if mesh.dim == 2:
        Grr, Grs, Gss = (g.reshape(E, -1) for g in mesh.fields())
        return [("r", "r", Grr), ("r", "s", Grs), ("s", "r", Grs), ("s", "s", Gss)]
    Grr, Gtt, Grs, Gts, Gss = (g.reshape(E, -1) for g in mesh.fields())
    return [("r", "r", Grr), ("t", "t", Gtt), ("r", "s", Grs), ("s", "r", Grs),
            ("t", "s", Gts), ("s", "t", Gts), ("s", "s", Gss)]


def element_matrices(mesh):
    """Dense element stiffness matrices, shape (E, NL, NL)."""
    ops = _kron_ops(mesh)
    NL = mesh.NL
    A = np.zeros((mesh.E, NL, NL))
    for a, b, G in _field_pairs(mesh):
        Da, Db = ops[a], ops[b]
        # D_a^T diag(G) D_b for every element
        A += np.einsum("ka,ek,kb->eab", Da, G, Db)
    return A


def assemble_stiffness(mesh):
    """Global stiffness (no boundary conditions) as CSR: sum of element matrices."""
    Ae = element_matrices(mesh)
    NL = Ae.shape[1]
    rows = np.repeat(mesh.l2g, NL, axis=1).ravel()
    cols = np.tile(mesh.l2g, (1, NL)).ravel()
    return sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(mesh.N, mesh.N)).tocsr()


def masked(A, dirichlet):
    """[A_ff 0; 0 I]: zero Dirichlet rows and columns, unit diagonal on Dirichlet rows."""
    n = A.shape[0]
    keep = np.ones(n)
    keep[dirichlet] = 0.0
    K = sp.diags(keep)
    Id = sp.diags(1.0 - keep)
    return (K @ A @ K + Id).tocsr()


def assemble_operator(mesh, dirichlet=True):
    A = assemble_stiffness(mesh)
    if dirichlet:
        A = masked(A, mesh.dirichlet_nodes())
    return A


def apply_matrix_free(mesh, x, dirichlet=True):
    """y = A x element by element (A_e u_e from the four/seven products), summed into y.

    Used where the CSR matrix would be too large.  Same operator as assemble_operator.
    """
    x = np.asarray(x, dtype=np.float64).copy()
    dn = mesh.dirichlet_nodes()
    if dirichlet:
        xd = x[dn].copy()
        x[dn] = 0.0
    NP, E, D = mesh.NP, mesh.E, mesh.D
    if mesh.dim == 2:
        Dz = mesh.Dz
        u = x[mesh.l2g].reshape(E, NP, mesh.NPz)
        ur = np.einsum("ik,ekj->eij", D, u)
        us = np.einsum("jk,eik->eij", Dz, u)
        wr = mesh.Grr * ur + mesh.Grs * us
        ws = mesh.Grs * ur + mesh.Gss * us
        v = np.einsum("ki,ekj->eij", D, wr) + np.einsum("kj,eik->eij", Dz, ws)
    else:
        u = x[mesh.l2g].reshape(E, NP, NP, NP)
        ur = np.einsum("ia,eamj->eimj", D, u)
        ut = np.einsum("ma,eiaj->eimj", D, u)
        us = np.einsum("ja,eima->eimj", D, u)
        wr = mesh.Grr * ur + mesh.Grs * us
        wt = mesh.Gtt * ut + mesh.Gts * us
        ws = mesh.Grs * ur + mesh.Gts * ut + mesh.Gss * us
        v = (np.einsum("ai,eamj->eimj", D, wr) + np.einsum("am,eiaj->eimj", D, wt)
             + np.einsum("aj,eima->eimj", D, ws))
    y = np.bincount(mesh.l2g.ravel(), weights=v.reshape(E, -1).ravel(), minlength=mesh.N)
    if dirichlet:
        y[dn] = xd
    return y


def lumped_mass(mesh):
    """Assembled GLL-lumped mass vector (diagonal of M)."""
    return np.bincount(mesh.l2g.ravel(), weights=mesh.mass.reshape(mesh.E, -1).ravel(),
                       minlength=mesh.N)


def assemble_rhs(mesh, f=None, gN=None, gD=None, A_full=None):
    """b = M f + sum_faces (surface quadrature of g_N); Dirichlet rows = g_D; lifting -A_fD g_D.

    f   : nodal source values (length N) or None
    gN  : dict face name -> nodal values on that face (see mesh.face_weights) or None
    gD  : values on the Dirichlet (top) nodes, ordered as mesh.dirichlet_nodes(), or None
    """
    b = np.zeros(mesh.N)
    if f is not None:
        b += lumped_mass(mesh) * np.asarray(f, dtype=np.float64)
    if gN is not None:
        fw = mesh.face_weights()
        for name, vals in gN.items():
            idx, wts = fw[name]
            np.add.at(b, idx, wts * np.asarray(vals, dtype=np.float64))
    dn = mesh.dirichlet_nodes()
    if gD is not None:
        gD = np.asarray(gD, dtype=np.float64)
        lift = np.zeros(mesh.N)
        lift[dn] = gD
        if A_full is not None:
            Al = A_full @ lift
        else:
            # unmasked operator applied to the lifting vector
            Al = apply_matrix_free(mesh, lift, dirichlet=False)
        b -= Al
        b[dn] = gD
    else:
        b[dn] = 0.0
    return b


def solve_direct(A_masked, b):
    """x = A^{-1} b with SuperLU (the discrete solution that p-multigrid converges to)."""
    lu = spla.splu(sp.csc_matrix(A_masked))
    return lu.solve(np.asarray(b, dtype=np.float64))
