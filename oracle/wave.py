"""Oracle: a stage loop around the pressure-type solve (test infrastructure only).

The paper solves a Poisson problem at every stage of its low-storage Runge-Kutta scheme (Sec. 3,
eq. poissonp) on the sigma-mapped mesh of that stage's free surface, with a time-constant
preconditioner (Sec. 5.4).  Its right-hand side needs the Navier-Stokes velocities, which are
out of scope here; the stage loop is driven instead by the linear free-surface potential-flow
model on the same mesh, whose per-stage solve is the same operator: with the state
(eta, Phi) at the surface nodes,
    phi solves  -lap phi = 0,  phi = Phi on the surface,  d phi / dn = 0 on walls and bottom,
    d eta / dt = d phi / dz at the surface,   d Phi / dt = -g eta,
on the mesh whose sigma transform follows eta.  d phi / dz at a surface node is (1/d) d phi /
d sigma (Sec. 2.2, sigma_z = 1/d), d phi / d sigma from the top element's nodal values with the
GLL differentiation matrix.  For small amplitude over a flat bottom a standing wave
eta = A cos(kx) cos(omega t) with omega^2 = g k tanh(k h) solves the model.
"""
import numpy as np

from . import assemble, lserk
from .mesh import Mesh2D, Mesh3D


def surface_dz(mesh, phi):
    """d phi / dz at the surface nodes (one per vertical node line, in node-line order)."""
    P, NP = mesh.P, mesh.NP
    Ps = mesh.Pz if mesh.dim == 2 else P
    Ds = mesh.Dz if mesh.dim == 2 else mesh.D
    nzn = mesh.nz_nodes
    lines = np.asarray(phi, dtype=np.float64).reshape(-1, nzn)
    top = lines[:, nzn - Ps - 1:]          # the top element's nodes of every line
    dsig_ref = top @ Ds[Ps]                # d phi / d r at r = 1
    dsig = 2.0 / mesh.dsig * dsig_ref      # d phi / d sigma
    x_dep = surface_depth(mesh)
    return dsig / x_dep


def surface_depth(mesh):
    """d = h + eta at every vertical node line."""
    if mesh.dim == 2:
        out = np.zeros(mesh.nx_nodes)
        for ex in range(mesh.Nx - 1, -1, -1):
            out[ex * mesh.P: ex * mesh.P + mesh.NP] = mesh.d[ex]
        return out
    out = np.zeros((mesh.nx_nodes, mesh.ny_nodes))
    P, NP = mesh.P, mesh.NP
    for ex in range(mesh.Nx - 1, -1, -1):
        for ey in range(mesh.Ny - 1, -1, -1):
            out[ex * P: ex * P + NP, ey * P: ey * P + NP] = mesh.d[ex, ey]
    return out.ravel()


class LinearWaves:
    """The model above on a 2D tank (Nx x Nz elements, order P, length Lx, still-water depth
    h at the fine horizontal GLL nodes); each right-hand side evaluation builds the mesh of the
    current surface and solves its Dirichlet problem exactly (sparse direct)."""

    def __init__(self, Nx, Nz, P, Lx, h, g=9.81):
        self.Nx, self.Nz, self.P, self.Lx = Nx, Nz, P, Lx
        self.h = np.asarray(h, dtype=np.float64)
        self.g = g
        self.ns = self.h.size
        self.last_phi = None

    def mesh(self, eta):
        return Mesh2D(self.Nx, self.Nz, self.P, self.Lx, self.h, eta)

    def solve_phi(self, eta, Phi):
        m = self.mesh(eta)
        A_full = assemble.assemble_stiffness(m)
        A = assemble.masked(A_full, m.dirichlet_nodes())
        b = assemble.assemble_rhs(m, gD=Phi, A_full=A_full)
        return m, assemble.solve_direct(A, b)

    def rhs(self, y, t):
        eta, Phi = y[:self.ns], y[self.ns:]
        m, phi = self.solve_phi(eta, Phi)
        self.last_phi = phi
        return np.concatenate([surface_dz(m, phi), -self.g * eta])

    def step(self, y, t, dt, stage_hook=None):
        return lserk.step(self.rhs, y, t, dt, stage_hook)
