"""Oracle-side construction of workload meshes and right-hand sides (tests only).

The oracle samples the analytic input fields of ``workloads`` at its own GLL nodes.
"""
import math

import numpy as np

import workloads as W
from oracle import assemble, gll, mesh, pmg


def fine_x_nodes(Nx, P, Lx):
    r = gll.gll_nodes(P)
    xe = Lx * (np.arange(Nx)[:, None] + (r[None, :] + 1.0) / 2.0) / Nx
    return np.concatenate([xe[:, :-1].ravel(), [Lx]])


def surface_samples(wl):
    """(h, eta) at the fine horizontal GLL nodes of a 2D or 3D workload."""
    if wl.dim == 2:
        x = fine_x_nodes(wl.Nx, wl.P, wl.Lx)
        if wl.kind == "manufactured":
            return x, np.ones_like(x), np.zeros_like(x)
        return x, W.bar_depth(x, wl.Lx), W.surface(x, wl.Lx, wl.surface_seed)
    x = fine_x_nodes(wl.Nx, wl.P, wl.Lx)
    y = fine_x_nodes(wl.Ny, wl.P, wl.Ly)
    X, Y = np.meshgrid(x, y, indexing="ij")
    h = W.bar_depth_3d(X, Y, wl.Lx, wl.surface_seed)
    eta = W.surface_3d(X, Y, 0.0, wl.Lx, wl.surface_seed)
    return (X, Y), h, eta


def mesh_args(wl):
    xs, h, eta = surface_samples(wl)
    if wl.dim == 2:
        return dict(dim=2, Nx=wl.Nx, Nz=wl.Nz, Lx=wl.Lx, h=h, eta=eta)
    return dict(dim=3, Nx=wl.Nx, Ny=wl.Ny, Nz=wl.Nz, Lx=wl.Lx, Ly=wl.Ly, h=h, eta=eta)


def fine_mesh(wl, P=None):
    a = mesh_args(wl)
    P = wl.P if P is None else P
    if wl.dim == 2:
        return mesh.Mesh2D(a["Nx"], a["Nz"], P, a["Lx"], a["h"], a["eta"], P_fine=wl.P,
                           Pz=wl.Pz)
    return mesh.Mesh3D(a["Nx"], a["Ny"], a["Nz"], P, a["Lx"], a["Ly"], a["h"], a["eta"],
                       P_fine=wl.P)


def hierarchy(wl, **kw):
    opts = dict(smoother=wl.smoother, nu_pre=wl.nu_pre, nu_post=wl.nu_post,
                cheb_degree=wl.cheb_degree, cheb_lo=wl.cheb_lo, cheb_hi=wl.cheb_hi,
                cheb_degree_coarse=wl.cheb_degree_coarse or None)
    opts.update(kw)
    orders = wl.orders if wl.orders else pmg.coarsen_orders_2d(wl.P, wl.pz)
    return pmg.Hierarchy(mesh_args(wl), orders, **opts)


def rhs(wl, m, A_full=None):
    """Assembled right-hand side b of a workload on the oracle mesh m."""
    if wl.kind == "manufactured":
        x, z = m.node_coords()
        fw = m.face_weights()
        dn = m.dirichlet_nodes()
        gN = W.mms_c1_neumann(z[fw["left"][0]], z[fw["right"][0]], x[fw["bottom"][0]])
        return assemble.assemble_rhs(m, f=np.zeros(m.N), gN=gN, gD=W.mms_c1(x[dn], z[dn]),
                                     A_full=A_full)
    if wl.dim == 2:
        x, z = m.node_coords()
        f = W.bumps(x, z, wl.Lx, wl.rhs_seed, lambda s: W.bar_depth(s, wl.Lx),
                    lambda s: W.surface(s, wl.Lx, wl.surface_seed))
        return assemble.assemble_rhs(m, f=f)
    x, y, z = m.node_coords()
    f = W.bumps_3d(x, y, z, 0.0, wl.Lx, wl.rhs_seed,
                   lambda a, b: W.bar_depth_3d(a, b, wl.Lx, wl.surface_seed),
                   lambda a, b: W.surface_3d(a, b, 0.0, wl.Lx, wl.surface_seed))
    return assemble.assemble_rhs(m, f=f)


def affine_mesh(Nx, Nz, P, Lx, depth, Pz=None):
    x = fine_x_nodes(Nx, P, Lx)
    return mesh.Mesh2D(Nx, Nz, P, Lx, np.full_like(x, depth), np.zeros_like(x), Pz=Pz)


def c1_fine_x(P):
    return fine_x_nodes(8, P, 2.0 * math.pi)
