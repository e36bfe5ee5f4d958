"""Set up solver contexts and right-hand sides for the synthetic workloads of ``workloads``.

The library's own GLL rule and node coordinates are used to sample the analytic inputs.
"""
import numpy as np

import workloads as W

from .binding import Solver, fine_x_nodes


def surface_samples(wl):
    x = fine_x_nodes(wl.Nx, wl.P, wl.Lx)
    if wl.dim == 2:
        if wl.kind == "manufactured":
            return np.ones_like(x), np.zeros_like(x)
        return W.bar_depth(x, wl.Lx), W.surface(x, wl.Lx, wl.surface_seed)
    y = fine_x_nodes(wl.Ny, wl.P, wl.Ly)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return (W.bar_depth_3d(X, Y, wl.Lx, wl.surface_seed),
            W.surface_3d(X, Y, 0.0, wl.Lx, wl.surface_seed))


def make_solver(wl, prec="f64", **kw):
    h, eta = surface_samples(wl)
    opts = dict(levels=wl.orders or None, prec=prec, smoother=wl.smoother, nu_pre=wl.nu_pre,
                nu_post=wl.nu_post, cheb_degree=wl.cheb_degree,
                cheb_degree_coarse=wl.cheb_degree_coarse, cheb_lo=wl.cheb_lo,
                cheb_hi=wl.cheb_hi, order_z=wl.Pz)
    opts.update(kw)
    ne = (wl.Nx, wl.Ny if wl.dim == 3 else 1, wl.Nz)
    length = (wl.Lx, wl.Ly if wl.dim == 3 else 1.0)
    return Solver(wl.dim, ne, wl.P, length, h, eta, **opts)


def make_rhs(wl, s):
    """Assembled right-hand side on the device for workload wl and solver s."""
    import torch
    dev = "cuda"
    if wl.kind == "manufactured":
        x, z = s.coords(0)
        nzn, nxn = wl.Nz * wl.pz + 1, wl.Nx * wl.P + 1
        zl = z[:nzn]
        zr = z[(nxn - 1) * nzn:]
        xb = x[::nzn]
        g = W.mms_c1_neumann(zl, zr, xb)
        gN = np.concatenate([g["left"], g["right"], g["bottom"]])
        top = np.arange(nxn) * nzn + nzn - 1
        gD = W.mms_c1(x[top], z[top])
        t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
        return s.assemble_rhs(f=None, gN=t(gN), gD=t(gD))
    if wl.dim == 2:
        x, z = s.coords(0)
        f = W.bumps(x, z, wl.Lx, wl.rhs_seed, lambda a: W.bar_depth(a, wl.Lx),
                    lambda a: W.surface(a, wl.Lx, wl.surface_seed))
    else:
        x, y, z = s.coords(0)
        f = W.bumps_3d(x, y, z, 0.0, wl.Lx, wl.rhs_seed,
                       lambda a, b: W.bar_depth_3d(a, b, wl.Lx, wl.surface_seed),
                       lambda a, b: W.surface_3d(a, b, 0.0, wl.Lx, wl.surface_seed))
    return s.assemble_rhs(f=torch.tensor(f, dtype=torch.float64, device=dev))
