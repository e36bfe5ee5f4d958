"""Training data and training of the learned smoothing stage, driven through the C ABI.

Pairs come from the library's own plain p-multigrid (FP64, Chebyshev(3), levels 8-4-2-1):
sem_learned_harvest runs defect-correction cycles x <- x + B(b - A x) on a training geometry
and, at each cycle, at the point where the stage acts (finest level, after pre-smoothing of the
cycle's residual r), writes element features of r_pre = r - A x_pre and the element-local error
that residual determines, (R_e A R_e^T)^{-1} R_e r_pre (the local solve of the Schwarz smoother,
Sec. 5.3), for a seeded sample of elements.  Right-hand sides: seeded smooth Gaussian sources
and white noise; in addition raw random residuals go through the same feature map so the network
sees every direction of the element residual space.  This module only chooses the geometries
and the seeded inputs; every arithmetic step runs in the library.

Geometries (layout="tank", default): windows of 64 x 16 elements of the 25.6 m wave tank at its
test element size (dx = 0.025 m) with seeded offsets and free surfaces whose seeds are disjoint
from the test surfaces; layout="c1": the 8 x 4 element layout on [0, 2 pi] with seeded depth, bar
and surface.  Training runs on the GPU with the library's BF16 MFMA kernels.
"""
import math

import numpy as np

import workloads as W

from .binding import (Solver, fine_x_nodes, sem_learned_harvest, sem_learned_train,
                      sem_mlp_train)

TANK_L = 25.6
WINDOW = (64, 16)   # elements of one training window (x, z)


def _orders(P):
    o = [P]
    while o[-1] > 1:
        o.append((o[-1] + 1) // 2)
    return o


def training_solver(s, P=8, smoother="chebyshev", layout="tank"):
    """FP64 solver of training geometry s, with the source term it takes: (solver, f(x, z, j)).
    Tank windows smooth as the large tanks do (their Chebyshev degree and interval), so the
    stage-point residuals are drawn from the cycle the stage runs in."""
    if layout == "c1":
        h_fn, eta_fn = W.training_geometry(s)
        x = fine_x_nodes(8, P, 2 * math.pi)
        sv = Solver(2, (8, 1, 4), P, (2 * math.pi,), h_fn(x), eta_fn(x), levels=_orders(P),
                    prec="f64", smoother=smoother)
        return sv, lambda xg, zg, j: W.training_bumps(xg, zg, s, j, h_fn, eta_fn)
    Nx, Nz = WINDOW
    dx = TANK_L / 1024
    x0 = np.random.default_rng(9000 + s).uniform(0.0, TANK_L - Nx * dx)

    def h_fn(a):
        return W.bar_depth(np.asarray(a), TANK_L)

    def eta_fn(a):
        return W.surface(np.asarray(a), TANK_L, 5000 + s)

    x = fine_x_nodes(Nx, P, Nx * dx)
    cheb = W.TANK_CHEB if smoother == "chebyshev" else {}
    sv = Solver(2, (Nx, 1, Nz), P, (Nx * dx,), h_fn(x + x0), eta_fn(x + x0), levels=_orders(P),
                prec="f64", smoother=smoother, **cheb)
    return sv, lambda xg, zg, j: W.bumps(xg + x0, zg, TANK_L, 6000 + 7 * s + j, h_fn, eta_fn)


TANK3_L = 6.4
WINDOW3 = (4, 4, 8)   # hexahedra of one 3D training window (x, y, sigma)


def training_solver3d(s, P=6, smoother="chebyshev"):
    """FP64 solver of 3D training window s: 4 x 4 x 8 hexahedra of the 64 x 64 x 8 tank at its
    element size (0.1 m), seeded offset, the tank's bathymetry and a seeded free surface (seeds
    5000+, disjoint from the tank's); with its source term f(x, y, z, j)."""
    Nx, Ny, Nz = WINDOW3
    dx = TANK3_L / 64
    rng = np.random.default_rng(9500 + s)
    x0, y0 = rng.uniform(0.0, TANK3_L - Nx * dx, size=2)

    def h_fn(a, b):
        return W.bar_depth_3d(np.asarray(a) + x0, np.asarray(b) + y0, TANK3_L, 300)

    def eta_fn(a, b):
        return W.surface_3d(np.asarray(a) + x0, np.asarray(b) + y0, 0.0, TANK3_L, 5000 + s)

    xs = fine_x_nodes(Nx, P, Nx * dx)
    ys = fine_x_nodes(Ny, P, Ny * dx)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    lv = [6, 3, 1] if P == 6 else _orders(P)
    cheb = W.TANK_CHEB if smoother == "chebyshev" else {}
    sv = Solver(3, (Nx, Ny, Nz), P, (Nx * dx, Ny * dx), h_fn(X, Y), eta_fn(X, Y), levels=lv,
                prec="f64", smoother=smoother, **cheb)

    def source(xg, yg, zg, j):
        return W.bumps_3d(np.asarray(xg) + x0, np.asarray(yg) + y0, zg, 0.0, TANK3_L,
                          6100 + 7 * s + j,
                          lambda a, b: W.bar_depth_3d(a, b, TANK3_L, 300),
                          lambda a, b: W.surface_3d(a, b, 0.0, TANK3_L, 5000 + s))
    return sv, source


def _surface_rows(sv):
    """Boolean mask of the free-surface (Dirichlet) rows of a solver's global vectors (the
    vertical index is fastest, so the top node of every vertical line)."""
    c = sv.coords(0)
    xg = c[0]
    same = xg == xg[0]
    if sv.dim == 3:
        same &= c[1] == c[1][0]
    nzn = int(np.count_nonzero(same))   # nodes of one vertical line
    m = np.zeros(sv.n_global, dtype=bool)
    m[nzn - 1::nzn] = True
    return m


def harvest3d(n_windows=16, n_bump=3, n_white=3, n_cycles=6, n_random=8, per=32, P=6, log=None):
    """Device tensors X [n x 7(P+1)^3], T [n x (P+1)^3] (float32) from sem_learned_harvest on
    3D training windows (see training_solver3d)."""
    import torch
    n = (P + 1) ** 3
    E = WINDOW3[0] * WINDOW3[1] * WINDOW3[2]
    each = per if 0 < per < E else E
    calls = n_windows * ((n_bump + n_white) * max(n_cycles, 1) + n_random)
    X = torch.zeros(calls * each, 7 * n, dtype=torch.float32, device="cuda")
    T = torch.zeros(calls * each, n, dtype=torch.float32, device="cuda")
    total = 0

    def dev(a):
        return torch.tensor(a, dtype=torch.float64, device="cuda")

    for s in range(n_windows):
        sv, source = training_solver3d(s, P)
        top = _surface_rows(sv)
        xg, yg, zg = sv.coords(0)
        for j in range(n_bump + n_white):
            if j < n_bump:
                b = sv.assemble_rhs(f=dev(source(xg, yg, zg, j)))
            else:
                bb = np.random.default_rng(8500 + 31 * s + j).standard_normal(sv.n_global)
                bb[top] = 0.0
                b = dev(bb)
            total += sem_learned_harvest(sv.ctx, b, n_cycles, per, 7500 + 97 * s + j,
                                         X[total:], T[total:])
        for j in range(n_random):
            rr = np.random.default_rng(12500 + 53 * s + j).standard_normal(sv.n_global)
            rr[top] = 0.0
            total += sem_learned_harvest(sv.ctx, dev(rr), 0, per, 11500 + 89 * s + j,
                                         X[total:], T[total:])
        sv.close()
        if log:
            log(f"[harvest3d] window {s}: {total} pairs")
    torch.cuda.synchronize()
    return X[:total].contiguous(), T[:total].contiguous()


def harvest(n_surfaces=40, n_bump=4, n_white=4, n_cycles=8, n_random=16, per=32, P=8,
            smoother="chebyshev", layout="tank", max_pairs=None, log=None):
    """Device tensors X [n x 5(P+1)^2], T [n x (P+1)^2] (float32) from sem_learned_harvest.

    per: elements drawn (seeded, inside the library) from each residual; 0 keeps all of them."""
    import torch
    n = (P + 1) ** 2
    E = (WINDOW[0] * WINDOW[1]) if layout == "tank" else 32
    each = per if 0 < per < E else E
    calls = n_surfaces * ((n_bump + n_white) * max(n_cycles, 1) + n_random)
    X = torch.zeros(calls * each, 5 * n, dtype=torch.float32, device="cuda")
    T = torch.zeros(calls * each, n, dtype=torch.float32, device="cuda")
    total = 0

    def dev(a):
        return torch.tensor(a, dtype=torch.float64, device="cuda")

    for s in range(n_surfaces):
        sv, source = training_solver(s, P, smoother, layout)
        top = _surface_rows(sv)
        xg, zg = sv.coords(0)
        for j in range(n_bump + n_white):
            if j < n_bump:
                b = sv.assemble_rhs(f=dev(source(xg, zg, j)))
            else:
                bb = np.random.default_rng(8000 + 31 * s + j).standard_normal(sv.n_global)
                bb[top] = 0.0
                b = dev(bb)
            total += sem_learned_harvest(sv.ctx, b, n_cycles, per, 7000 + 97 * s + j,
                                         X[total:], T[total:])
        for j in range(n_random):
            rr = np.random.default_rng(12000 + 53 * s + j).standard_normal(sv.n_global)
            rr[top] = 0.0   # residuals of the correction problem vanish on the surface
            total += sem_learned_harvest(sv.ctx, dev(rr), 0, per, 11000 + 89 * s + j,
                                         X[total:], T[total:])
        sv.close()
        if log:
            log(f"[harvest] geometry {s}: {total} pairs")
        if max_pairs and total >= max_pairs:
            break
    torch.cuda.synchronize()
    keep = min(total, max_pairs) if max_pairs else total
    return X[:keep].contiguous(), T[:keep].contiguous()


def train(X, T, epochs=600, batch=512, lr=2e-3, seed=1234, val_frac=0.1):
    """Blob of the trained network and its per-epoch (train, validation) losses (no context)."""
    nin, nout = X.shape[1], T.shape[1]
    return sem_mlp_train(X, T, nin, nout, epochs=epochs, batch=batch, lr=lr, val_frac=val_frac,
                         seed=seed)


def train_into(ctx, X, T, epochs=600, batch=512, lr=2e-3, seed=1234, val_frac=0.1):
    """Train the stage network of a solver context (sem_learned_train: the network is loaded
    into it); returns the blob, whose header holds the final training and validation losses."""
    return sem_learned_train(ctx, X, T, epochs=epochs, batch=batch, lr=lr, val_frac=val_frac,
                             seed=seed)
