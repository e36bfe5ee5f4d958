"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds NONE of the solver's arithmetic: no quadrature, no differentiation, no
geometric factors.  It only defines the analytic input fields (bathymetry h(x), free surface
eta(x), right-hand-side bumps f(x, z), manufactured solutions and their boundary data) and the
mesh sizes of each workload, all evaluated at coordinates the caller supplies.  Each side (the
CPU oracle and the HIP library) computes its own node coordinates.

Workloads (wave-tank shaped, after the paper's submerged-bar test, Sec. 6.2: still-water depth
0.4 m over 0.1 m on the bar, incident wavelength 3.74 m so kh = 0.67 at h = 0.4):
  c1  manufactured sin(x) cosh(z+1) on [0, 2pi] x [-1, 0], 8 x 4 elements, P = 4, levels 4-2-1,
      Jacobi(2,2);
  c2  tank 256 x 8, P = 6, L_x = 25.6, levels 6-3-1, Chebyshev(3), FP64;
  c3  tank 2048 x 16, P = 8, levels 8-4-2-1, FP32 inner (G in FP32 or BF16);
  c4  tank 1024 x 16, P = 8, learned stage, test surfaces 1000..1019;
  c5  3D tank 64 x 64 x 8, P = 6, L = 6.4, levels 6-3-1.
The bar is a trapezoid of our own (the paper's figure is not available): depth 0.4, linear
ramp to 0.1 over [4, 7] L/16, flat to 9 L/16, linear back to 0.4 at 11 L/16.
"""
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

G_ACC = 9.81                  # gravitational acceleration used by the surface dispersion
K0 = 2.0 * math.pi / 3.74     # incident wave number of the bar test


@dataclass
class Workload:
    name: str
    dim: int
    Nx: int
    Nz: int
    P: int
    Lx: float
    Ny: int = 1
    Ly: float = 0.0
    orders: List[int] = field(default_factory=list)
    smoother: str = "chebyshev"       # "jacobi" | "chebyshev"
    nu_pre: int = 2
    nu_post: int = 2
    cheb_degree: int = 3
    cheb_degree_coarse: int = 0       # Chebyshev degree below the finest level (0: cheb_degree)
    cheb_lo: float = 0.1              # Chebyshev interval [cheb_lo, cheb_hi] x lambda_hat
    cheb_hi: float = 1.1
    kind: str = "tank"                # "manufactured" | "tank" | "tank3d"
    surface_seed: int = 7
    rhs_seed: int = 107
    tol: float = 1e-10
    Pz: Optional[int] = None          # 2D: order along sigma when it differs from P (along x)

    @property
    def pz(self):
        return self.P if self.Pz is None else self.Pz

    @property
    def n_global(self):
        if self.dim == 2:
            return (self.Nx * self.P + 1) * (self.Nz * self.pz + 1)
        return (self.Nx * self.P + 1) * (self.Ny * self.P + 1) * (self.Nz * self.P + 1)

    @property
    def n_elements(self):
        return self.Nx * self.Nz * (self.Ny if self.dim == 3 else 1)


# Chebyshev smoothing of the large tanks (1024 and 2048 x 16, P = 8; 64 x 64 x 8, P = 6) and of
# the windows the learned stage is trained on: degree 6 on [0.02, 1.1] x lambda_hat (the c2 tank
# keeps Chebyshev(3) on [0.1, 1.1])
TANK_CHEB = dict(cheb_degree=6, cheb_lo=0.02, cheb_hi=1.1)


def c1(P=4):
    return Workload("c1", 2, 8, 4, P, 2.0 * math.pi, orders=_orders(P), smoother="jacobi",
                    nu_pre=2, nu_post=2, kind="manufactured", tol=1e-12)


def c2():
    return Workload("c2", 2, 256, 8, 6, 25.6, orders=[6, 3, 1])


def c3():
    return Workload("c3", 2, 2048, 16, 8, 25.6, orders=[8, 4, 2, 1], **TANK_CHEB)


def c4(test_index=0):
    return Workload("c4", 2, 1024, 16, 8, 25.6, orders=[8, 4, 2, 1],
                    surface_seed=1000 + test_index, rhs_seed=2000 + test_index, **TANK_CHEB)


def c5():
    return Workload("c5", 3, 64, 8, 6, 6.4, Ny=64, Ly=6.4, orders=[6, 3, 1], kind="tank3d",
                    surface_seed=300, rhs_seed=301, **TANK_CHEB)


def tank(Nx, Nz, P, Lx=25.6, orders=None, name="tank", surface_seed=7, rhs_seed=107,
         smoother="chebyshev"):
    return Workload(name, 2, Nx, Nz, P, Lx, orders=orders or _orders(P),
                    surface_seed=surface_seed, rhs_seed=rhs_seed, smoother=smoother)


def tank_semi(Nx, Nz, Px, Pz, Lx=25.6, name="tank_semi", surface_seed=7, rhs_seed=107,
              smoother="chebyshev"):
    """2D tank with order Px along x and Pz along sigma; the level orders are left to the
    solver (empty list: its own semi-coarsened hierarchy)."""
    return Workload(name, 2, Nx, Nz, Px, Lx, orders=[], surface_seed=surface_seed,
                    rhs_seed=rhs_seed, smoother=smoother, Pz=Pz)


def tank3d(Nx, Ny, Nz, P, L=6.4, orders=None, name="tank3d", surface_seed=300, rhs_seed=301):
    return Workload(name, 3, Nx, Nz, P, L, Ny=Ny, Ly=L, orders=orders or _orders(P),
                    kind="tank3d", surface_seed=surface_seed, rhs_seed=rhs_seed)


def _orders(P):
    out = [P]
    while out[-1] > 1:
        out.append((out[-1] + 1) // 2)
    return out


# ---------------------------------------------------------------------------------------
# analytic fields
# ---------------------------------------------------------------------------------------
def bar_depth(x, Lx=25.6):
    """Still-water depth h(x) of the trapezoidal bar: 0.4 -> 0.1 -> 0.4."""
    x = np.asarray(x, dtype=np.float64)
    a, b, c, d = 4 * Lx / 16, 7 * Lx / 16, 9 * Lx / 16, 11 * Lx / 16
    h = np.full_like(x, 0.4)
    up = (x > a) & (x < b)
    h[up] = 0.4 - 0.3 * (x[up] - a) / (b - a)
    h[(x >= b) & (x <= c)] = 0.1
    dn = (x > c) & (x < d)
    h[dn] = 0.1 + 0.3 * (x[dn] - c) / (d - c)
    return h


def surface_params(seed, n=5):
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.0, 0.005, n)
    amp = np.where(amp == 0.0, 0.005, amp)
    modes = rng.integers(1, 65, n)
    phase = rng.uniform(0.0, 2.0 * math.pi, n)
    return amp, modes, phase


def surface(x, Lx, seed):
    """eta(x) = 0.02 sin(k0 x) + sum_j a_j sin(2 pi m_j x / Lx + phi_j), a_j <= 0.005."""
    x = np.asarray(x, dtype=np.float64)
    amp, modes, phase = surface_params(seed)
    eta = 0.02 * np.sin(K0 * x)
    for a, m, ph in zip(amp, modes, phase):
        eta = eta + a * np.sin(2.0 * math.pi * m * x / Lx + ph)
    return eta


def bump_params(seed, Lx, n=8):
    rng = np.random.default_rng(seed)
    return dict(c=rng.uniform(-1.0, 1.0, n), xm=rng.uniform(0.05, 0.95, n) * Lx,
                sm=rng.uniform(0.2, 0.8, n), lx=rng.uniform(0.5, 2.0, n),
                lz=rng.uniform(0.05, 0.15, n))


def bumps(x, z, Lx, seed, h_fn, eta_fn):
    """Smooth Gaussian source f(x, z): 8 seeded bumps centred at (x_m, -h + sigma_m (h+eta))."""
    p = bump_params(seed, Lx)
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    f = np.zeros_like(x)
    for c, xm, sm, lx, lz in zip(p["c"], p["xm"], p["sm"], p["lx"], p["lz"]):
        hm = float(h_fn(np.array([xm]))[0])
        em = float(eta_fn(np.array([xm]))[0])
        zm = -hm + sm * (hm + em)
        f += c * np.exp(-(x - xm) ** 2 / (2 * lx * lx) - (z - zm) ** 2 / (2 * lz * lz))
    return f


# ---- 3D tank -----------------------------------------------------------------------------
def bar_params_3d(seed, L):
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-15.0, 15.0) * math.pi / 180.0
    xc = rng.uniform(0.4, 0.6) * L
    yc = rng.uniform(0.4, 0.6) * L
    return theta, xc, yc


def _smoothstep(y):
    # f_g(y) = -2 y^3 + 3 y^2 (the relaxation-zone blend of the paper's appendix)
    y = np.clip(y, 0.0, 1.0)
    return -2.0 * y ** 3 + 3.0 * y ** 2


def bar_depth_3d(x, y, L=6.4, seed=300):
    """Bar profile along the rotated coordinate xi (centred on the tank), C^1 ramps."""
    theta, xc, yc = bar_params_3d(seed, L)
    xi = (np.asarray(x) - xc) * math.cos(theta) + (np.asarray(y) - yc) * math.sin(theta)
    s = xi + 0.5 * L      # shift so the profile sits inside [0, L] along xi
    a, b, c, d = 4 * L / 16, 7 * L / 16, 9 * L / 16, 11 * L / 16
    up = _smoothstep((s - a) / (b - a))
    dn = _smoothstep((s - c) / (d - c))
    return 0.4 - 0.3 * up + 0.3 * dn


def surface_3d(x, y, t, L=6.4, seed=300):
    """eta = 0.02 sin(k0 x - w0 t) + 5 seeded harmonics with integer wave vectors in [-16,16]^2,
    w^2 = g |k| tanh(0.4 |k|)."""
    rng = np.random.default_rng(seed + 1)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w0 = math.sqrt(G_ACC * K0 * math.tanh(0.4 * K0))
    eta = 0.02 * np.sin(K0 * x - w0 * t)
    for _ in range(5):
        a = rng.uniform(0.0, 0.005)
        kx, ky = rng.integers(-16, 17, 2)
        if kx == 0 and ky == 0:
            kx = 1
        ph = rng.uniform(0.0, 2.0 * math.pi)
        kv = 2.0 * math.pi * np.array([kx, ky]) / L
        kk = float(np.hypot(*kv))
        w = math.sqrt(G_ACC * kk * math.tanh(0.4 * kk))
        eta = eta + a * np.sin(kv[0] * x + kv[1] * y - w * t + ph)
    return eta


def bumps_3d(x, y, z, t, L=6.4, seed=301, h_fn=None, eta_fn=None):
    """8 Gaussian bumps whose centres drift at <= 0.1 m/s."""
    rng = np.random.default_rng(seed)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    f = np.zeros_like(x)
    for _ in range(8):
        c = rng.uniform(-1.0, 1.0)
        x0, y0 = rng.uniform(0.1, 0.9, 2) * L
        vx, vy = rng.uniform(-0.07, 0.07, 2)
        sm = rng.uniform(0.2, 0.8)
        lh = rng.uniform(0.2, 0.6)
        lz = rng.uniform(0.05, 0.15)
        xm, ym = x0 + vx * t, y0 + vy * t
        hm = float(h_fn(np.array([xm]), np.array([ym]))[0])
        em = float(eta_fn(np.array([xm]), np.array([ym]))[0])
        zm = -hm + sm * (hm + em)
        f += c * np.exp(-((x - xm) ** 2 + (y - ym) ** 2) / (2 * lh * lh) - (z - zm) ** 2 / (2 * lz * lz))
    return f


# ---- manufactured solutions ----------------------------------------------------------------
def mms_c1(x, z):
    """u = sin(x) cosh(z + 1): harmonic, so f = 0."""
    return np.sin(x) * np.cosh(z + 1.0)


def mms_c1_neumann(z_left, z_right, x_bottom):
    """Outward normal derivatives on the walls x = 0, x = 2 pi and the flat bottom z = -1."""
    return {"left": -np.cosh(np.asarray(z_left) + 1.0),
            "right": np.cos(2.0 * math.pi) * np.cosh(np.asarray(z_right) + 1.0),
            "bottom": -np.sin(np.asarray(x_bottom)) * np.sinh(0.0)}


def mms_wave(x, z, k, h0):
    """u = cos(k x) cosh(k (z + h0)): harmonic; zero normal derivative on walls x = 0, x = m pi/k
    and on the flat bottom z = -h0."""
    return np.cos(k * x) * np.cosh(k * (z + h0))


# ---- training geometries for the learned stage ---------------------------------------------
def training_geometry(s):
    """Seeded (h, eta) functions of surface s on the config-1 layout domain x in [0, 2 pi]:
    mean depth H_s ~ U(0.5, 3) with a smooth seeded bar of relative height <= 0.6 (aspect ratios
    of the 8 x 4 elements from about 1 to 8) and a 5-harmonic free surface, amplitude <= 0.02 H."""
    rng = np.random.default_rng(5000 + s)
    H = rng.uniform(0.5, 3.0)
    frac = rng.uniform(0.0, 0.6)
    c0 = rng.uniform(1.0, 2 * math.pi - 1.0)
    w = rng.uniform(0.5, 2.0)
    amps = rng.uniform(0.0, 0.02 * H / 5, 5)
    modes = rng.integers(1, 9, 5)
    phases = rng.uniform(0.0, 2 * math.pi, 5)

    def h(x):
        x = np.asarray(x, dtype=np.float64)
        return H * (1.0 - frac * np.exp(-((x - c0) / w) ** 2))

    def eta(x):
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros_like(x)
        for a, m, ph in zip(amps, modes, phases):
            out = out + a * np.sin(m * x + ph)
        return out

    return h, eta


def training_bumps(x, z, s, j, h_fn, eta_fn):
    """8 seeded Gaussian sources (right-hand side j of training surface s)."""
    L = 2 * math.pi
    rng = np.random.default_rng(7000 + 97 * s + j)
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    f = np.zeros_like(x)
    for _ in range(8):
        c = rng.uniform(-1.0, 1.0)
        xm = rng.uniform(0.05, 0.95) * L
        sm = rng.uniform(0.2, 0.8)
        lx = rng.uniform(0.2, 1.0)
        hm = float(h_fn(np.array([xm]))[0])
        em = float(eta_fn(np.array([xm]))[0])
        zm = -hm + sm * (hm + em)
        lz = rng.uniform(0.05, 0.2) * hm
        f += c * np.exp(-(x - xm) ** 2 / (2 * lx * lx) - (z - zm) ** 2 / (2 * lz * lz))
    return f


def random_vector(n, seed):
    return np.random.default_rng(seed).standard_normal(n)
