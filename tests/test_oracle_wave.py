"""Pins of the oracle's stage-loop model (linear free-surface waves in potential form around the
same Poisson solve).

* Dirichlet-to-Neumann closed forms: for surface data cos(kx) (2D) or cos(kx) cos(ly) (3D) over
  a flat bottom the solve plus the surface derivative gives kappa tanh(kappa h) times the data;
  on a mapped mesh (wavy surface) the exact harmonic cos(kx) cosh(k(z+h)) gives
  k cos(kx) sinh(k(eta+h)).
* Standing wave: A cos(kx) returns as -A cos(kx) after half the linear-theory period
  (omega^2 = g k tanh(k h)), through the moving mesh and the five-stage scheme.
"""
import math

import numpy as np

from oracle import assemble, mesh, wave
from tests import oracle_cases as oc

LX, H0, NX, NZ, P = 2.0, 0.5, 8, 2, 8


def model():
    x = oc.fine_x_nodes(NX, P, LX)
    return x, wave.LinearWaves(NX, NZ, P, LX, np.full_like(x, H0))


def test_dtn_closed_form_flat_2d():
    x, W = model()
    k = 2 * math.pi / LX
    m, phi = W.solve_phi(np.zeros_like(x), np.cos(k * x))
    w = wave.surface_dz(m, phi)
    assert np.abs(w - k * math.tanh(k * H0) * np.cos(k * x)).max() < 1e-8


def test_dtn_exact_harmonic_on_mapped_mesh_2d():
    x, W = model()
    k = 2 * math.pi / LX
    eta = 0.03 * np.sin(2 * math.pi * x / LX + 0.4)
    m, phi = W.solve_phi(eta, np.cos(k * x) * np.cosh(k * (eta + H0)))
    w = wave.surface_dz(m, phi)
    assert np.abs(w - k * np.cos(k * x) * np.sinh(k * (eta + H0))).max() < 2e-8


def test_dtn_closed_form_flat_3d():
    Nx, Ny, Nz, p, L = 2, 2, 2, 6, 1.2
    xs = oc.fine_x_nodes(Nx, p, L)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    k, l = math.pi / L, 2 * math.pi / L
    kap = math.hypot(k, l)
    m = mesh.Mesh3D(Nx, Ny, Nz, p, L, L, np.full_like(X, 0.4), np.zeros_like(X))
    A_full = assemble.assemble_stiffness(m)
    A = assemble.masked(A_full, m.dirichlet_nodes())
    data = (np.cos(k * X) * np.cos(l * Y)).ravel()
    phi = assemble.solve_direct(A, assemble.assemble_rhs(m, gD=data, A_full=A_full))
    w = wave.surface_dz(m, phi)
    assert np.abs(w - kap * math.tanh(kap * 0.4) * data).max() < 2e-5 * kap


def test_standing_wave_half_period():
    x, W = model()
    k = 2 * math.pi / LX
    A = 1e-4
    T = 2 * math.pi / math.sqrt(W.g * k * math.tanh(k * H0))
    n = 40
    dt = T / n
    y = np.concatenate([A * np.cos(k * x), np.zeros_like(x)])
    for s in range(n // 2):
        y = W.step(y, s * dt, dt)
    assert np.abs(y[:x.size] + A * np.cos(k * x)).max() < 1e-3 * A
    # the potential passes through zero again at the half period
    assert np.abs(y[x.size:]).max() < 1e-2 * A * W.g * T / (2 * math.pi)
