"""Pins of the oracle's low-storage Runge-Kutta stage loop (Sec. 3).

The coefficients are checked by what a five-stage fourth-order scheme must satisfy, not by
retyping them: the stability polynomial equals exp's Taylor series through z^4 (exactly, in
rational arithmetic), the global error on nonlinear problems falls by 2^4 when dt halves, and
the stage values of y' = 1 land on the stage times.
"""
import math
from fractions import Fraction

import numpy as np

from oracle import lserk


def test_stability_polynomial_matches_exp_to_fourth_order():
    R = lserk.stability_polynomial()
    for k in range(5):
        assert abs(R[k] - Fraction(1, math.factorial(k))) < Fraction(1, 10 ** 11), (k, float(R[k]))
    # a fifth-order term remains (the scheme is fourth order, not fifth)
    assert abs(float(R[5]) - 1.0 / 120.0) > 1e-4


def _integrate(f, y0, t1, n):
    y, dt = np.array(y0, dtype=np.float64), t1 / n
    for s in range(n):
        y = lserk.step(f, y, s * dt, dt)
    return y


def test_fourth_order_convergence_nonlinear():
    # y' = y cos t, y(0) = 1: y = exp(sin t)
    f = lambda y, t: y * np.cos(t)
    errs = [abs(_integrate(f, [1.0], 2.0, n)[0] - math.exp(math.sin(2.0))) for n in (10, 20, 40)]
    assert 14.0 < errs[0] / errs[1] < 18.0 and 14.0 < errs[1] / errs[2] < 18.0, errs
    # a 2 x 2 nonlinear system (Lotka-Volterra) against a fine reference
    g = lambda y, t: np.array([y[0] * (1.0 - y[1]), y[1] * (y[0] - 1.0)])
    ref = _integrate(g, [1.5, 0.5], 3.0, 2560)
    e = [np.abs(_integrate(g, [1.5, 0.5], 3.0, n) - ref).max() for n in (20, 40, 80)]
    assert 13.0 < e[0] / e[1] < 19.0 and 13.0 < e[1] / e[2] < 19.0, e


def test_stage_times():
    """On y' = 1 from y = 0, the state seen by stage k is c_k dt (the times f is evaluated at
    are consistent with the state), and one step gives dt."""
    seen = []
    dt = 0.3
    y1 = lserk.step(lambda y, t: np.ones_like(y), np.zeros(1), 0.0, dt,
                    stage_hook=lambda k, y, tk: seen.append((float(y[0]), tk)))
    a, b, c = lserk.coefficients()
    for k, (yk, tk) in enumerate(seen):
        assert abs(yk - c[k] * dt) < 1e-14 and abs(tk - c[k] * dt) < 1e-15
    assert abs(y1[0] - dt) < 1e-14
    # y' = t: one step integrates the linear function exactly
    y2 = lserk.step(lambda y, t: np.full_like(y, t), np.zeros(1), 0.0, dt)
    assert abs(y2[0] - dt * dt / 2) < 1e-14
