"""Oracle: the low-storage explicit Runge-Kutta stage loop (test infrastructure only).

Sec. 3 ("Temporal discretization") advances dy/dt = f(y, t) with an s-stage low-storage scheme:
    y^(0) = y^n, K^0 = 0,
    K^k = alpha_k K^(k-1) + dt f(y^(k-1), t_n + c_k dt),
    y^(k) = y^(k-1) + beta_k K^k,   k = 1..s,      y^(n+1) = y^(s),
and uses only the five-stage fourth-order member (Carpenter and Kennedy 1994).  The paper does
not print its coefficients; those below are the published five-stage fourth-order 2N-storage
solution of Carpenter and Kennedy (NASA TM-109112, 1994), as rational numbers.  They are pinned
by what they must satisfy, not by retyping: the scheme's stability polynomial on y' = lambda y
equals the Taylor series of exp(lambda dt) through the fourth power, the global error on
nonlinear problems falls sixteen-fold when dt halves, and on y' = 1 the stage values sit at the
stage times c_k dt.

In the solver each stage needs a pressure solve on that stage's geometry (eq. poissonp); the
preconditioner is kept time-constant (Sec. 5.4), built once from the small-amplitude
(still-water, eta = 0) geometry, while the operator follows the stage's surface.
"""
from fractions import Fraction

import numpy as np

ALPHA = [Fraction(0), Fraction(-567301805773, 1357537059087),
         Fraction(-2404267990393, 2016746695238), Fraction(-3550918686646, 2091501179385),
         Fraction(-1275806237668, 842570457699)]
BETA = [Fraction(1432997174477, 9575080441755), Fraction(5161836677717, 13612068292357),
        Fraction(1720146321549, 2090206949498), Fraction(3134564353537, 4481467310338),
        Fraction(2277821191437, 14882151754819)]
C = [Fraction(0), Fraction(1432997174477, 9575080441755),
     Fraction(2526269341429, 6820363962896), Fraction(2006345519317, 3224310063776),
     Fraction(2802321613138, 2924317926251)]
STAGES = 5


def coefficients():
    """(alpha, beta, c) as float64 arrays."""
    return (np.array([float(a) for a in ALPHA]), np.array([float(b) for b in BETA]),
            np.array([float(c) for c in C]))


def step(f, y, t, dt, stage_hook=None):
    """One time step of the low-storage scheme; f(y, t) -> dy/dt.  stage_hook(k, y, t_k), if
    given, sees the state and time each stage's right-hand side is evaluated at."""
    a, b, c = coefficients()
    y = np.array(y, dtype=np.float64, copy=True)
    K = np.zeros_like(y)
    for k in range(STAGES):
        tk = t + c[k] * dt
        if stage_hook is not None:
            stage_hook(k, y, tk)
        K = a[k] * K + dt * np.asarray(f(y, tk), dtype=np.float64)
        y = y + b[k] * K
    return y


def stability_polynomial():
    """Coefficients R_0..R_5 of R(z) = y^(n+1) / y^n for y' = lambda y, z = lambda dt, in exact
    rational arithmetic (the stage recursion applied to polynomials in z)."""
    def mul(p, q):
        out = [Fraction(0)] * (len(p) + len(q) - 1)
        for i, x in enumerate(p):
            for j, w in enumerate(q):
                out[i + j] += x * w
        return out

    def add(p, q):
        n = max(len(p), len(q))
        return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0) for i in range(n)]

    y = [Fraction(1)]
    K = [Fraction(0)]
    z = [Fraction(0), Fraction(1)]
    for k in range(STAGES):
        K = add([ALPHA[k] * v for v in K], mul(z, y))
        y = add(y, [BETA[k] * v for v in K])
    return y
