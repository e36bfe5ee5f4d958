"""Pins of the oracle's 1D building blocks against closed forms and library quadrature."""
import math

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

from oracle import gll


def test_recurrence_start_and_p2():
    # Sec. 4.3: P~0 = 1/sqrt(2), P~1 = sqrt(3/2) x; the recurrence then gives
    # P~2 = sqrt(5/2) (3x^2 - 1)/2 (orthonormal Legendre, textbook closed form).
    x = np.linspace(-1, 1, 7)
    p = gll.legendre_orthonormal(2, x)
    assert np.allclose(p[0], 1 / math.sqrt(2), atol=0, rtol=1e-15)
    assert np.allclose(p[1], math.sqrt(1.5) * x, atol=1e-16)
    assert np.allclose(p[2], math.sqrt(2.5) * (3 * x * x - 1) / 2, atol=1e-15)


@pytest.mark.parametrize("N", [3, 8, 14])
def test_orthonormality_gauss_legendre(N):
    xg, wg = npleg.leggauss(N + 2)          # exact for degree <= 2N+3
    p = gll.legendre_orthonormal(N, xg)
    G = (p * wg) @ p.T
    assert np.abs(G - np.eye(N + 1)).max() < 1e-13


@pytest.mark.parametrize("N", [1, 4, 9])
def test_derivative_of_recurrence(N):
    x = np.linspace(-0.95, 0.95, 11)
    h = 1e-6
    fd = (gll.legendre_orthonormal(N, x + h) - gll.legendre_orthonormal(N, x - h)) / (2 * h)
    assert np.abs(gll.legendre_orthonormal_deriv(N, x) - fd).max() < 1e-7


def test_gll_closed_forms():
    r2, w2 = gll.gll_nodes(2), gll.gll_weights(2)
    assert np.allclose(r2, [-1, 0, 1], atol=0)
    assert np.allclose(w2, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    r4, w4 = gll.gll_nodes(4), gll.gll_weights(4)
    s = math.sqrt(3 / 7)
    assert np.allclose(r4, [-1, -s, 0, s, 1], atol=1e-15)
    assert np.allclose(w4, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)
    r3, w3 = gll.gll_nodes(3), gll.gll_weights(3)
    t = 1 / math.sqrt(5)
    assert np.allclose(r3, [-1, -t, t, 1], atol=1e-15)
    assert np.allclose(w3, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("P", [1, 2, 3, 5, 8, 12])
def test_gll_exactness(P):
    r, w = gll.gll_nodes(P), gll.gll_weights(P)
    assert abs(w.sum() - 2) < 1e-14
    for k in range(0, 2 * P):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((w * r ** k).sum() - exact) < 1e-13
    # degree 2P is NOT integrated exactly (P >= 1): the rule is sharp
    assert abs((w * r ** (2 * P)).sum() - 2.0 / (2 * P + 1)) > 1e-9


@pytest.mark.parametrize("P", [2, 4, 7, 10])
def test_diff_matrix(P):
    D = gll.diff_matrix(P)
    r = gll.gll_nodes(P)
    assert np.abs(D @ np.ones(P + 1)).max() < 1e-12
    for m in range(1, P + 1):
        assert np.abs(D @ r ** m - m * r ** (m - 1)).max() < 1e-11 * max(1, P * P)
    assert np.abs(D - gll.diff_matrix_closed_form(P)).max() < 1e-11 * P * P


@pytest.mark.parametrize("pc,pf", [(1, 2), (2, 4), (3, 6), (4, 8), (1, 8)])
def test_transfer_reproduces_polynomials(pc, pf):
    J = gll.transfer_matrix(pc, pf)
    rc, rf = gll.gll_nodes(pc), gll.gll_nodes(pf)
    assert J.shape == (pf + 1, pc + 1)
    for m in range(pc + 1):
        assert np.abs(J @ rc ** m - rf ** m).max() < 1e-13
    # end points and coinciding nodes carry delta rows
    assert np.abs(J[0] - np.eye(pc + 1)[0]).max() < 1e-14
    assert np.abs(J[-1] - np.eye(pc + 1)[-1]).max() < 1e-14
    # interpolating back down is the identity on coarse polynomials
    Jd = gll.transfer_matrix(pf, pc)
    assert np.abs(Jd @ J - np.eye(pc + 1)).max() < 1e-13
