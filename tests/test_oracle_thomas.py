"""Pins of the column solve (Appendix B, Alg. "Tridiagonal matrix algorithm")
against library and exact-arithmetic references."""
import math
from fractions import Fraction

import numpy as np
import pytest


def column_matrix(s, Tz):
    nz = len(s)
    D = np.zeros((nz, nz))
    for k in range(nz):
        D[k, k] = s[k] + Tz[k] + Tz[k + 1]
        if k > 0:
            D[k, k - 1] = -Tz[k]
        if k < nz - 1:
            D[k, k + 1] = -Tz[k + 1]
    return D


@pytest.mark.parametrize("nz", [1, 2, 3, 16, 128])
def test_excess_form_matches_dense_solve(orc, nz):
    rng = np.random.default_rng(nz)
    s = rng.uniform(0.1, 2.0, nz)
    Tz = np.concatenate([[0.0], rng.uniform(0.0, 5.0, nz - 1), [0.0]])
    g = rng.standard_normal(nz)
    w = orc.column_solve(s, Tz, g)
    ref = np.linalg.solve(column_matrix(s, Tz), g)
    np.testing.assert_allclose(w, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("n", [1, 2, 5, 40])
def test_printed_algorithm_matches_dense_solve(orc, n):
    """The algorithm in the paper's own notation (a diagonal, b super, c sub)."""
    rng = np.random.default_rng(100 + n)
    b = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    a = np.abs(b) + np.abs(c) + rng.uniform(0.5, 1.5, n)
    f = rng.standard_normal(n)
    M = np.diag(a)
    for i in range(n - 1):
        M[i, i + 1] = b[i]
        M[i + 1, i] = c[i + 1]
    u = orc.thomas_plain(a, b, c, f)
    np.testing.assert_allclose(u, np.linalg.solve(M, f), rtol=1e-12, atol=1e-14)


def test_excess_and_printed_forms_agree(orc):
    """On moderate coefficient ranges both eliminations give the same answer."""
    rng = np.random.default_rng(5)
    nz = 50
    s = rng.uniform(0.5, 1.0, nz)
    Tz = np.concatenate([[0.0], rng.uniform(0.0, 10.0, nz - 1), [0.0]])
    g = rng.standard_normal(nz)
    a = s + Tz[:-1] + Tz[1:]
    b = -Tz[1:]
    c = -Tz[:-1]
    np.testing.assert_allclose(orc.column_solve(s, Tz, g), orc.thomas_plain(a, b, c, g),
                               rtol=1e-11)


@pytest.mark.parametrize("m", [0, 1, 5, 31])
def test_neumann_cosine_mode(orc, m):
    """Constant coupling T and excess s: cos(pi m (k+1/2)/nz) (DCT-II) is an
    eigenvector of the Neumann column matrix with eigenvalue s + 4T sin^2(pi m/(2nz))."""
    nz, T, s0 = 32, 7.5, 0.3
    s = np.full(nz, s0)
    Tz = np.concatenate([[0.0], np.full(nz - 1, T), [0.0]])
    k = np.arange(nz)
    v = np.cos(math.pi * m * (k + 0.5) / nz)
    lam = s0 + 4 * T * math.sin(math.pi * m / (2 * nz)) ** 2
    np.testing.assert_allclose(orc.column_solve(s, Tz, v), v / lam, rtol=0, atol=1e-13)


def exact_solve(s, Tz, g):
    """Gaussian elimination on the tridiagonal system in rational arithmetic."""
    nz = len(s)
    S = [Fraction(x) for x in s]
    T = [Fraction(x) for x in Tz]
    G = [Fraction(x) for x in g]
    diag = [S[k] + T[k] + T[k + 1] for k in range(nz)]
    sup = [-T[k + 1] for k in range(nz)]
    for k in range(1, nz):
        fac = -T[k] / diag[k - 1]
        diag[k] -= fac * sup[k - 1]
        G[k] -= fac * G[k - 1]
    w = [Fraction(0)] * nz
    w[-1] = G[-1] / diag[-1]
    for k in range(nz - 2, -1, -1):
        w[k] = (G[k] - sup[k] * w[k + 1]) / diag[k]
    return np.array([float(x) for x in w])


def test_extreme_anisotropy_exact(orc):
    """Vertical couplings 1e18 times the excess, as at the bottom of the graded
    grids: the excess-form elimination stays accurate to rounding, compared with
    an exact rational solve."""
    nz = 12
    rng = np.random.default_rng(2)
    s = rng.uniform(0.5, 1.0, nz)
    Tz = np.concatenate([[0.0], 10.0 ** rng.uniform(14, 18, nz - 1), [0.0]])
    g = rng.standard_normal(nz)
    ref = exact_solve(s, Tz, g)
    w = orc.column_solve(s, Tz, g)
    np.testing.assert_allclose(w, ref, rtol=1e-13)
    # the assembled diagonal loses the excess to rounding: the printed form drifts
    a = s + Tz[:-1] + Tz[1:]
    plain = orc.thomas_plain(a, -Tz[1:], -Tz[:-1], g)
    assert np.abs(plain - ref).max() > 1e3 * np.abs(w - ref).max()
