"""Pins of the oracle's GLL rule and derivative matrix (CPU only).

The element basis is the tensor product of Lagrange interpolants on the
Gauss-Lobatto-Legendre points (paper section 2); Algorithm 1 differentiates
with dxm1 and its transpose.  Pinned against textbook closed forms, numpy's
Legendre roots, quadrature exactness and polynomial differentiation.
"""
import math
import os

import numpy as np
import pytest

from bruteforce import gll_numpy, lagrange_deriv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gll_lobatto_closed_forms.txt")


def _load_golden():
    rows = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        n, node, weight = line.split()
        ev = lambda s: eval(s, {"__builtins__": {}}, {"sqrt": math.sqrt})  # noqa: E731
        rows.setdefault(int(n), []).append((ev(node), ev(weight)))
    return rows


def test_gll_textbook_values(oracle_mod):
    for N, pts in _load_golden().items():
        xi, w = oracle_mod.gll(N)
        np.testing.assert_allclose(xi, [p[0] for p in pts], rtol=0, atol=2e-16)
        np.testing.assert_allclose(w, [p[1] for p in pts], rtol=0, atol=4e-16)


@pytest.mark.parametrize("N", range(1, 20))
def test_gll_against_numpy_roots(oracle_mod, N):
    xi, w = oracle_mod.gll(N)
    xr, wr = gll_numpy(N)
    np.testing.assert_allclose(xi, xr, rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, wr, rtol=1e-13, atol=0)
    assert abs(w.sum() - 2.0) < 1e-14
    np.testing.assert_allclose(xi, -xi[::-1], atol=1e-15)
    np.testing.assert_allclose(w, w[::-1], rtol=1e-14)


@pytest.mark.parametrize("N", range(1, 18))
def test_gll_quadrature_exactness(oracle_mod, N):
    xi, w = oracle_mod.gll(N)
    for k in range(0, 2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13, (N, k)
    # degree 2N is NOT integrated exactly by a Lobatto rule
    k = 2 * N
    assert abs(np.dot(w, xi ** k) - 2.0 / (k + 1)) > 1e-11


@pytest.mark.parametrize("N", range(1, 18))
def test_derivative_matrix(oracle_mod, N):
    xi, _ = oracle_mod.gll(N)
    D = oracle_mod.deriv(N, xi)
    P = N + 1
    scale = max(1.0, N * N)
    # differentiates every polynomial of degree <= N exactly
    for k in range(0, N + 1):
        dk = k * xi ** (k - 1) if k > 0 else np.zeros(P)
        assert np.max(np.abs(D @ xi ** k - dk)) < 1e-13 * scale, (N, k)
    # row sums vanish (derivative of a constant)
    assert np.max(np.abs(D.sum(axis=1))) < 1e-13 * scale
    # diagonal closed form
    diag = np.zeros(P)
    diag[0], diag[N] = -N * (N + 1) / 4.0, N * (N + 1) / 4.0
    np.testing.assert_allclose(np.diag(D), diag, atol=1e-13)
    # centro-antisymmetry D[i][j] = -D[N-i][N-j]
    np.testing.assert_allclose(D, -D[::-1, ::-1], atol=1e-13 * scale)
    # independent construction from explicit Lagrange polynomials
    Db = lagrange_deriv(gll_numpy(N)[0])
    np.testing.assert_allclose(D, Db, atol=1e-10 * scale)
