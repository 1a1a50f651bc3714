"""CPU tests of the library's host-side Schwarz factors (no GPU): the 1-D
generalised eigenvectors that the fast-diagonalisation local solves use must
diagonalise the oracle's 1-D stiffness and mass of the extended element
(oracle.schwarz.one_d, pinned against brute-force assembly), on the same kept
index range, for every side combination."""
import itertools

import numpy as np
import pytest

from oracle.schwarz import one_d


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9, 12])
@pytest.mark.parametrize("ell", [0.3, 1.7])
def test_fdm_factors_diagonalise_oracle_1d(oracle_mod, N, ell):
    import paper_2109_03592_amd as sem
    xi, w = oracle_mod.gll(N)
    D = oracle_mod.deriv(N, xi)
    for left, right in itertools.product((0, 1, 2), repeat=2):
        if N == 1 and left == 1 and right == 1:
            continue  # no unknown left in a one-element Dirichlet-Dirichlet line
        A1, B1, kept = one_d(N, xi, w, D, ell, left, right)
        S, lam, lo = sem.fdm_1d(N, ell, left, right)
        assert lo == kept[0] and S.shape == (len(kept), len(kept)), (left, right)
        eye = S.T @ (B1[:, None] * S)
        assert np.max(np.abs(eye - np.eye(len(kept)))) <= 1e-12, (left, right)
        lamA = S.T @ A1 @ S
        scale = max(1.0, float(np.max(np.abs(lam))))
        assert np.max(np.abs(lamA - np.diag(lam))) <= 1e-12 * scale, (left, right)
        # the spectrum is that of the generalised problem (a reference eigensolver)
        ref = np.sort(np.linalg.eigvalsh(A1 / np.sqrt(np.outer(B1, B1))))
        assert np.max(np.abs(np.sort(lam) - ref)) <= 1e-12 * scale, (left, right)


def test_fdm_argument_checks():
    import paper_2109_03592_amd as sem
    from paper_2109_03592_amd import _lib as L
    for args in ((0, 1.0, 0, 0), (18, 1.0, 0, 0), (3, 0.0, 0, 0), (3, 1.0, 3, 0), (3, 1.0, 0, -1)):
        with pytest.raises(L.SemError) as e:
            sem.fdm_1d(*args)
        assert e.value.status == L.SEM_EINVAL
