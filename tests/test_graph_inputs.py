"""Input construction of the dense-subgraph workload (CPU).

The GBS encoding must give a pure Gaussian state whose kernel B (the
symmetric matrix with Q^-1 = I - [[0, B*], [B, 0]] in the a, a-dagger basis,
Q the complex Husimi covariance) is c A up to a global sign: that is what
makes the click statistics favour dense subgraphs.  Checked from the
covariance itself, independently of how it was built.
"""
import numpy as np
import pytest

import gbs_inputs as gi


def _kernel(cov):
    """B of a pure zero-mean state (hbar = 1, interleaved covariance)."""
    m = cov.shape[0] // 2
    perm = np.concatenate([np.arange(0, 2 * m, 2), np.arange(1, 2 * m, 2)])
    s = cov[np.ix_(perm, perm)]                       # xxpp
    W = np.block([[np.eye(m), 1j * np.eye(m)], [np.eye(m), -1j * np.eye(m)]]) / np.sqrt(2)
    Q = W @ s @ W.conj().T + 0.5 * np.eye(2 * m)      # a, a-dagger basis, Husimi
    O = np.eye(2 * m) - np.linalg.inv(Q)
    return O[m:, :m], O[:m, m:]


def test_takagi_and_kernel():
    A, clique = gi.planted_clique_graph(30, 0.5, 8, 3)
    U, lam = gi.takagi_real_symmetric(A)
    assert np.abs(U @ np.diag(lam) @ U.T - A).max() < 1e-12
    assert np.abs(U.conj().T @ U - np.eye(30)).max() < 1e-12
    c = 0.6 / lam.max()
    B, Bc = _kernel(gi.graph_covariance(A, c))
    s = np.sign(np.real(B[np.unravel_index(np.abs(B).argmax(), B.shape)]) * A[np.unravel_index(np.abs(B).argmax(), B.shape)])
    assert np.abs(B - s * c * A).max() < 1e-10
    assert np.abs(Bc - np.conj(B)).max() < 1e-10


def test_planted_clique_and_loss():
    A, clique = gi.planted_clique_graph(200, 0.5, 20, 40)
    assert gi.subgraph_density(A, clique) == 1.0
    assert abs(A.sum() / (200 * 199) - 0.5) < 0.02
    assert np.all(A == A.T) and np.all(np.diag(A) == 0)
    U, lam = gi.takagi_real_symmetric(A)
    cov = gi.graph_covariance(A, 0.5 / lam.max(), eta=0.25)
    cov1 = gi.graph_covariance(A, 0.5 / lam.max())
    assert np.abs(cov - (0.25 * cov1 + 0.75 * 0.5 * np.eye(400))).max() < 1e-12
    with pytest.raises(ValueError):
        gi.graph_covariance(A, 1.0 / lam.max())


def test_calibrate_scale_bisection():
    A, _ = gi.planted_clique_graph(20, 0.5, 5, 1)
    U, lam = gi.takagi_real_symmetric(A)

    def mean_sq(cov):       # any increasing function of c serves the bisection
        return float(np.trace(cov))

    target = mean_sq(gi.graph_covariance(A, 0.37 / lam.max()))
    c = gi.calibrate_scale(A, target, mean_sq)
    assert c * lam.max() == pytest.approx(0.37, rel=1e-9)
