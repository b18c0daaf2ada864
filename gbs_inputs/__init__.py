"""Seeded synthetic inputs for threshold-detector Gaussian boson sampling.

This module only *generates* inputs: Haar-random interferometers, squeezing
parameters, the resulting pure-state covariance matrices and click patterns.
It contains none of the probability arithmetic, so both the CPU oracle and the
GPU library can consume its outputs without sharing any of the method's code.

Conventions (used everywhere in this repository):

* hbar = 1: the vacuum covariance is I/2.
* quadratures are interleaved per mode, (x1, p1, x2, p2, ...), as in the
  paper's definition of the quadrature vector (Sec. II, Eq. 1).
* the paper uses hbar = 2 (vacuum V = I); the two are related by V = 2 * sigma.
* GBS inputs are squeezed vacua and so zero-mean; displaced states carry a
  mean vector in the same interleaved order and units (a coherent state
  |alpha> has mean (sqrt(2) Re alpha, sqrt(2) Im alpha) and covariance I/2).

The benchmark states of the paper (Sec. III, "Memory") are 8 dB squeezed
inputs sent through Haar-random interferometers; the workloads below use the
same construction with the squeezing ranges of the benchmark configurations.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar_unitary",
    "gbs_covariance",
    "single_mode_covariance",
    "direct_sum",
    "tmsv_covariance",
    "thermal_covariance",
    "apply_loss",
    "random_click_set",
    "marginal_pattern",
    "full_pattern",
    "state_config1",
    "state_config2",
    "state_m800",
    "config5_pattern",
    "config3_queries",
    "random_product_state",
    "random_mean",
    "coherent_mean",
    "planted_clique_graph",
    "takagi_real_symmetric",
    "graph_covariance",
    "calibrate_scale",
    "subgraph_density",
]


def haar_unitary(m: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random m x m unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal moved into Q (Mezzadri, Notices AMS 54, 2007);
    without that phase fix the distribution is not Haar."""
    z = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    ph = d / np.abs(d)
    return q * ph[None, :]


def _xxpp_to_interleaved(mat: np.ndarray) -> np.ndarray:
    m = mat.shape[0] // 2
    perm = np.empty(2 * m, dtype=np.int64)
    perm[0::2] = np.arange(m)          # x_i
    perm[1::2] = np.arange(m) + m      # p_i
    return mat[np.ix_(perm, perm)]


def _symmetrize_exact(a: np.ndarray) -> np.ndarray:
    """Return a matrix that is bit-exactly symmetric (lower triangle mirrored)."""
    low = np.tril(a)
    return low + np.tril(a, -1).T


def gbs_covariance(U: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Covariance (hbar = 1, interleaved) of single-mode squeezed vacua with
    squeezing r_i sent through the interferometer U.

    S = S_U * diag(e^{-r}, e^{+r}) in xxpp order with
    S_U = [[Re U, -Im U], [Im U, Re U]], sigma = S S^T / 2.
    The result is made bit-exactly symmetric.
    """
    U = np.asarray(U, dtype=np.complex128)
    r = np.asarray(r, dtype=np.float64)
    m = U.shape[0]
    SU = np.block([[U.real, -U.imag], [U.imag, U.real]])
    sq = np.concatenate([np.exp(-r), np.exp(r)])
    S = SU * sq[None, :]
    sig = (S @ S.T) / 2.0
    sig = _xxpp_to_interleaved(sig)
    return np.ascontiguousarray(_symmetrize_exact(sig))


def single_mode_covariance(r: float = 0.0, phi: float = 0.0, nbar: float = 0.0) -> np.ndarray:
    """2x2 covariance (hbar = 1) of a squeezed thermal state: thermal
    occupation nbar, squeezing r along angle phi."""
    c, s = np.cos(phi), np.sin(phi)
    R = np.array([[c, -s], [s, c]])
    D = np.diag([np.exp(-2 * r), np.exp(2 * r)]) * (nbar + 0.5)
    return _symmetrize_exact(R @ D @ R.T)


def direct_sum(blocks) -> np.ndarray:
    """Block-diagonal covariance of a product state (one 2x2 block per mode)."""
    m = len(blocks)
    out = np.zeros((2 * m, 2 * m))
    for i, b in enumerate(blocks):
        out[2 * i:2 * i + 2, 2 * i:2 * i + 2] = b
    return out


def tmsv_covariance(r: float) -> np.ndarray:
    """Two-mode squeezed vacuum (hbar = 1, interleaved x1,p1,x2,p2)."""
    ch, sh = np.cosh(2 * r), np.sinh(2 * r)
    s = 0.5 * np.array([
        [ch, 0, sh, 0],
        [0, ch, 0, -sh],
        [sh, 0, ch, 0],
        [0, -sh, 0, ch],
    ])
    return _symmetrize_exact(s)


def thermal_covariance(nbar) -> np.ndarray:
    nbar = np.atleast_1d(np.asarray(nbar, dtype=np.float64))
    return np.diag(np.repeat(nbar + 0.5, 2))


def apply_loss(sigma: np.ndarray, eta: float) -> np.ndarray:
    """Uniform pure loss with transmission eta: sigma -> eta sigma + (1-eta) I/2."""
    out = eta * sigma + (1.0 - eta) * 0.5 * np.eye(sigma.shape[0])
    return _symmetrize_exact(out)


def random_click_set(m: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform n-subset of range(m), sorted ascending."""
    return np.sort(rng.choice(m, size=n, replace=False)).astype(np.int64)


def marginal_pattern(m: int, clicks) -> np.ndarray:
    """int8 pattern: 1 at the clicked modes, -1 (unobserved) elsewhere."""
    p = np.full(m, -1, dtype=np.int8)
    p[np.asarray(clicks, dtype=np.int64)] = 1
    return p


def full_pattern(m: int, clicks) -> np.ndarray:
    """int8 pattern: 1 at the clicked modes, 0 (no click) elsewhere."""
    p = np.zeros(m, dtype=np.int8)
    p[np.asarray(clicks, dtype=np.int64)] = 1
    return p


# ---- the benchmark workloads -------------------------------------------------

def state_config1(seed: int = 1) -> np.ndarray:
    """m = 8 modes, Haar U, r_i ~ U[0.5, 1.0]."""
    rng = np.random.default_rng(seed)
    U = haar_unitary(8, rng)
    r = rng.uniform(0.5, 1.0, size=8)
    return gbs_covariance(U, r)


def state_config2(seed: int = 2, m: int = 100, r: float = 0.6) -> np.ndarray:
    """m = 100 modes, Haar U, r_i = 0.6 on every mode."""
    rng = np.random.default_rng(seed)
    U = haar_unitary(m, rng)
    return gbs_covariance(U, np.full(m, r))


def state_m800(seed: int, m: int = 800) -> np.ndarray:
    """m = 800 modes, Haar U, r_i ~ U[0.3, 0.9] (serving and large-Torontonian states)."""
    rng = np.random.default_rng(seed)
    U = haar_unitary(m, rng)
    r = rng.uniform(0.3, 0.9, size=m)
    return gbs_covariance(U, r)


def config5_pattern(n: int, seed: int = 50, m: int = 800) -> np.ndarray:
    """Click set of the large single Torontonians: a uniform n-subset of the
    m modes, drawn from a stream seeded by (seed, n); marginal semantics."""
    rng = np.random.default_rng([seed, n])
    return marginal_pattern(m, random_click_set(m, n, rng))


def config3_queries(nq: int, n_states: int = 4, seed: int = 34, m: int = 800,
                    n_lo: int = 8, n_hi: int = 24):
    """Query stream of the serving workload: (state index, n, marginal pattern)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nq):
        s = int(rng.integers(n_states))
        n = int(rng.integers(n_lo, n_hi + 1))
        out.append((s, n, marginal_pattern(m, random_click_set(m, n, rng))))
    return out


def random_product_state(m: int, rng: np.random.Generator):
    """Random product of squeezed thermal single-mode states; returns the
    covariance and the list of 2x2 blocks."""
    blocks = [single_mode_covariance(rng.uniform(0.1, 1.0), rng.uniform(0, np.pi),
                                     rng.uniform(0.0, 0.5)) for _ in range(m)]
    return direct_sum(blocks), blocks


def random_mean(m: int, rng: np.random.Generator, scale: float = 0.5) -> np.ndarray:
    """Random displacement: 2m independent normal quadrature means (hbar = 1)."""
    return scale * rng.standard_normal(2 * m)


def coherent_mean(alpha) -> np.ndarray:
    """Mean vector (hbar = 1, interleaved) of the coherent states |alpha_k>."""
    alpha = np.atleast_1d(np.asarray(alpha, dtype=np.complex128))
    out = np.empty(2 * alpha.shape[0])
    out[0::2] = np.sqrt(2.0) * alpha.real
    out[1::2] = np.sqrt(2.0) * alpha.imag
    return out


# ---------------------------------------------------------------------------
# Graph workloads (dense-subgraph search with GBS, Sec. IV): the graph is
# encoded in the squeezing and interferometer of a pure Gaussian state whose
# kernel is proportional to the adjacency matrix.  Only input construction
# lives here; the mean click number used to pick the scale comes from the
# caller (the library or the oracle).


def planted_clique_graph(n: int = 200, p: float = 0.5, k: int = 20, seed: int = 40):
    """Erdos-Renyi G(n, p) with a clique planted on k uniformly chosen
    vertices.  Returns (adjacency as float64 0/1, sorted clique vertices)."""
    rng = np.random.default_rng(seed)
    up = np.triu(rng.random((n, n)) < p, 1)
    A = (up | up.T).astype(np.float64)
    clique = np.sort(rng.choice(n, k, replace=False))
    A[np.ix_(clique, clique)] = 1.0
    np.fill_diagonal(A, 0.0)
    return A, clique


def takagi_real_symmetric(A: np.ndarray):
    """Takagi factorisation A = U diag(lam) U^T (lam >= 0, U unitary) of a real
    symmetric matrix: from its eigendecomposition, with the columns of
    negative eigenvalues multiplied by i."""
    mu, V = np.linalg.eigh(np.asarray(A, dtype=np.float64))
    U = V.astype(np.complex128) * np.where(mu < 0, 1j, 1.0)[None, :]
    return U, np.abs(mu)


def graph_covariance(A: np.ndarray, c: float, eta: float = 1.0) -> np.ndarray:
    """Covariance (hbar = 1, interleaved) of the GBS encoding of the graph A at
    scale c (0 < c max|eig A| < 1): squeezing r_i = artanh(c lam_i) into the
    Takagi unitary of A, so that the state's kernel is c A up to a global
    sign; then uniform loss with transmission eta."""
    U, lam = takagi_real_symmetric(A)
    if not (0.0 < c * lam.max() < 1.0):
        raise ValueError("scale c must satisfy 0 < c * max|eig A| < 1")
    cov = gbs_covariance(U, np.arctanh(c * lam))
    return apply_loss(cov, eta) if eta != 1.0 else cov


def calibrate_scale(A: np.ndarray, target: float, mean_clicks, eta: float = 1.0, iters: int = 60) -> float:
    """Scale c at which mean_clicks(graph_covariance(A, c, eta)) equals target,
    by bisection on (0, 1 / max|eig A|) (the mean click number grows with c)."""
    lam_max = np.abs(np.linalg.eigvalsh(np.asarray(A, dtype=np.float64))).max()
    lo, hi = 0.0, (1.0 - 1e-9) / lam_max
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mean_clicks(graph_covariance(A, mid, eta)) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def subgraph_density(A: np.ndarray, vertices) -> float:
    """Edge density of the subgraph of A induced by `vertices`."""
    v = np.asarray(vertices)
    k = len(v)
    if k < 2:
        return 0.0
    return float(A[np.ix_(v, v)].sum() / (k * (k - 1)))
