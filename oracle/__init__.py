"""CPU oracle for threshold-detector GBS click probabilities.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the GPU library
never does, and this package imports nothing from it.

Routes (all compute the same exact quantity, arXiv:1810.00900 Sec. II):

* ``prob`` / ``formP`` / ``formS``  -- the plain definition, in binary128
  (the quadruple precision the paper reports as necessary, Sec. III "Memory"),
  compiled from ``tor_oracle.c``:
  p(C, N) = sum_{Y subset of C} (-1)^{|Y|} det(sigma_Q[Y u N])^{-1/2}.
* ``prob_sequential`` -- the paper's own algorithm (Sec. II update rule):
  measure modes one at a time from the last, keep a signed linear combination
  of Gaussian components, with the coin outcomes fixed in advance as in the
  paper's benchmark mode (Sec. III "Runtime"); the pattern probability is the
  product of the step probabilities.
* ``prob_mp`` / ``torontonian_mp`` -- the definition and the Torontonian form
  Tor(O) = sum_Z (-1)^{n-|Z|} det(I - O_Z)^{-1/2}, O = I - Sigma_C^{-1}, in
  mpmath at high precision (small n only).

parity unpinned: none -- every route is pinned by the closed forms and
invariants in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "tor_oracle.c")


def build(force: bool = True, extra_flags=(), out_path: str | None = None) -> str:
    """Compile tor_oracle.c with gcc (OpenMP, -O2, no fast-math)."""
    out = out_path or _LIB_PATH
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-ffp-contract=off", *extra_flags, _SRC, "-o", out, "-lquadmath", "-lm"]
    if force or not os.path.exists(out):
        subprocess.run(cmd, check=True)
    return out


class _Result(ctypes.Structure):
    _fields_ = [("p_hi", ctypes.c_double), ("p_lo", ctypes.c_double),
                ("t_hi", ctypes.c_double), ("t_lo", ctypes.c_double),
                ("abs_sum", ctypes.c_double), ("pvac_n", ctypes.c_double),
                ("n_terms", ctypes.c_double)]


_lib_cache: dict = {}


def _lib(path: str | None = None):
    path = path or _LIB_PATH
    if path not in _lib_cache:
        if not os.path.exists(path):
            build(out_path=path)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i8p = ctypes.POINTER(ctypes.c_int8)
        for name in ("oracle_formP", "oracle_formS"):
            f = getattr(lib, name)
            f.argtypes = [dp, ctypes.c_int, i8p, ctypes.c_int, ctypes.POINTER(_Result)]
            f.restype = ctypes.c_int
        for name in ("oracle_formP_range", "oracle_formS_range"):
            f = getattr(lib, name)
            f.argtypes = [dp, ctypes.c_int, i8p, ctypes.c_uint64, ctypes.c_uint64,
                          ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_Result)]
            f.restype = ctypes.c_int
        lib.oracle_formP_mean.argtypes = [dp, dp, ctypes.c_int, i8p, ctypes.c_int, ctypes.POINTER(_Result)]
        lib.oracle_formP_mean.restype = ctypes.c_int
        lib.oracle_conditioned.argtypes = [dp, ctypes.c_int, i8p, dp, dp, dp]
        lib.oracle_conditioned.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib_cache[path] = lib
    return _lib_cache[path]


class OracleError(RuntimeError):
    def __init__(self, code: int):
        names = {-1: "EINVAL", -2: "ENOTPD", -3: "ETOOBIG", -4: "ENOMEM"}
        super().__init__(f"oracle error {code} ({names.get(code, '?')})")
        self.code = code


@dataclass
class OracleResult:
    p: float            # probability (hi part)
    p_lo: float         # low part: p_hi + p_lo is the binary128 value to ~106 bits
    T: float            # p / P_vac(N)
    T_lo: float
    abs_sum: float      # sum of |terms| (times P_vac(N)), for the cancellation ratio
    pvac_n: float
    n_terms: float

    @property
    def cancel_ratio(self) -> float:
        return self.abs_sum / abs(self.p) if self.p != 0 else float("inf")


def _prep(cov, pattern):
    cov = np.ascontiguousarray(cov, dtype=np.float64)
    pattern = np.ascontiguousarray(pattern, dtype=np.int8)
    m = pattern.shape[0]
    if cov.shape != (2 * m, 2 * m):
        raise ValueError("cov must be 2m x 2m")
    return cov, pattern, m


def _call(fname, cov, pattern, threads=0, rng=None, lib_path=None):
    cov, pattern, m = _prep(cov, pattern)
    lib = _lib(lib_path)
    res = _Result()
    dp = cov.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    pp = pattern.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
    if rng is None:
        rc = getattr(lib, fname)(dp, m, pp, int(threads), ctypes.byref(res))
    else:
        begin, stride, count = rng
        rc = getattr(lib, fname + "_range")(dp, m, pp, int(begin), int(stride), int(count),
                                             int(threads), ctypes.byref(res))
    if rc != 0:
        raise OracleError(rc)
    return OracleResult(res.p_hi, res.p_lo, res.t_hi, res.t_lo, res.abs_sum, res.pvac_n,
                        res.n_terms)


def formP(cov, pattern, threads: int = 0, lib_path=None) -> OracleResult:
    """Definition route: one Cholesky of sigma_Q[Y u N] per subset (binary128)."""
    return _call("oracle_formP", cov, pattern, threads, lib_path=lib_path)


def formP_mean(cov, mean, pattern, threads: int = 0, lib_path=None) -> OracleResult:
    """Definition route for a displaced state (mean: 2m, hbar = 1, interleaved):
    each vacuum probability gains exp(-mu^T sigma_Q^-1 mu / 2) (binary128)."""
    cov, pattern, m = _prep(cov, pattern)
    mean = np.ascontiguousarray(mean, dtype=np.float64)
    if mean.shape != (2 * m,):
        raise ValueError("mean must have 2m entries")
    lib = _lib(lib_path)
    res = _Result()
    rc = lib.oracle_formP_mean(cov.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               mean.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), m,
                               pattern.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), int(threads),
                               ctypes.byref(res))
    if rc != 0:
        raise OracleError(rc)
    return OracleResult(res.p_hi, res.p_lo, res.t_hi, res.t_lo, res.abs_sum, res.pvac_n, res.n_terms)


def formS(cov, pattern, threads: int = 0, lib_path=None) -> OracleResult:
    """Conditioned route: Schur complement on the no-click modes once, then one
    Cholesky of Sigma_C[Y] per subset (binary128)."""
    return _call("oracle_formS", cov, pattern, threads, lib_path=lib_path)


def formS_range(cov, pattern, begin: int, stride: int, count: int, threads: int = 0):
    """Partial sum of form S over masks begin + j*stride (j < count); used to time
    a bounded sample of a large sum."""
    return _call("oracle_formS", cov, pattern, threads, rng=(begin, stride, count))


def prob(cov, pattern, threads: int = 0) -> OracleResult:
    """Oracle probability: form P when the pattern touches few modes, else form S."""
    pattern = np.asarray(pattern)
    k = int(np.sum(pattern >= 0))
    if k <= 12:
        return formP(cov, pattern, threads)
    return formS(cov, pattern, threads)


def conditioned(cov, pattern):
    """Sigma_C (binary128 as hi/lo arrays) and P_vac(N) from the oracle."""
    cov, pattern, m = _prep(cov, pattern)
    n = int(np.sum(pattern == 1))
    hi = np.zeros((2 * n, 2 * n))
    lo = np.zeros((2 * n, 2 * n))
    pv = ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = _lib().oracle_conditioned(cov.ctypes.data_as(dp), m,
                                   pattern.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                                   hi.ctypes.data_as(dp), lo.ctypes.data_as(dp), ctypes.byref(pv))
    if rc != 0:
        raise OracleError(rc)
    return hi, lo, pv.value


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


# ---------------------------------------------------------------------------
# The paper's sequential algorithm (Sec. II), fixed outcomes (Sec. III).
# ---------------------------------------------------------------------------

def prob_sequential(cov, pattern, dps: int | None = None, steps: bool = False, mean=None):
    """Probability of a click pattern by the paper's mode-by-mode update rule.

    The state is the signed linear combination sum_k a_k rho_k(V_k) (hbar = 2,
    V = 2 sigma, zero mean).  Modes are measured from the last one down, as in
    the paper.  For each component the covariance is split into the remaining
    modes A and the measured mode B; q_k = 2 / sqrt(det(V_B + 1)) and
    p = sum_k a_k q_k is the probability of *no* click.  A no-click outcome keeps
    (a_k q_k / p, V'_A) with V'_A = V_A - V_AB (V_B + 1)^-1 V_AB^T (Eq.
    MatrixUpdate); a click keeps both (a_k / (1-p), V_A) and
    (-a_k q_k / (1-p), V'_A).  An unobserved mode is traced out (V -> V_A).  The
    pattern probability is the product of the step probabilities.

    With ``mean`` (hbar = 1, interleaved, 2m entries) the state is displaced:
    r = sqrt(2) mean in the paper's units, the no-click update also moves the
    mean, r'_A = r_A - V_AB (V_B + 1)^-1 r_B (Sec. II), and q_k gains the
    factor exp(-r_B^T (V_B + 1)^-1 r_B / 2) (the overlap with the vacuum; the
    exponent is printed without the 1/2).
    With ``dps`` set, everything runs in mpmath at that many digits.  With
    ``steps`` the step probabilities are returned too: (total, {mode: P(outcome
    of mode | outcomes of the modes measured before it)}) for observed modes.
    """
    pattern = np.asarray(pattern, dtype=np.int64)
    m = pattern.shape[0]
    if dps is None:
        one = 1.0
        V0 = 2.0 * np.asarray(cov, dtype=np.float64)

        def inv2(B):
            return np.linalg.inv(B)

        def det2(B):
            return B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]

        def sqrt(x):
            return np.sqrt(x)

        def eye2():
            return np.eye(2)
    else:
        import mpmath as mp
        mp.mp.dps = dps
        one = mp.mpf(1)
        V0 = mp.matrix(2 * m, 2 * m)
        for i in range(2 * m):
            for j in range(2 * m):
                V0[i, j] = 2 * mp.mpf(float(cov[max(i, j)][min(i, j)]))

        def inv2(B):
            return B ** -1

        def det2(B):
            return B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]

        def sqrt(x):
            return mp.sqrt(x)

        def eye2():
            return mp.eye(2)

    def block(V, r0, r1, c0, c1):
        if dps is None:
            return V[r0:r1, c0:c1]
        out = mp.matrix(r1 - r0, c1 - c0)
        for i in range(r0, r1):
            for j in range(c0, c1):
                out[i - r0, j - c0] = V[i, j]
        return out

    def transpose(M):
        return M.T

    if mean is None:
        r0 = None
    elif dps is None:
        r0 = np.sqrt(2.0) * np.asarray(mean, dtype=np.float64)
    else:
        r0 = mp.matrix([mp.sqrt(2) * mp.mpf(float(x)) for x in mean])

    def vblock(r, i0, i1):
        if r is None:
            return None
        if dps is None:
            return r[i0:i1]
        out = mp.matrix(i1 - i0, 1)
        for i in range(i0, i1):
            out[i - i0] = r[i]
        return out

    def quad(rB, M):          # rB^T M rB
        if dps is None:
            return float(rB @ M @ rB)
        return (rB.T * M * rB)[0, 0]

    def exp_(x):
        return np.exp(x) if dps is None else mp.exp(x)

    comps = [(one, V0, r0)]
    total = one
    step_p = {}

    def done(value):
        return (value, step_p) if steps else value

    for mode in range(m - 1, -1, -1):
        d = 2 * mode          # size of the remaining block A
        outcome = int(pattern[mode])
        new = []
        if outcome == -1:
            for a, V, r in comps:
                new.append((a, block(V, 0, d, 0, d), vblock(r, 0, d)))
            comps = new
            continue
        qs, updated = [], []
        for a, V, r in comps:
            VA = block(V, 0, d, 0, d)
            VAB = block(V, 0, d, d, d + 2)
            VB = block(V, d, d + 2, d, d + 2)
            VB1 = VB + eye2()
            q = 2 / sqrt(det2(VB1))
            rA, rAp = vblock(r, 0, d), None
            if r is not None:
                rB = vblock(r, d, d + 2)
                W = inv2(VB1)
                q = q * exp_(-quad(rB, W) / 2)
                if d > 0:
                    rAp = rA - (VAB * W * rB if dps is not None else VAB @ W @ rB)
            if d > 0:
                VAp = VA - VAB * inv2(VB1) * transpose(VAB) if dps is not None else \
                    VA - VAB @ inv2(VB1) @ VAB.T
            else:
                VAp = VA
            qs.append(q)
            updated.append((a, VA, VAp, rA, rAp))
        p = sum(a * q for (a, _, _, _, _), q in zip(updated, qs))
        if outcome == 0:
            step_p[mode] = p
            if p == 0:
                return done(0.0 if dps is None else mp.mpf(0))
            total = total * p
            comps = [(a * q / p, VAp, rAp) for (a, _, VAp, _, rAp), q in zip(updated, qs)]
        else:
            pc = one - p
            step_p[mode] = pc
            if pc == 0:
                return done(0.0 if dps is None else mp.mpf(0))
            total = total * pc
            comps = []
            for (a, VA, VAp, rA, rAp), q in zip(updated, qs):
                comps.append((a / pc, VA, rA))
                comps.append((-a * q / pc, VAp, rAp))
    return done(total)


# ---------------------------------------------------------------------------
# mpmath checkers (small n): the definition and the Torontonian form.
# ---------------------------------------------------------------------------

def _mp_sigq(cov, modes, mp):
    k = len(modes)
    M = mp.matrix(2 * k, 2 * k)
    for a in range(2 * k):
        for b in range(2 * k):
            ga = 2 * modes[a // 2] + (a % 2)
            gb = 2 * modes[b // 2] + (b % 2)
            v = mp.mpf(float(cov[max(ga, gb)][min(ga, gb)]))
            if ga == gb:
                v += mp.mpf(1) / 2
            M[a, b] = v
    return M


def prob_mp(cov, pattern, dps: int = 50):
    """The definition, term by term, with mpmath determinants at ``dps`` digits."""
    import mpmath as mp
    mp.mp.dps = dps
    pattern = np.asarray(pattern)
    C = [int(i) for i in np.nonzero(pattern == 1)[0]]
    N = [int(i) for i in np.nonzero(pattern == 0)[0]]
    n = len(C)
    s = mp.mpf(0)
    for mask in range(1 << n):
        Y = [C[i] for i in range(n) if (mask >> i) & 1]
        modes = sorted(Y + N)
        t = mp.mpf(1) if not modes else 1 / mp.sqrt(mp.det(_mp_sigq(cov, modes, mp)))
        s += -t if (len(Y) % 2) else t
    return s


def torontonian_mp(O, dps: int = 50):
    """Tor(O) = sum_{Z subset of [n]} (-1)^{n-|Z|} det(I - O_Z)^{-1/2}, O given as a
    2n x 2n mpmath (or array-like) matrix, modes as 2x2 blocks."""
    import mpmath as mp
    mp.mp.dps = dps
    O = mp.matrix(O)
    n = O.rows // 2
    s = mp.mpf(0)
    for mask in range(1 << n):
        Z = [i for i in range(n) if (mask >> i) & 1]
        k = len(Z)
        if k == 0:
            t = mp.mpf(1)
        else:
            M = mp.matrix(2 * k, 2 * k)
            for a in range(2 * k):
                for b in range(2 * k):
                    ia = 2 * Z[a // 2] + a % 2
                    ib = 2 * Z[b // 2] + b % 2
                    M[a, b] = (1 if a == b else 0) - O[ia, ib]
            t = 1 / mp.sqrt(mp.det(M))
        s += t if ((n - k) % 2 == 0) else -t
    return s


def prob_torontonian_mp(cov, pattern, dps: int = 50):
    """p(C, N) = P_vac(N) * det(Sigma_C)^{-1/2} * Tor(I - Sigma_C^{-1}) in mpmath,
    with Sigma_C the Schur complement of sigma_Q on the no-click modes."""
    import mpmath as mp
    mp.mp.dps = dps
    pattern = np.asarray(pattern)
    C = [int(i) for i in np.nonzero(pattern == 1)[0]]
    N = [int(i) for i in np.nonzero(pattern == 0)[0]]
    SC = _mp_sigq(cov, C, mp)
    pv = mp.mpf(1)
    if N:
        SN = _mp_sigq(cov, N, mp)
        # cross block sigma_Q[C, N]
        X = mp.matrix(2 * len(C), 2 * len(N))
        for a in range(2 * len(C)):
            for b in range(2 * len(N)):
                ga = 2 * C[a // 2] + a % 2
                gb = 2 * N[b // 2] + b % 2
                X[a, b] = mp.mpf(float(cov[max(ga, gb)][min(ga, gb)]))
        SC = SC - X * SN ** -1 * X.T
        pv = 1 / mp.sqrt(mp.det(SN))
    if not C:
        return pv
    O = mp.eye(2 * len(C)) - SC ** -1
    return pv * torontonian_mp(O, dps) / mp.sqrt(mp.det(SC))
