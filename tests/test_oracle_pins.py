"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each pin is independent of the oracle's own arithmetic: closed forms written
from the state parameters (not from the covariance matrix), exact invariants of
a probability distribution, the paper's own sequential algorithm (Sec. II,
fixed outcomes as in Sec. III "Runtime"), and mpmath at high precision.
A mutation test (at the end) plants plausible mistakes in a copy of the oracle
and checks that every mutant fails at least one pin.
"""
import itertools
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import gbs_inputs as gi
import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def _pat(*v):
    return np.array(v, dtype=np.int8)


# --------------------------------------------------------------------------
# pins, written so they can run against any build of the oracle library
# --------------------------------------------------------------------------

def pin_vacuum(lib=None):
    """Vacuum: no clicks with probability 1, any click pattern exactly 0."""
    cov = 0.5 * np.eye(10)
    for route in (oracle.formP, oracle.formS):
        assert route(cov, _pat(0, 0, 0, 0, 0), lib_path=lib).p == 1.0
        assert route(cov, _pat(-1, 0, -1, 0, -1), lib_path=lib).p == 1.0
        for pat in ([1, 0, 0, 0, 0], [1, 1, -1, 0, 1], [1, 1, 1, 1, 1]):
            assert route(cov, np.array(pat, np.int8), lib_path=lib).p == 0.0


def pin_single_mode(lib=None):
    """Squeezed (thermal) single mode: P(no click) = 1/sqrt(det sigma_Q) with the
    closed form det = (nbar+1/2)^2 + (nbar+1/2) cosh 2r + 1/4, which is cosh^2 r
    for a pure squeezed vacuum (q_k of Eq. (prob) at zero mean)."""
    for r, phi, nbar in [(0.6, 0.0, 0.0), (0.3, 1.1, 0.0), (1.2, 2.0, 0.0),
                         (0.0, 0.0, 0.7), (0.5, 0.4, 0.3)]:
        cov = gi.single_mode_covariance(r, phi, nbar)
        det = (nbar + 0.5) ** 2 + (nbar + 0.5) * np.cosh(2 * r) + 0.25
        pvac = 1.0 / np.sqrt(det)
        for route in (oracle.formP, oracle.formS):
            assert route(cov, _pat(0), lib_path=lib).p == pytest.approx(pvac, rel=1e-15)
            assert route(cov, _pat(1), lib_path=lib).p == pytest.approx(1 - pvac, rel=1e-14)
    # pure squeezed vacuum: P(click) = 1 - 1/cosh r
    for r in (0.1, 0.6, 0.92, 1.5):
        cov = gi.single_mode_covariance(r)
        assert oracle.formP(cov, _pat(1), lib_path=lib).p == pytest.approx(1 - 1 / np.cosh(r), rel=1e-14)


def pin_thermal(lib=None):
    """Thermal state: P(vac) = 1/(1 + nbar) per mode, independent modes."""
    nb = np.array([0.2, 1.5, 0.05])
    cov = gi.thermal_covariance(nb)
    q = 1.0 / (1.0 + nb)
    assert oracle.formP(cov, _pat(0, 0, 0), lib_path=lib).p == pytest.approx(np.prod(q), rel=1e-15)
    assert oracle.formS(cov, _pat(1, 0, 1), lib_path=lib).p == pytest.approx(
        (1 - q[0]) * q[1] * (1 - q[2]), rel=1e-14)


def _product_closed_form(params, pattern):
    p = 1.0
    for (r, phi, nbar), v in zip(params, pattern):
        det = (nbar + 0.5) ** 2 + (nbar + 0.5) * np.cosh(2 * r) + 0.25
        q = 1.0 / np.sqrt(det)
        if v == 1:
            p *= 1 - q
        elif v == 0:
            p *= q
    return p


def pin_product(lib=None, m=7, seed=3):
    """Product states factorise: p = prod_C (1 - q_i) prod_N q_j."""
    rng = np.random.default_rng(seed)
    params = [(rng.uniform(0.1, 1.0), rng.uniform(0, np.pi), rng.uniform(0, 0.5)) for _ in range(m)]
    cov = gi.direct_sum([gi.single_mode_covariance(*p) for p in params])
    for _ in range(6):
        pat = rng.integers(-1, 2, size=m).astype(np.int8)
        want = _product_closed_form(params, pat)
        for route in (oracle.formP, oracle.formS):
            assert route(cov, pat, lib_path=lib).p == pytest.approx(want, rel=1e-13, abs=1e-300)


def pin_tmsv(lib=None):
    """Two-mode squeezed vacuum: photon numbers are perfectly correlated, so
    P(click, no click) = 0, P(no click, no click) = 1/cosh^2 r,
    P(click, click) = 1 - 1/cosh^2 r, and one mode alone is thermal with
    nbar = sinh^2 r, P(click) = tanh^2 r."""
    for r in (0.3, 0.7, 1.1):
        cov = gi.tmsv_covariance(r)
        for route in (oracle.formP, oracle.formS):
            # the FP64 input is a TMSV only to ~1e-16, so "0" is ~1e-16
            assert abs(route(cov, _pat(1, 0), lib_path=lib).p) < 1e-15
            assert abs(route(cov, _pat(0, 1), lib_path=lib).p) < 1e-15
            assert route(cov, _pat(0, 0), lib_path=lib).p == pytest.approx(1 / np.cosh(r) ** 2, rel=1e-14)
            assert route(cov, _pat(1, 1), lib_path=lib).p == pytest.approx(1 - 1 / np.cosh(r) ** 2, rel=1e-14)
            assert route(cov, _pat(1, -1), lib_path=lib).p == pytest.approx(np.tanh(r) ** 2, rel=1e-14)


def pin_normalisation(lib=None, m=8, seed=1):
    """The 2^m click patterns of a state form a distribution: they sum to 1."""
    cov = gi.state_config1(seed) if m == 8 else gi.gbs_covariance(
        gi.haar_unitary(m, np.random.default_rng(seed)),
        np.random.default_rng(seed + 100).uniform(0.3, 1.0, m))
    tot = 0.0
    for bits in itertools.product((0, 1), repeat=m):
        p = oracle.formP(cov, np.array(bits, np.int8), lib_path=lib).p
        assert p >= -1e-15
        tot += p
    assert tot == pytest.approx(1.0, abs=1e-13)


def pin_paper_algorithm(lib=None, seed=5):
    """The paper's sequential update rule (Sec. II) with fixed outcomes gives
    the same pattern probability as the subset sum."""
    rng = np.random.default_rng(seed)
    m = 5
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 1.0, m))
    for pat in ([1, 1, 1, 1, 1], [1, 0, 1, -1, 0], [0, 1, -1, 1, 1], [-1, -1, 1, 0, 1]):
        pat = np.array(pat, np.int8)
        want = float(oracle.prob_sequential(cov, pat, dps=40))
        for route in (oracle.formP, oracle.formS):
            assert route(cov, pat, lib_path=lib).p == pytest.approx(want, rel=1e-13)


PINS = [pin_vacuum, pin_single_mode, pin_thermal, pin_product, pin_tmsv,
        pin_normalisation, pin_paper_algorithm]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(pin, oracle_lib):
    pin()


# --------------------------------------------------------------------------
# further invariants and cross-route checks
# --------------------------------------------------------------------------

def test_normalisation_m10(oracle_lib):
    pin_normalisation(m=10, seed=7)


def test_marginal_consistency(oracle_lib):
    """p(C, N; j unobserved) = p(C + j, N) + p(C, N + j) (the POVM elements of
    one mode sum to the identity)."""
    rng = np.random.default_rng(11)
    cov = gi.gbs_covariance(gi.haar_unitary(9, rng), rng.uniform(0.3, 1.0, 9))
    for _ in range(8):
        pat = rng.integers(-1, 2, size=9).astype(np.int8)
        j = int(rng.integers(9))
        pat[j] = -1
        a = pat.copy(); a[j] = 1
        b = pat.copy(); b[j] = 0
        lhs = oracle.formP(cov, pat)
        rhs = oracle.formP(cov, a).p + oracle.formP(cov, b).p
        assert lhs.p == pytest.approx(rhs, rel=1e-13)


def test_permutation_invariance(oracle_lib):
    """Relabelling modes (both quadratures together) leaves p unchanged."""
    rng = np.random.default_rng(12)
    m = 8
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 1.0, m))
    pat = np.array([1, 1, 0, -1, 1, 0, 1, -1], np.int8)
    perm = rng.permutation(m)
    q = np.empty(2 * m, np.int64)
    q[0::2] = 2 * perm
    q[1::2] = 2 * perm + 1
    cov2 = np.ascontiguousarray(cov[np.ix_(q, q)])
    pat2 = pat[perm]
    assert oracle.formP(cov2, pat2).p == pytest.approx(oracle.formP(cov, pat).p, rel=1e-14)
    assert oracle.formS(cov2, pat2).p == pytest.approx(oracle.formS(cov, pat).p, rel=1e-14)


def test_routes_agree_mpmath(oracle_lib):
    """Definition (binary128), conditioned route, mpmath definition, mpmath
    Torontonian form and the paper's algorithm agree."""
    cov = gi.state_config1()
    for pat in ([1] * 8, [1, 0, 1, 1, 0, -1, 1, 0], [0, 0, 1, -1, -1, 1, 0, 1]):
        pat = np.array(pat, np.int8)
        a = oracle.formP(cov, pat)
        b = oracle.formS(cov, pat)
        c = oracle.prob_mp(cov, pat, dps=50)
        d = oracle.prob_torontonian_mp(cov, pat, dps=50)
        e = oracle.prob_sequential(cov, pat, dps=50)
        ref = float(c)
        assert abs(float(d - c)) < 1e-40
        assert abs(float(e - c)) < 1e-40
        # binary128 with cancellation ratio R: error ~ R * 1e-33
        assert abs((a.p + a.p_lo) - ref) <= 1e-28 * abs(ref) * a.cancel_ratio
        assert abs((b.p + b.p_lo) - ref) <= 1e-28 * abs(ref) * b.cancel_ratio


def test_complementary_minor_route(oracle_lib):
    """The identity behind full patterns on an inverted state: with
    K = sigma_Q^-1 and G = K[C], p(C, N) = (-1)^n det(sigma_Q)^-1/2 T(G) when
    every mode is observed (Jacobi: det sigma_Q[S] = det sigma_Q det K[S^c]).
    Evaluated by brute force in mpmath (inverse, determinants and the subset
    sum of G) against the oracle's definition route."""
    import mpmath as mp
    mp.mp.dps = 60
    rng = np.random.default_rng(160)
    m = 7
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.9, m))
    d = 2 * m
    sq = mp.matrix(d, d)
    for a in range(d):
        for b in range(d):
            sq[a, b] = mp.mpf(float(cov[a, b])) + (mp.mpf(1) / 2 if a == b else 0)
    K = sq ** -1
    rdet = mp.det(sq) ** (-mp.mpf(1) / 2)
    for clicks in ([2], [0, 5], [1, 3, 6], [0, 2, 4, 6], list(range(m))):
        pat = gi.full_pattern(m, clicks)
        n = len(clicks)
        rows = [2 * c + t for c in clicks for t in (0, 1)]
        T = mp.mpf(0)
        for mask in range(1 << n):
            sub = [rows[2 * i + t] for i in range(n) if mask >> i & 1 for t in (0, 1)]
            det = mp.det(mp.matrix([[K[a, b] for b in sub] for a in sub])) if sub else mp.mpf(1)
            T += (-1) ** bin(mask).count("1") / mp.sqrt(det)
        want = (-1) ** n * rdet * T
        o = oracle.formP(cov, pat)
        got = mp.mpf(o.p) + mp.mpf(o.p_lo)
        assert abs(got - want) <= 1e-28 * abs(want) * max(o.cancel_ratio, 1.0)


def test_information_form_route(oracle_lib):
    """The identity behind full patterns of an inverted displaced state: with
    K = sigma_Q^-1, h = K mu, G = K[C], and Z the clicked modes left out of a
    term, det sigma_Q[S] = det sigma_Q det K[Z] and
    mu_S^T sigma_Q[S]^-1 mu_S = mu^T K mu - h_Z^T K[Z]^-1 h_Z, so
    p(C, N) = (-1)^n det(sigma_Q)^-1/2 exp(-mu^T K mu / 2)
              sum_Z (-1)^|Z| det(G[Z])^-1/2 exp(+h_Z^T G[Z]^-1 h_Z / 2).
    Brute force in mpmath against the oracle's definition route with means."""
    import mpmath as mp
    mp.mp.dps = 60
    rng = np.random.default_rng(161)
    m = 6
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.8, m))
    mean = gi.random_mean(m, rng, 0.5)
    d = 2 * m
    sq = mp.matrix(d, d)
    for a in range(d):
        for b in range(d):
            sq[a, b] = mp.mpf(float(cov[a, b])) + (mp.mpf(1) / 2 if a == b else 0)
    mu = mp.matrix([mp.mpf(float(x)) for x in mean])
    K = sq ** -1
    h = K * mu
    pre = mp.det(sq) ** (-mp.mpf(1) / 2) * mp.exp(-(mu.T * K * mu)[0] / 2)
    for clicks in ([4], [1, 3], [0, 2, 5], list(range(m))):
        pat = gi.full_pattern(m, clicks)
        n = len(clicks)
        rows = [2 * c + t for c in clicks for t in (0, 1)]
        T = mp.mpf(0)
        for mask in range(1 << n):
            sub = [rows[2 * i + t] for i in range(n) if mask >> i & 1 for t in (0, 1)]
            term = mp.mpf(1)
            if sub:
                Gz = mp.matrix([[K[a, b] for b in sub] for a in sub])
                hz = mp.matrix([h[a] for a in sub])
                term = mp.exp((hz.T * Gz ** -1 * hz)[0] / 2) / mp.sqrt(mp.det(Gz))
            T += (-1) ** bin(mask).count("1") * term
        want = (-1) ** n * pre * T
        o = oracle.formP_mean(cov, mean, pat)
        got = mp.mpf(o.p) + mp.mpf(o.p_lo)
        assert abs(got - want) <= 1e-28 * abs(want) * max(o.cancel_ratio, 1.0), clicks


def test_product_state_many_clicks(oracle_lib):
    """A product state with 14 clicks: heavy cancellation (R ~ 1e7+), closed
    form known, so binary128 accuracy is pinned at a size where FP64 fails."""
    rng = np.random.default_rng(21)
    m = 14
    params = [(rng.uniform(0.2, 0.5), rng.uniform(0, np.pi), 0.0) for _ in range(m)]
    cov = gi.direct_sum([gi.single_mode_covariance(*p) for p in params])
    pat = np.ones(m, np.int8)
    want = _product_closed_form(params, pat)
    res = oracle.formS(cov, pat)
    assert res.cancel_ratio > 1e6
    assert res.p == pytest.approx(want, rel=1e-12)


def test_tmsv_pairs_many_clicks(oracle_lib):
    """Six independent two-mode squeezed pairs, all 12 modes clicked:
    p = prod_k (1 - 1/cosh^2 r_k)."""
    rs = [0.3, 0.45, 0.6, 0.75, 0.9, 1.05]
    cov = np.zeros((24, 24))
    for k, r in enumerate(rs):
        cov[4 * k:4 * k + 4, 4 * k:4 * k + 4] = gi.tmsv_covariance(r)
    want = np.prod([1 - 1 / np.cosh(r) ** 2 for r in rs])
    res = oracle.formS(cov, np.ones(12, np.int8))
    assert res.p == pytest.approx(want, rel=1e-12)


def test_errors(oracle_lib):
    cov = 0.5 * np.eye(4)
    with pytest.raises(oracle.OracleError):
        oracle.formP(cov, np.array([1, 2], np.int8))
    bad = cov.copy()
    bad[0, 0] = -3.0
    with pytest.raises(oracle.OracleError):
        oracle.formP(bad, np.array([1, 1], np.int8))
    nan = cov.copy()
    nan[1, 0] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.formS(nan, np.array([1, 1], np.int8))


# --------------------------------------------------------------------------
# planted mistakes: each mutant of the oracle must fail at least one pin
# --------------------------------------------------------------------------

MUTANTS = {
    "sign_dropped": (r"if \(__builtin_popcountll\(mask\) & 1\) s -= t; else s \+= t;", "s += t;"),
    "sign_dropped_S": (r"if \(k & 1\) s -= t; else s \+= t;", "s += t;"),
    "no_half_identity": (r"if \(ga == gb\) v \+= \(qf\)0\.5;", ""),
    "wrong_quadrature_index": (r"int ga = 2 \* modes\[a / 2\] \+ \(a & 1\);", "int ga = 2 * modes[a / 2];"),
    "det_power_minus_one": (r"prod /= ljj;", "prod /= s;"),
    "schur_sign": (r"sig_c\[a \* dc \+ b\] -= v;", "sig_c[a * dc + b] += v;"),
    "forgot_no_click_modes": (r"modes\[k\+\+\] = nidx\[ni\+\+\];", "ni++;"),
    "transposed_cross_block": (r"qf v = sigq\(cov, m, 2 \* nidx\[i / 2\] \+ \(i & 1\), gc\);",
                               "qf v = sigq(cov, m, 2 * nidx[i / 2] + 1 - (i & 1), gc);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    src = open(os.path.join(os.path.dirname(oracle.__file__), "tor_oracle.c")).read()
    pat, rep = MUTANTS[name]
    mutated, k = re.subn(pat, rep, src)
    assert k >= 1, f"mutation {name} did not apply"
    path = tmp_path / "mut.c"
    path.write_text(mutated)
    so = str(tmp_path / f"libmut_{name}.so")
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", str(path), "-o", so,
                    "-lquadmath", "-lm"], check=True)
    failed = []
    for pin in PINS:
        try:
            pin(lib=so)
        except (AssertionError, oracle.OracleError):
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"


# ---------------------------------------------------------------------------
# Displaced states (means): each vacuum probability gains the Gaussian
# overlap factor exp(-mu^T sigma_Q^-1 mu / 2).  Pinned to closed forms that do
# not go through that formula.

def _mean_of(alphas):
    """hbar = 1 quadrature means of coherent amplitudes, interleaved."""
    out = np.empty(2 * len(alphas))
    out[0::2] = np.sqrt(2) * np.real(alphas)
    out[1::2] = np.sqrt(2) * np.imag(alphas)
    return out


def test_displaced_coherent_states_through_interferometer():
    """Coherent states stay a product of coherent states (beta = U alpha):
    P = prod_clicks (1 - e^{-|beta|^2}) prod_no_clicks e^{-|beta|^2}."""
    rng = np.random.default_rng(71)
    m = 6
    U = gi.haar_unitary(m, rng)
    alpha = rng.normal(0, 0.6, m) + 1j * rng.normal(0, 0.6, m)
    beta = U @ alpha
    cov = gi.gbs_covariance(U, np.zeros(m))
    pat = np.array([1, 0, 1, -1, 1, 0], np.int8)
    want = 1.0
    for i in range(m):
        if pat[i] == 1:
            want *= 1 - np.exp(-abs(beta[i]) ** 2)
        elif pat[i] == 0:
            want *= np.exp(-abs(beta[i]) ** 2)
    o = oracle.formP_mean(cov, _mean_of(beta), pat)
    assert abs((o.p + o.p_lo) - want) <= 1e-14 * want
    assert float(oracle.prob_sequential(cov, pat, mean=_mean_of(beta), dps=40)) == pytest.approx(want, rel=1e-13)


def test_displaced_tmsv_closed_forms():
    """Two-mode squeezed vacuum with both modes displaced: from the Fock
    expansion sech r sum_n tanh^n r |n, n>, the vacuum amplitude is
    sech r exp(-(|a|^2 + |b|^2)/2 + tanh r a* b*), so
    P_vac(a, b) = sech^2 r exp(-|a|^2 - |b|^2 + 2 tanh r Re(a b)); each mode
    alone is displaced thermal with nbar = sinh^2 r:
    P_vac(a) = exp(-|a|^2 / cosh^2 r) / cosh^2 r.  Click patterns follow by
    inclusion-exclusion; (1, 0) and (0, 1) need the conditioned mean."""
    r = 0.7
    a, b = 0.5 - 0.3j, -0.2 + 0.6j
    cov = gi.tmsv_covariance(r)
    mean = _mean_of([a, b])
    c2 = np.cosh(r) ** 2
    pa = np.exp(-abs(a) ** 2 / c2) / c2
    pb = np.exp(-abs(b) ** 2 / c2) / c2
    pab = np.exp(-abs(a) ** 2 - abs(b) ** 2 + 2 * np.tanh(r) * (a * b).real) / c2
    want = {(0, 0): pab, (1, 0): pb - pab, (0, 1): pa - pab, (1, 1): 1 - pa - pb + pab,
            (1, -1): 1 - pa, (-1, 0): pb}
    for pat, w in want.items():
        pat = np.array(pat, np.int8)
        o = oracle.formP_mean(cov, mean, pat)
        assert abs((o.p + o.p_lo) - w) <= 1e-14, (pat, o.p, w)
        s = oracle.prob_sequential(cov, pat, mean=mean, dps=40)
        assert abs(float(s) - w) <= 1e-14, (pat, float(s), w)


def test_displaced_zero_mean_limit_and_routes_agree():
    cov = gi.state_config1()
    pat = np.array([1, 0, 1, 1, 0, -1, 1, 0], np.int8)
    assert oracle.formP_mean(cov, np.zeros(16), pat).p == oracle.formP(cov, pat).p
    mu = np.random.default_rng(3).normal(0, 0.5, 16)
    o = oracle.formP_mean(cov, mu, pat)
    s = oracle.prob_sequential(cov, pat, mean=mu, dps=40)
    assert abs((o.p + o.p_lo) - float(s)) <= 1e-14 * abs(float(s))
