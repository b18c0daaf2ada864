"""The reported Torontonian and log p against the oracle, on every path.

tor_result.tor is Tor(O) with O = I - Sigma_C^-1 (the quantity of the
Torontonian form of the click probability, p = P_vac(N) det(Sigma_C)^-1/2
Tor(O)), and log_p is log p.  The oracle computes Tor(O) by its own route: the
signed sum over Z of det(I - O_Z)^-1/2 in mpmath (``oracle.torontonian_mp``),
with Sigma_C from the oracle's binary128 Schur complement; for larger n the
binary128 subset sum of form S times det(Sigma_C)^1/2 (Jacobi's identity,
pinned on the CPU by the agreement of forms S and T).

Paths: single queries (marginal, mixed and full patterns), tor_batch on plain
and inverted states (the complementary-minor route with its sign (-1)^n),
the server, tor_batch_async (marginal and inverted full patterns), and
displaced states.  A second group checks that rel_err_bound covers the error
of the no-click conditioning and of the per-state inverse: double-double and
binary64 results of 800-mode full patterns against quad-double.
"""
import mpmath as mp
import numpy as np
import pytest

import gbs_inputs as gi
import oracle
import paper_1810_00900_amd as tg

pytestmark = pytest.mark.gpu

DPS = 60


@pytest.fixture(scope="module")
def ctx():
    c = tg.Context(0)
    yield c
    c.close()


def _mpv(hi, lo=0.0):
    mp.mp.dps = DPS
    return mp.mpf(hi) + mp.mpf(lo)


def _rel(a, b):
    mp.mp.dps = DPS
    a, b = mp.mpf(a), mp.mpf(b)
    return float(abs((a - b) / b)) if b != 0 else float(abs(a))


def _sigma_c(cov, pattern):
    """Sigma_C of the oracle (binary128 Schur complement on N) as an mpmath matrix."""
    hi, lo, _ = oracle.conditioned(cov, pattern)
    mp.mp.dps = DPS
    d = hi.shape[0]
    S = mp.matrix(d, d)
    for a in range(d):
        for b in range(d):
            S[a, b] = mp.mpf(float(hi[a, b])) + mp.mpf(float(lo[a, b]))
    return S


def _oracle_tor_mp(cov, pattern):
    """Tor(I - Sigma_C^-1) by the oracle's Torontonian route (small n)."""
    n = int(np.sum(np.asarray(pattern) == 1))
    if n == 0:
        return mp.mpf(1)
    S = _sigma_c(cov, pattern)
    O = mp.eye(2 * n) - S ** -1
    return oracle.torontonian_mp(O, DPS)


def _oracle_tor_formS(cov, pattern):
    """Tor(I - Sigma_C^-1) = det(Sigma_C)^1/2 T(Sigma_C) with T from the binary128
    form S sum (larger n)."""
    o = oracle.formS(cov, pattern)
    S = _sigma_c(cov, pattern)
    return mp.sqrt(mp.det(S)) * _mpv(o.T, o.T_lo)


def _oracle_p(cov, pattern):
    o = oracle.prob(cov, pattern)
    return _mpv(o.p, o.p_lo)


def _check(r, tor_want, p_want, tol_tor=1e-12, tol_logp=1e-13):
    assert r.status >= 0
    assert _rel(r.tor, tor_want) <= tol_tor + r.rel_err_bound, (r.tor, tor_want)
    mp.mp.dps = DPS
    lw = mp.log(p_want)
    assert abs(r.log_p - float(lw)) <= tol_logp * max(1.0, abs(float(lw))) + r.rel_err_bound, (r.log_p, lw)


def _state(m, seed, lo=0.3, hi=0.9):
    rng = np.random.default_rng(seed)
    U = gi.haar_unitary(m, rng)
    r = rng.uniform(lo, hi, size=m)
    return gi.gbs_covariance(U, r), rng


# ------------------------------------------------------------------ single queries

def test_config1_all_click(ctx):
    cov = gi.state_config1()
    pat = np.ones(8, np.int8)
    r = ctx.probability(cov, pat, prec="dd", tol=1e-10)
    tor_o = _oracle_tor_mp(cov, pat)
    p_o = oracle.prob_torontonian_mp(cov, pat, DPS)
    _check(r, tor_o, p_o)
    assert _rel(_mpv(r.p, r.p_lo), p_o) <= 1e-10
    # marginal pattern: P_vac(N) = 1, so p = det(Sigma_C)^-1/2 Tor
    assert r.log_pvac_n == 0.0


@pytest.mark.parametrize("prec", ["dd", "f64"])
def test_mixed_small_patterns(ctx, prec):
    rng = np.random.default_rng(901)
    for m in (3, 6, 9):
        cov, _ = _state(m, 900 + m, 0.4, 1.0)
        for _ in range(6):
            pat = rng.integers(-1, 2, size=m).astype(np.int8)
            r = ctx.probability(cov, pat, prec=prec, tol=1e-10)
            p_o = oracle.prob_torontonian_mp(cov, pat, DPS)
            if p_o == 0:
                continue
            tol = 1e-12 if prec == "dd" else 1e-9
            _check(r, _oracle_tor_mp(cov, pat), p_o, tol_tor=tol, tol_logp=tol)


def test_m800_marginal_n12(ctx):
    cov = gi.state_m800(50)
    pat = gi.config5_pattern(12)
    r = ctx.probability(cov, pat, prec="dd", tol=1e-10)
    _check(r, _oracle_tor_formS(cov, pat), _oracle_p(cov, pat), tol_tor=1e-10, tol_logp=1e-12)
    assert r.status == tg.TOR_OK


def test_displaced_tor_definition(ctx):
    # displaced states: tor = det(Sigma_C)^1/2 T with T = p / P_vac(N) of the
    # conditioned mean; both from the oracle's definition route with mean factors
    cov, rng = _state(7, 905)
    mean = gi.random_mean(7, rng, 0.4)
    for pat in ([1, 1, 0, -1, 1, 0, 1], [1, -1, 1, 1, -1, 1, -1]):
        pat = np.array(pat, np.int8)
        r = ctx.probability_displaced(cov, mean, pat, prec="dd", tol=1e-10)
        o = oracle.formP_mean(cov, mean, pat)
        p_o = _mpv(o.p, o.p_lo)
        T_o = p_o / mp.mpf(o.pvac_n)
        tor_o = mp.sqrt(mp.det(_sigma_c(cov, pat))) * T_o
        _check(r, tor_o, p_o, tol_tor=1e-12, tol_logp=1e-13)


# ------------------------------------------------------------------ batches, inverted states, server, async

@pytest.fixture(scope="module")
def small_state(ctx):
    cov, rng = _state(10, 910)
    plain = ctx.state(cov)
    inv_dd = ctx.state(cov).invert("dd")
    inv_qd = ctx.state(cov).invert("qd")
    pats = [gi.full_pattern(10, gi.random_click_set(10, n, rng)) for n in (1, 2, 3, 4, 5, 6)]
    pats += [gi.marginal_pattern(10, gi.random_click_set(10, n, rng)) for n in (2, 5)]
    pats = np.stack(pats)
    want = [(_oracle_tor_mp(cov, p), oracle.prob_torontonian_mp(cov, p, DPS)) for p in pats]
    yield cov, plain, inv_dd, inv_qd, pats, want
    for s in (plain, inv_dd, inv_qd):
        s.close()


@pytest.mark.parametrize("which", ["plain", "inv_dd", "inv_qd"])
def test_batch_full_patterns(ctx, small_state, which):
    cov, plain, inv_dd, inv_qd, pats, want = small_state
    st = {"plain": plain, "inv_dd": inv_dd, "inv_qd": inv_qd}[which]
    res, _ = ctx.batch(st, pats, prec="dd")
    for r, p, (tor_o, p_o) in zip(res, pats, want):
        assert r.n_clicks == int(np.sum(p == 1))
        _check(r, tor_o, p_o)
        assert _rel(_mpv(r.p, r.p_lo), p_o) <= 1e-12


def test_qd_full_patterns_on_qd_inverse(ctx, small_state):
    cov, plain, inv_dd, inv_qd, pats, want = small_state
    res, _ = ctx.batch(inv_qd, pats, prec="qd")
    for r, (tor_o, p_o) in zip(res, want):
        assert r.prec_used == tg.PREC_QD
        _check(r, tor_o, p_o)


def test_server_results(ctx, small_state):
    cov, plain, inv_dd, inv_qd, pats, want = small_state
    with tg.Server(ctx, workers=2, prec="dd", tol=1e-10, max_batch=16) as srv:
        tickets = [(srv.submit(st, p), k) for st in (plain, inv_dd) for k, p in enumerate(pats)]
        for t, k in tickets:
            r, _ = srv.wait(t)
            _check(r, want[k][0], want[k][1])


def test_async_inverted_full_patterns(ctx, small_state):
    import torch
    cov, plain, inv_dd, inv_qd, pats, want = small_state
    d_out = ctx.batch_async(inv_dd, torch.from_numpy(pats).to("cuda"), prec="dd")
    torch.cuda.synchronize()
    res = tg.results_from_device(d_out)
    for r, (tor_o, p_o) in zip(res, want):
        # the device rescales the sums with a binary64 det(G)^1/2
        _check(r, tor_o, p_o, tol_tor=1e-12, tol_logp=1e-13)


def test_m800_marginals_batch_server_async(ctx):
    import torch
    cov = gi.state_m800(30)
    st = ctx.state(cov)
    rng = np.random.default_rng(913)
    pats = np.stack([gi.marginal_pattern(800, gi.random_click_set(800, n, rng)) for n in (0, 3, 6, 8, 11)])
    want = []
    for p in pats:
        n = int(np.sum(p == 1))
        tor_o = _oracle_tor_mp(cov, p) if n <= 8 else _oracle_tor_formS(cov, p)
        want.append((tor_o, _oracle_p(cov, p)))
    res_b, _ = ctx.batch(st, pats, prec="dd")
    with tg.Server(ctx, workers=2, prec="dd", tol=1e-10) as srv:
        res_s = [srv.wait(srv.submit(st, p))[0] for p in pats]
    d_out = ctx.batch_async(st, torch.from_numpy(pats).to("cuda"), prec="dd")
    torch.cuda.synchronize()
    res_a = tg.results_from_device(d_out)
    for res in (res_b, res_s, res_a):
        for r, (tor_o, p_o) in zip(res, want):
            _check(r, tor_o, p_o, tol_tor=1e-11, tol_logp=1e-12)
    st.close()


# ------------------------------------------------------------------ the bound covers conditioning

def _qd_ref(ctx, cov, pat):
    r = ctx.probability(cov, pat, prec="qd", tol=1e-30)
    assert r.prec_used == tg.PREC_QD
    return r


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_bound_covers_conditioning_m800(ctx, n):
    """Full 800-mode patterns (800 - n no-click modes conditioned in double-double)
    against the quad-double route: the observed error of the double-double and
    binary64 results stays within their rel_err_bound."""
    cov = gi.state_m800(30)
    rng = np.random.default_rng(920 + n)
    pat = gi.full_pattern(800, gi.random_click_set(800, n, rng))
    ref = _qd_ref(ctx, cov, pat)
    want = _mpv(ref.p, ref.p_lo)
    assert ref.rel_err_bound <= 1e-20
    for prec in ("dd", "f64"):
        r = ctx.probability(cov, pat, prec=prec, tol=1e-10)
        err = _rel(_mpv(r.p, r.p_lo), want)
        assert err <= r.rel_err_bound, (prec, err, r.rel_err_bound, r.cancel_ratio)
        # the conditioning term: at least 16 k u_dd R on top of the tree's 16 n u R
        k = 800 - n
        assert r.rel_err_bound >= 16 * k * 2.0 ** -104 * r.cancel_ratio * (1 - 1e-12)


def test_bound_covers_inverse_m800(ctx):
    """The same full patterns from a state inverted in double-double: the bound
    carries the 800 sweeps of the inverse."""
    cov = gi.state_m800(30)
    st = ctx.state(cov).invert("dd")
    rng = np.random.default_rng(930)
    pats = np.stack([gi.full_pattern(800, gi.random_click_set(800, n, rng)) for n in (5, 7, 9)])
    res, _ = ctx.batch(st, pats, prec="dd")
    for p, r in zip(pats, res):
        ref = _qd_ref(ctx, cov, p)
        err = _rel(_mpv(r.p, r.p_lo), _mpv(ref.p, ref.p_lo))
        assert err <= r.rel_err_bound, (err, r.rel_err_bound)
        assert r.rel_err_bound >= 16 * 800 * 2.0 ** -104 * r.cancel_ratio * (1 - 1e-12)
    st.close()


def test_marginal_bound_unchanged(ctx):
    """Marginal patterns have no elimination steps: the bound is the tree's alone."""
    cov = gi.state_m800(50)
    pat = gi.config5_pattern(12)
    r = ctx.probability(cov, pat, prec="dd", tol=1e-10)
    want = 16 * 12 * 2.0 ** -104 * (r.abs_sum / abs(r.T))
    assert r.rel_err_bound == pytest.approx(want, rel=1e-12)
