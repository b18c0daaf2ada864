"""Quad-double term tier (TOR_PREC_QD): conditioning, factorisation and sums in
quad-double, for alternating sums that cancel beyond double-double.

Exact references come from closed forms whose cancellation ratio R is set by
construction (R = prod (1 + q_k) / (1 - q_k) for a product state):
* product states, marginal and full patterns, up to n = 28 clicks on 800
  modes (R ~ 1e15 - 1e37): double-double must flag its bound, quad-double
  must match the exact product to far below 1e-10;
* lossy two-mode squeezed pairs with the partner of every clicked mode a
  no-click mode (correlated conditioning in quad-double);
* a Haar-random mixing state against the binary128 oracle, and quad-double
  against double-double wherever the latter's bound is small;
* displaced states (mean row, quad-double exp): the oracle's definition route
  with mean factors, double-double within its bound, and weak coherent states
  whose exact product cancels by R ~ 1e40.
"""
import numpy as np
import pytest

import gbs_inputs as gi
import oracle
import paper_1810_00900_amd as tg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tg.Context(0)
    yield c
    c.close()


def _mp_val(r):
    import mpmath as mp
    return mp.mpf(r.p) + mp.mpf(r.p_lo)


def _pvac_block(block):
    """det(block + I/2)^-1/2 in mpmath (60 digits) from the binary64 entries."""
    import mpmath as mp
    mp.mp.dps = 60
    k = block.shape[0]
    M = mp.matrix([[mp.mpf(float(block[a, b])) + (mp.mpf(1) / 2 if a == b else 0) for b in range(k)]
                   for a in range(k)])
    return 1 / mp.sqrt(mp.det(M))


def _product_state(m, rng, r_lo=0.4, r_hi=0.6):
    blocks = [gi.single_mode_covariance(rng.uniform(r_lo, r_hi), rng.uniform(0, np.pi), rng.uniform(0.0, 0.05))
              for _ in range(m)]
    return gi.direct_sum(blocks), blocks


def _product_exact(blocks, pat):
    import mpmath as mp
    mp.mp.dps = 60
    p = mp.mpf(1)
    R = mp.mpf(1)
    for k, v in enumerate(pat):
        if v < 0:
            continue
        q = _pvac_block(blocks[k])
        if v == 1:
            p *= 1 - q
            R *= (1 + q) / (1 - q)
        else:
            p *= q
    return p, R


def _rel(r, want):
    import mpmath as mp
    return abs(float((_mp_val(r) - want) / want))


@pytest.mark.parametrize("m,n,full", [(30, 12, False), (30, 12, True), (40, 20, False), (40, 20, True),
                                      (800, 28, True)])
def test_product_state_beyond_double_double(ctx, m, n, full):
    rng = np.random.default_rng(200 + m + n + full)
    cov, blocks = _product_state(m, rng)
    clicks = sorted(rng.choice(m, n, replace=False).tolist())
    if full and m == 800:
        pat = np.full(m, -1, np.int8)
        pat[clicks] = 1
        others = [i for i in range(m) if pat[i] != 1]
        pat[others[::2]] = 0  # 386 no-click modes
    else:
        pat = gi.full_pattern(m, clicks) if full else gi.marginal_pattern(m, clicks)
    want, R = _product_exact(blocks, pat)
    r = ctx.probability(cov, pat, prec="qd", tol=1e-10)
    assert r.prec_used == tg.PREC_QD
    assert _rel(r, want) <= 1e-10, (_rel(r, want), r.rel_err_bound, float(R))
    assert r.rel_err_bound <= 1e-10
    assert r.cancel_ratio == pytest.approx(float(R), rel=1e-6)
    assert r.status == tg.TOR_OK
    if n >= 20:
        d = ctx.probability(cov, pat, prec="dd", tol=1e-10)
        assert d.rel_err_bound > 1e-10 and d.status == tg.TOR_WARN_PRECISION
        # the dd result is as wrong as its bound allows, never more
        assert _rel(d, want) <= d.rel_err_bound


def test_lossy_tmsv_pairs_conditioned_in_qd(ctx):
    """Pairs (2i, 2i+1) of lossy two-mode squeezed vacua; for 16 pairs one mode
    clicks and its partner is a no-click mode: P = prod (P_vac(b) - P_vac(a, b))."""
    import mpmath as mp
    rng = np.random.default_rng(230)
    npairs = 24
    blocks = []
    for _ in range(npairs):
        blocks.append(gi.apply_loss(gi.tmsv_covariance(rng.uniform(0.3, 0.6)), rng.uniform(0.9, 0.98)))
    cov = np.zeros((4 * npairs, 4 * npairs))
    for i, b in enumerate(blocks):
        cov[4 * i:4 * i + 4, 4 * i:4 * i + 4] = b
    m = 2 * npairs
    pat = np.full(m, -1, np.int8)
    want = mp.mpf(1)
    R = mp.mpf(1)
    for i in range(16):
        a, b = (2 * i, 2 * i + 1) if i % 2 == 0 else (2 * i + 1, 2 * i)
        pat[a], pat[b] = 1, 0
        pb = _pvac_block(blocks[i][2 * (b % 2):2 * (b % 2) + 2, 2 * (b % 2):2 * (b % 2) + 2])
        pab = _pvac_block(blocks[i])
        want *= pb - pab
        R *= (pb + pab) / (pb - pab)
    r = ctx.probability(cov, pat, prec="qd", tol=1e-10)
    assert _rel(r, want) <= 1e-10, (_rel(r, want), r.rel_err_bound, float(R))
    assert r.rel_err_bound <= 1e-10
    d = ctx.probability(cov, pat, prec="dd", tol=1e-10)
    assert _rel(d, want) <= max(d.rel_err_bound, 1e-30)


@pytest.mark.parametrize("seed", [240, 241])
def test_mixing_state_against_oracle_and_dd(ctx, seed):
    m = 14
    rng = np.random.default_rng(seed)
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), np.full(m, 0.5))
    pats = [gi.marginal_pattern(m, [0, 2, 3, 5, 7, 8, 11, 13]),
            gi.full_pattern(m, [1, 4, 6, 9, 10, 12]),
            gi.full_pattern(m, list(range(10))),
            np.array([1, 0, -1, 1, 1, 0, -1, 1, 0, 1, 1, -1, 0, 1], np.int8)]
    for pat in pats:
        o = oracle.prob(cov, pat)
        want = o.p + o.p_lo
        q = ctx.probability(cov, pat, prec="qd")
        d = ctx.probability(cov, pat, prec="dd")
        # binary128 oracle: rounding ~1e-34 R
        tol_o = max(1e-20, 1e-32 * o.cancel_ratio)
        assert abs((q.p + q.p_lo) - want) <= tol_o * abs(want), (pat.tolist(), q.p, want)
        assert abs((q.p + q.p_lo) - (d.p + d.p_lo)) <= max(d.rel_err_bound, 1e-30) * abs(want)
        assert q.n_clicks == d.n_clicks and q.log_pvac_n == pytest.approx(d.log_pvac_n, rel=1e-14)


@pytest.mark.parametrize("n", [1, 5, 8, 9, 14])
def test_subset_sum_qd_matches_dd(ctx, n):
    """tor_subset_sum: every tier boundary (n <= 8 is one wave task; above, HBM
    levels); SPD input with moderate cancellation."""
    rng = np.random.default_rng(250 + n)
    m = 3 * n
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), np.full(m, 0.4))
    idx = [q for k in range(n) for q in (2 * k, 2 * k + 1)]
    sig = cov[np.ix_(idx, idx)] + 0.5 * np.eye(2 * n)
    q = ctx.subset_sum(sig, prec="qd")
    d = ctx.subset_sum(sig, prec="dd")
    assert q.prec_used == tg.PREC_QD
    assert abs((q.T + q.T_lo) - (d.T + d.T_lo)) <= max(d.rel_err_bound, 1e-31) * abs(d.T)
    assert q.abs_sum == pytest.approx(d.abs_sum, rel=1e-14)


def test_qd_batch_equals_single_and_rejections(ctx):
    """tor_batch with quad-double terms (one query at a time): every result is
    the single query's, failures stay per query."""
    rng = np.random.default_rng(260)
    m = 16
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), np.full(m, 0.5))
    pats = [gi.marginal_pattern(m, [1, 4, 9]), gi.full_pattern(m, [0, 2, 3, 7, 11]), np.full(m, -1, np.int8)]
    bad = np.full(m, -1, np.int8)
    bad[3] = 5
    st = ctx.state(cov)
    res, status = ctx.batch(st, np.stack(pats + [bad]), prec="qd")
    assert status == tg.TOR_EINVAL
    for p, r in zip(pats, res):
        q = ctx.probability(cov, p, prec="qd")
        assert (r.p, r.p_lo, r.T, r.abs_sum, r.prec_used) == (q.p, q.p_lo, q.T, q.abs_sum, tg.PREC_QD)
    assert res[-1].status == tg.TOR_EINVAL
    st.close()


@pytest.mark.parametrize("seed", [270, 271])
def test_displaced_qd_against_oracle_and_dd(ctx, seed):
    """Displaced states with quad-double terms (mean row in every matrix, the
    overlap factors by the quad-double exp, conditioning in qd, 7-mode tasks):
    against the binary128 definition route with mean factors, and against
    double-double terms within the latter's bound; batches on a displaced
    state equal the single queries."""
    import mpmath as mp
    mp.mp.dps = 60
    rng = np.random.default_rng(seed)
    m = 18
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.8, m))
    mean = gi.random_mean(m, rng, 0.4)
    pats = []
    for n in (0, 3, 7, 10):
        c = gi.random_click_set(m, n, rng)
        pats.append(gi.full_pattern(m, c))
        pats.append(gi.marginal_pattern(m, c))
    for pat in pats:
        q = ctx.probability_displaced(cov, mean, pat, prec="qd")
        d = ctx.probability_displaced(cov, mean, pat, prec="dd")
        o = oracle.formP_mean(cov, mean, pat)
        want = mp.mpf(o.p) + mp.mpf(o.p_lo)
        assert q.prec_used == tg.PREC_QD and q.status == tg.TOR_OK
        assert abs(_mp_val(q) - want) <= abs(want) * max(1e-28, 1e-33 * o.cancel_ratio)
        assert abs(_mp_val(d) - _mp_val(q)) <= abs(_mp_val(q)) * (d.rel_err_bound + 1e-28)
        assert q.rel_err_bound <= 1e-40 * max(1.0, q.cancel_ratio)
    st = ctx.state(cov, mean=mean)
    res, _ = ctx.batch(st, np.stack(pats), prec="qd")
    for pat, r in zip(pats, res):
        s = ctx.probability_displaced(cov, mean, pat, prec="qd")
        assert (r.p, r.p_lo, r.T, r.abs_sum) == (s.p, s.p_lo, s.T, s.abs_sum)
    st.close()


def test_displaced_qd_coherent_beyond_double_double(ctx):
    """Weak coherent states (|beta|^2 = 1e-3 on 12 clicked modes of 30, the rest
    observed without a click): the click factors 1 - e^{-|beta|^2} make the
    alternating sum cancel by R ~ (2 / |beta|^2)^12 ~ 1e40.  Double-double
    flags its bound; quad-double matches the exact product."""
    import mpmath as mp
    mp.mp.dps = 80
    rng = np.random.default_rng(272)
    m, n = 30, 12
    clicks = sorted(rng.choice(m, n, replace=False).tolist())
    beta = 0.2 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    beta[clicks] = np.sqrt(1e-3) * np.exp(2j * np.pi * rng.random(n))
    cov = 0.5 * np.eye(2 * m)
    mean = gi.coherent_mean(beta)
    pat = gi.full_pattern(m, clicks)
    want = mp.mpf(1)
    for i in range(m):
        # |beta|^2 = |mu|^2 / 2 (hbar = 1), from the binary64 mean actually passed
        a2 = (mp.mpf(float(mean[2 * i])) ** 2 + mp.mpf(float(mean[2 * i + 1])) ** 2) / 2
        want *= (1 - mp.exp(-a2)) if pat[i] == 1 else mp.exp(-a2)
    q = ctx.probability_displaced(cov, mean, pat, prec="qd")
    d = ctx.probability_displaced(cov, mean, pat, prec="dd")
    assert q.cancel_ratio > 1e35
    assert d.status == tg.TOR_WARN_PRECISION and d.rel_err_bound > 1e-6
    err = abs(_mp_val(q) - want) / want
    assert err <= q.rel_err_bound and err <= 1e-15, (float(err), q.rel_err_bound)


def test_qd_errors(ctx):
    # a tree whose quad-double pool exceeds the context's memory budget
    sig = np.eye(64)
    with pytest.raises(tg.TorError) as ei:
        ctx.subset_sum(sig, prec="qd")
    assert ei.value.status == tg.TOR_ENOMEM
    assert "quad-double" in tg.last_error()
    # not positive definite: sigma_Q has a negative eigenvalue
    cov = 0.5 * np.eye(4)
    cov[0, 0] = -2.0
    with pytest.raises(tg.TorError) as ei:
        ctx.probability(cov, np.array([1, 1], np.int8), prec="qd")
    assert ei.value.status == tg.TOR_ENOTPD
