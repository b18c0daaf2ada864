"""Per-state inverse (tor_state_invert) and the complementary-minor route for
full patterns: with K = sigma_Q^-1 and G = K[C], p(C, N) = (-1)^n
det(sigma_Q)^-1/2 T(G) (Jacobi's identity det sigma_Q[S] = det sigma_Q
det K[S^c] applied to every vacuum probability of Eq. (prob)).

* the all-no-click pattern is det(sigma_Q)^-1/2: against the binary128 oracle
  and the closed form prod_k sech(r_k) of squeezed vacua (the interferometer
  keeps the vacuum overlap);
* full patterns against the oracle's definition route (form P) and its
  conditioned route (form S), and against the per-query conditioning of the
  library itself, in double-double and quad-double;
* the 800-mode full pattern of the bench workload: quad-double inverse against
  quad-double per-query conditioning;
* batches mixing full, partial and marginal patterns, the server, and errors.
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


def _mp(r):
    import mpmath as mp
    mp.mp.dps = 80
    return mp.mpf(r.p) + mp.mpf(r.p_lo)


def _rel(a, b):
    import mpmath as mp
    mp.mp.dps = 80
    a, b = mp.mpf(a), mp.mpf(b)
    return float(abs((a - b) / b)) if b != 0 else float(abs(a))


def _orc(o):
    import mpmath as mp
    mp.mp.dps = 80
    return mp.mpf(o.p) + mp.mpf(o.p_lo)


def _state(m, seed, lo=0.3, hi=0.9):
    rng = np.random.default_rng(seed)
    U = gi.haar_unitary(m, rng)
    r = rng.uniform(lo, hi, size=m)
    return gi.gbs_covariance(U, r), r, rng


@pytest.mark.parametrize("prec", ["dd", "qd"])
def test_all_no_click_is_det_rsqrt(ctx, prec):
    cov, r, _ = _state(40, 150)
    st = ctx.state(cov).invert(prec)
    pat = np.zeros(40, np.int8)
    res, status = ctx.batch(st, pat[None, :], prec=prec)  # qd: the one-query quad-double path
    got = _mp(res[0])
    want = _orc(oracle.formS(cov, pat))
    assert _rel(got, want) <= 1e-28
    import mpmath as mp
    mp.mp.dps = 50
    closed = mp.mpf(1)
    for x in r:
        closed /= mp.cosh(mp.mpf(float(x)))
    assert _rel(got, closed) <= 1e-12  # the binary64 covariance is exact only to ~1e-16
    assert res[0].n_clicks == 0 and res[0].status == tg.TOR_OK
    st.close()


@pytest.mark.parametrize("prec", ["dd", "f64"])
def test_full_patterns_dd_inverse(ctx, prec):
    m = 20
    cov, _, rng = _state(m, 151)
    plain = ctx.state(cov)
    inv = ctx.state(cov).invert("dd")
    pats = [gi.full_pattern(m, gi.random_click_set(m, n, rng)) for n in (1, 3, 6, 9, 12)]
    pats = np.stack(pats)
    got, _ = ctx.batch(inv, pats, prec=prec)
    cond, _ = ctx.batch(plain, pats, prec=prec)
    for pat, g, c in zip(pats, got, cond):
        n = int(pat.sum())
        o = oracle.formP(cov, pat) if n <= 6 else oracle.formS(cov, pat)
        err = _rel(_mp(g), _orc(o))
        assert err <= g.rel_err_bound + 1e-28
        if prec == "dd":
            assert err <= 1e-10
        # the other route of the library: same quantity, same cancellation
        assert g.n_clicks == c.n_clicks == n
        both = g.rel_err_bound + c.rel_err_bound
        assert _rel(g.cancel_ratio, c.cancel_ratio) <= both + 1e-10
        assert _rel(_mp(g), _mp(c)) <= both + 1e-28
        assert _rel(g.T, c.T) <= both + 1e-14  # T of Sigma_C from the sum of G
        assert _rel(g.tor, c.tor) <= both + 1e-9
        assert abs(g.log_p - c.log_p) <= both + 1e-12 * abs(c.log_p)
    plain.close()
    inv.close()


def test_full_patterns_qd_inverse(ctx):
    m = 24
    cov, _, rng = _state(m, 152)
    inv = ctx.state(cov).invert("qd")
    plain = ctx.state(cov)
    pats = np.stack([gi.full_pattern(m, gi.random_click_set(m, n, rng)) for n in (2, 5, 10, 14)])
    got, _ = ctx.batch(inv, pats, prec="qd")
    cond, _ = ctx.batch(plain, pats, prec="qd")
    dd_on_qd, _ = ctx.batch(inv, pats, prec="dd")  # double-double terms from the rounded qd inverse
    for pat, g, c, d in zip(pats, got, cond, dd_on_qd):
        assert g.prec_used == tg.PREC_QD
        o = oracle.formS(cov, pat)
        assert _rel(_mp(g), _orc(o)) <= 1e-25
        # results are reported as double-double (p + p_lo), the factors
        # det(sigma_Q)^-1/2 and det(G)^1/2 formed in double-double
        assert _rel(_mp(g), _mp(c)) <= g.rel_err_bound + c.rel_err_bound + 1e-29
        assert _rel(_mp(d), _mp(g)) <= d.rel_err_bound + 1e-28
    inv.close()
    plain.close()


def test_m800_full_pattern_qd_routes_agree(ctx):
    """An 800-mode full pattern with 20 clicks (all modes observed, 780
    without a click): quad-double inverse against quad-double per-query
    conditioning."""
    cov = gi.state_m800(50)
    m = 800
    rng = np.random.default_rng(153)
    clicks = gi.random_click_set(m, 20, rng)
    pat = gi.full_pattern(m, clicks)
    inv = ctx.state(cov).invert("qd")
    got, _ = ctx.batch(inv, pat[None, :], prec="qd")
    want = ctx.probability(cov, pat, prec="qd")
    g = got[0]
    print("m800 n20 full: p", g.p, "bound", g.rel_err_bound, want.rel_err_bound,
          "routes differ by", _rel(_mp(g), _mp(want)))
    assert g.status in (tg.TOR_OK, tg.TOR_WARN_PRECISION)
    assert g.cancel_ratio == pytest.approx(want.cancel_ratio, rel=1e-6)
    assert _rel(_mp(g), _mp(want)) <= g.rel_err_bound + want.rel_err_bound + 1e-29  # observed 8.7e-31
    inv.close()


def test_mixed_batch_and_server(ctx):
    m = 30
    cov, _, rng = _state(m, 154)
    inv = ctx.state(cov).invert("dd")
    pats = []
    for n in (2, 5, 8, 11):
        c = gi.random_click_set(m, n, rng)
        pats.append(gi.full_pattern(m, c))          # inverse route
        pats.append(gi.marginal_pattern(m, c))      # gather of sigma_Q[C]
        part = gi.full_pattern(m, c)
        part[np.setdiff1d(np.arange(m), c)[:4]] = -1
        pats.append(part)                          # per-query conditioning
    pats = np.stack(pats)
    a, _ = ctx.batch(inv, pats, prec="dd")
    b, _ = ctx.batch(inv, pats, prec="dd")
    for x, y in zip(a, b):
        assert (x.p, x.p_lo, x.T, x.T_lo, x.abs_sum) == (y.p, y.p_lo, y.T, y.T_lo, y.abs_sum)
    for pat, x in zip(pats, a):
        if (pat == -1).any():  # not a full pattern: the single-query path, bitwise
            s = ctx.probability(cov, pat, prec="dd")
            assert (x.p, x.p_lo, x.T, x.T_lo) == (s.p, s.p_lo, s.T, s.T_lo)
        assert _rel(_mp(x), _orc(oracle.formS(cov, pat))) <= 1e-10
    srv = tg.Server(ctx, workers=2, prec="dd")
    tickets = [srv.submit(inv, p) for p in pats]
    for t, x in zip(tickets, a):
        r, _lat = srv.wait(t)
        assert (r.p, r.p_lo, r.T, r.T_lo) == (x.p, x.p_lo, x.T, x.T_lo)
    srv.stop()
    inv.close()


@pytest.mark.parametrize("inv_prec,prec", [("dd", "dd"), ("dd", "f64"), ("qd", "dd")])
def test_async_full_patterns(ctx, inv_prec, prec):
    """tor_batch_async on an inverted state: full patterns gathered from the
    device copy of the inverse; p bitwise tor_batch's, the sums rescaled to
    Sigma_C within 1e-13; partial patterns still rejected per query."""
    import torch
    m = 40
    cov, _, rng = _state(m, 156)
    st = ctx.state(cov).invert(inv_prec)
    pats = [np.zeros(m, np.int8)]
    for n in (1, 4, 9, 12, 16):
        c = gi.random_click_set(m, n, rng)
        pats.append(gi.full_pattern(m, c))
        pats.append(gi.marginal_pattern(m, c))
    part = gi.full_pattern(m, [3, 7])
    part[10] = -1
    pats.append(part)
    pats = np.stack(pats)
    want, _ = ctx.batch(st, pats, prec=prec)
    d_out = ctx.batch_async(st, torch.from_numpy(pats).to("cuda"), prec=prec)
    torch.cuda.synchronize()
    got = tg.results_from_device(d_out)
    for pat, g, w in zip(pats, got, want):
        if (pat == 0).any() and (pat == -1).any():
            assert g.status == tg.TOR_EINVAL
            continue
        assert (g.p, g.p_lo, g.n_clicks, g.prec_used, g.status) == (w.p, w.p_lo, w.n_clicks, w.prec_used, w.status)
        for f in ("T", "abs_sum", "cancel_ratio", "rel_err_bound", "tor", "log_p", "log_pvac_n"):
            assert getattr(g, f) == pytest.approx(getattr(w, f), rel=1e-13, abs=1e-300), f
    st.close()


@pytest.mark.parametrize("inv_prec,prec", [("dd", "dd"), ("dd", "f64"), ("qd", "dd")])
def test_async_displaced_full_patterns(ctx, inv_prec, prec):
    """tor_batch_async on an inverted displaced state: marginal patterns run
    the displaced trees and full patterns the information-form trees, in one
    call (two tree kinds); p bitwise tor_batch's, the other fields within
    1e-13; partial patterns still rejected per query."""
    import torch
    m = 36
    cov, _, rng = _state(m, 158, 0.3, 0.8)
    mean = gi.random_mean(m, rng, 0.4)
    st = ctx.state(cov, mean=mean).invert(inv_prec)
    pats = [np.zeros(m, np.int8)]
    for n in (1, 5, 10, 14, 20, 24):
        c = gi.random_click_set(m, n, rng)
        pats.append(gi.full_pattern(m, c))
        pats.append(gi.marginal_pattern(m, c))
    part = gi.full_pattern(m, [2, 9])
    part[11] = -1
    pats.append(part)
    pats = np.stack(pats)
    want, _ = ctx.batch(st, pats, prec=prec)
    d_out = ctx.batch_async(st, torch.from_numpy(pats).to("cuda"), prec=prec)
    torch.cuda.synchronize()
    got = tg.results_from_device(d_out)
    for pat, g, w in zip(pats, got, want):
        if (pat == 0).any() and (pat == -1).any():
            assert g.status == tg.TOR_EINVAL
            continue
        assert (g.p, g.p_lo, g.n_clicks, g.prec_used, g.status) == (w.p, w.p_lo, w.n_clicks, w.prec_used, w.status)
        for f in ("T", "abs_sum", "cancel_ratio", "rel_err_bound", "tor", "log_p", "log_pvac_n"):
            assert getattr(g, f) == pytest.approx(getattr(w, f), rel=1e-13, abs=1e-300), (f, int((pat == 1).sum()))
    st.close()


def _coherent(beta, pat):
    import mpmath as mp
    mp.mp.dps = 60
    want = mp.mpf(1)
    for i, v in enumerate(pat):
        a2 = mp.mpf(float(beta[i].real)) ** 2 + mp.mpf(float(beta[i].imag)) ** 2
        want *= (1 - mp.exp(-a2)) if v == 1 else mp.exp(-a2) if v == 0 else 1
    return want


@pytest.mark.parametrize("prec", ["dd", "f64"])
def test_displaced_full_patterns_inverse(ctx, prec):
    """Full patterns of an inverted displaced state: the information-form tree
    over [0, h_C; h_C, G] with h = sigma_Q^-1 mu, against the oracle's
    definition route with mean factors and against the per-query conditioning
    of the displaced state."""
    m = 16
    cov, _, rng = _state(m, 157, 0.3, 0.7)
    mean = gi.random_mean(m, rng, 0.4)
    plain = ctx.state(cov, mean=mean)
    inv = ctx.state(cov, mean=mean).invert("dd")
    pats = np.stack([np.zeros(m, np.int8)] + [gi.full_pattern(m, gi.random_click_set(m, n, rng))
                                              for n in (1, 3, 6, 9)])
    got, _ = ctx.batch(inv, pats, prec=prec)
    cond, _ = ctx.batch(plain, pats, prec=prec)
    for pat, g, c in zip(pats, got, cond):
        o = oracle.formP_mean(cov, mean, pat)
        err = _rel(_mp(g), _orc(o))
        assert err <= g.rel_err_bound + 1e-27, (int(pat.sum()), err, g.rel_err_bound)
        if prec == "dd":
            assert err <= 1e-10
        both = g.rel_err_bound + c.rel_err_bound
        assert _rel(_mp(g), _mp(c)) <= both + 1e-27
        assert _rel(g.T, c.T) <= both + 1e-13  # T of Sigma_C with its conditioned mean
        assert abs(g.log_p - c.log_p) <= both + 1e-12 * abs(c.log_p)
        assert abs(g.log_pvac_n - c.log_pvac_n) <= 1e-11 * max(1.0, abs(c.log_pvac_n))
    # the server and a second batch give the same words
    srv = tg.Server(ctx, workers=2, prec=prec)
    tickets = [srv.submit(inv, p) for p in pats]
    for t, g in zip(tickets, got):
        r, _lat = srv.wait(t)
        assert (r.p, r.p_lo, r.T, r.T_lo) == (g.p, g.p_lo, g.T, g.T_lo)
    srv.stop()
    plain.close()
    inv.close()


def test_displaced_inverse_quad_double(ctx):
    """Quad-double full patterns of a displaced state inverted in quad-double:
    the information-form tree over [0, h_C; h_C, G] with h = K mu in qd,
    against the per-query qd route and the oracle, and weak coherent states
    (R ~ 1e40) against their exact product."""
    import mpmath as mp
    mp.mp.dps = 80
    m = 16
    cov, _, rng = _state(m, 160, 0.3, 0.7)
    mean = gi.random_mean(m, rng, 0.4)
    inv = ctx.state(cov, mean=mean).invert("qd")
    pats = np.stack([np.zeros(m, np.int8)] + [gi.full_pattern(m, gi.random_click_set(m, n, rng)) for n in (2, 6, 9)])
    got, _ = ctx.batch(inv, pats, prec="qd")
    for pat, g in zip(pats, got):
        w = ctx.probability_displaced(cov, mean, pat, prec="qd")
        o = oracle.formP_mean(cov, mean, pat)
        assert g.prec_used == tg.PREC_QD
        assert _rel(_mp(g), _mp(w)) <= 1e-28
        assert _rel(_mp(g), _orc(o)) <= max(1e-28, 1e-33 * o.cancel_ratio)
    inv.close()
    m, n = 30, 12
    rng = np.random.default_rng(161)
    clicks = sorted(rng.choice(m, n, replace=False).tolist())
    beta = 0.2 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    beta[clicks] = np.sqrt(1e-3) * np.exp(2j * np.pi * rng.random(n))
    cov, mean = 0.5 * np.eye(2 * m), gi.coherent_mean(beta)
    st = ctx.state(cov, mean=mean).invert("qd")
    pat = gi.full_pattern(m, clicks)
    r, _ = ctx.batch(st, pat[None, :], prec="qd")
    want = mp.mpf(1)
    for i in range(m):
        a2 = (mp.mpf(float(mean[2 * i])) ** 2 + mp.mpf(float(mean[2 * i + 1])) ** 2) / 2
        want *= (1 - mp.exp(-a2)) if pat[i] == 1 else mp.exp(-a2)
    assert r[0].cancel_ratio > 1e35
    assert _rel(_mp(r[0]), want) <= 1e-15 and _rel(_mp(r[0]), want) <= r[0].rel_err_bound
    st.close()


def test_displaced_inverse_coherent_closed_form(ctx):
    """Coherent states through an interferometer (beta = U alpha) on an
    inverted state, all 40 modes observed: prod_clicks (1 - e^{-|beta|^2})
    prod_no_clicks e^{-|beta|^2}."""
    m, n = 40, 12
    rng = np.random.default_rng(158)
    clicks = sorted(rng.choice(m, n, replace=False).tolist())
    beta = 0.3 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    beta[clicks] = np.sqrt(rng.uniform(0.7, 3.0, n)) * np.exp(2j * np.pi * rng.random(n))
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), np.zeros(m))
    st = ctx.state(cov, mean=gi.coherent_mean(beta)).invert("dd")
    pats = np.stack([gi.full_pattern(m, clicks), gi.full_pattern(m, clicks[:5]), np.zeros(m, np.int8)])
    res, _ = ctx.batch(st, pats, prec="dd")
    for pat, r in zip(pats, res):
        assert _rel(_mp(r), _coherent(beta, pat)) <= 1e-12, (int(pat.sum()), r.rel_err_bound)
        assert r.status == tg.TOR_OK
    st.close()


def _product_state(r):
    d = np.empty(2 * len(r))
    d[0::2] = np.exp(-2 * r) / 2
    d[1::2] = np.exp(2 * r) / 2
    return np.diag(d), d


def _product_closed_form(d, pat):
    import mpmath as mp
    mp.mp.dps = 60
    want = mp.mpf(1)
    half = mp.mpf(1) / 2
    for k, v in enumerate(pat):
        p0 = 1 / mp.sqrt((mp.mpf(d[2 * k]) + half) * (mp.mpf(d[2 * k + 1]) + half))
        want *= (1 - p0) if v == 1 else p0 if v == 0 else 1
    return want


def test_single_mode_and_largest_state(ctx):
    """m = 1, and m = 2048 (the largest inverse; twice the observed modes the
    per-query conditioning takes): squeezed product states, whose full
    patterns factorise into sech r_k and 1 - sech r_k per mode."""
    cov1, d1 = _product_state(np.array([0.5]))
    st = ctx.state(cov1).invert("dd")
    res, _ = ctx.batch(st, np.array([[0], [1]], np.int8), prec="dd")
    for pat, r in zip(([0], [1]), res):
        assert _rel(_mp(r), _product_closed_form(d1, pat)) <= 1e-30
    st.close()
    m = 2048
    rng = np.random.default_rng(159)
    cov, d = _product_state(rng.uniform(0.2, 0.8, m))
    st = ctx.state(cov).invert("dd")
    pats = np.stack([gi.full_pattern(m, gi.random_click_set(m, n, rng)) for n in (0, 5, 12)])
    res, _ = ctx.batch(st, pats, prec="dd")
    for pat, r in zip(pats, res):
        # a product state cancels by prod (1 + sech r)/(1 - sech r): R ~ 1e15 at 12 clicks
        err = _rel(_mp(r), _product_closed_form(d, pat))
        assert err <= r.rel_err_bound + 1e-28 and err <= 1e-20, (int(pat.sum()), err, r.rel_err_bound)
    plain = ctx.state(cov)  # per-query conditioning: more than 1024 observed modes
    with pytest.raises(tg.TorError) as e:
        ctx.batch(plain, pats[1:2], prec="dd")
    assert e.value.status == tg.TOR_ETOOBIG
    plain.close()
    st.close()
    big = ctx.state(0.5 * np.eye(2 * (m + 1)))
    with pytest.raises(tg.TorError) as e:
        big.invert("dd")
    assert e.value.status == tg.TOR_ETOOBIG
    big.close()


def test_invert_errors(ctx):
    m = 6
    cov, _, rng = _state(m, 155)
    mean = gi.random_mean(m, rng, 0.3)
    disp = ctx.state(cov, mean=mean).invert("qd")  # displaced: allowed
    # quad-double full patterns of a state inverted in qd take the
    # information-form route: the per-query route's value to the output words
    fp = gi.full_pattern(m, [1])
    r, _ = ctx.batch(disp, fp[None, :], prec="qd")
    w = ctx.probability_displaced(cov, mean, fp, prec="qd")
    assert r[0].prec_used == tg.PREC_QD and _rel(_mp(r[0]), _mp(w)) <= 1e-29
    disp.close()
    bad = ctx.state(-np.eye(2 * m))  # sigma_Q = -I/2: not positive definite
    with pytest.raises(tg.TorError) as e:
        bad.invert("dd")
    assert e.value.status == tg.TOR_ENOTPD
    # a failed inversion leaves the state usable by the per-query route
    with pytest.raises(tg.TorError) as e:
        ctx.batch(bad, gi.marginal_pattern(m, [1])[None, :], prec="dd")
    assert e.value.status == tg.TOR_ENOTPD
    bad.close()
    st = ctx.state(cov)
    import ctypes
    assert tg.lib().tor_state_invert(st.handle, ctypes.c_int(9)) == tg.TOR_EINVAL
    st.invert("dd").invert("qd")  # re-inversion replaces the inverse
    res, _ = ctx.batch(st, gi.full_pattern(m, [0, 3])[None, :], prec="qd")
    assert _rel(_mp(res[0]), _orc(oracle.formP(cov, gi.full_pattern(m, [0, 3])))) <= 1e-28
    st.close()
