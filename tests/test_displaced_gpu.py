"""Displaced Gaussian states on the GPU (tor_probability_displaced): every
vacuum probability carries the overlap factor of its mean, and the no-click
conditioning moves the mean with the covariance (Sec. II with non-zero means).

* zero mean: bitwise the zero-mean path (the mean row stays zero, every
  overlap factor is exactly one);
* random displaced states, marginal and full patterns, against the binary128
  oracle (form P with mean factors);
* coherent states through an interferometer (a product of coherent states,
  closed form) up to n = 28 clicks on 800 modes: the HBM expansion and the
  10-mode top kernels with the mean row;
* a displaced product state factorises over its modes;
* a displaced two-mode squeezed vacuum against its Fock-expansion closed form;
* host validation of the mean.
"""
import ctypes

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


def _p(r):
    return r.p + r.p_lo


def _haar_state(m, seed, r=0.6):
    rng = np.random.default_rng(seed)
    U = gi.haar_unitary(m, rng)
    return gi.gbs_covariance(U, np.full(m, r)), rng


def _coherent_closed_form(beta, pat):
    import mpmath as mp
    mp.mp.dps = 50
    want = mp.mpf(1)
    for i, v in enumerate(pat):
        a2 = mp.mpf(float(beta[i].real)) ** 2 + mp.mpf(float(beta[i].imag)) ** 2
        if v == 1:
            want *= 1 - mp.exp(-a2)
        elif v == 0:
            want *= mp.exp(-a2)
    return want


def _rel_mp(r, want):
    import mpmath as mp
    return abs(float((mp.mpf(r.p) + mp.mpf(r.p_lo) - want) / want))


@pytest.mark.parametrize("prec", ["f64", "dd"])
def test_zero_mean_is_the_zero_mean_path(ctx, prec):
    cov, rng = _haar_state(14, 81)
    for pat in (gi.marginal_pattern(14, [0, 2, 3, 5, 8, 9, 11, 13]),
                gi.full_pattern(14, [1, 4, 6, 7, 10, 12])):
        a = ctx.probability(cov, pat, prec=prec)
        b = ctx.probability_displaced(cov, np.zeros(28), pat, prec=prec)
        assert (a.p, a.p_lo, a.T, a.T_lo, a.abs_sum) == (b.p, b.p_lo, b.T, b.T_lo, b.abs_sum)
        assert a.rel_err_bound == b.rel_err_bound
        assert a.n_clicks == b.n_clicks and a.prec_used == b.prec_used


@pytest.mark.parametrize("seed", [90, 91, 92])
def test_random_displaced_against_oracle(ctx, seed):
    m = 10
    cov, rng = _haar_state(m, seed, r=0.5)
    cov = gi.apply_loss(cov, 0.8)
    mean = gi.random_mean(m, rng, scale=0.6)
    pats = [np.full(m, -1, np.int8),
            gi.marginal_pattern(m, [3]),
            gi.marginal_pattern(m, [0, 1, 4, 6, 9]),
            gi.full_pattern(m, [2, 5, 7]),
            gi.full_pattern(m, list(range(m))),
            gi.full_pattern(m, []),
            np.array([1, 0, -1, 1, 1, 0, -1, 1, 0, 1], np.int8)]
    for pat in pats:
        o = oracle.formP_mean(cov, mean, pat)
        want = o.p + o.p_lo
        for prec in ("auto", "dd"):
            r = ctx.probability_displaced(cov, mean, pat, prec=prec, tol=1e-12)
            assert abs(_p(r) - want) <= 1e-12 * abs(want) + 1e-300, (prec, pat.tolist(), _p(r), want)
            assert r.n_clicks == int(np.sum(pat == 1))
            # T is the conditioned sum: p = P_vac(N) T
            assert abs(np.exp(r.log_pvac_n) * (r.T + r.T_lo) - want) <= 1e-12 * abs(want)
        # binary64 terms: the reported bound covers the actual error
        r = ctx.probability_displaced(cov, mean, pat, prec="f64")
        assert abs(_p(r) - want) <= max(r.rel_err_bound, 1e-15) * abs(want), (pat.tolist(), r.rel_err_bound)


@pytest.mark.parametrize("n", [14, 16])
def test_mixing_displaced_larger_trees_against_oracle(ctx, n):
    """n >= 14 clicks: the HBM expansion levels above the 10-mode top kernel."""
    m = 20
    cov, rng = _haar_state(m, 95 + n, r=0.45)
    mean = gi.random_mean(m, rng, scale=0.4)
    clicks = sorted(rng.choice(m, n, replace=False).tolist())
    pat = gi.marginal_pattern(m, clicks)
    if n == 16:
        pat = pat.copy()
        pat[[i for i in range(m) if i not in clicks][:2]] = 0
    o = oracle.formP_mean(cov, mean, pat)
    want = o.p + o.p_lo
    r = ctx.probability_displaced(cov, mean, pat, prec="dd")
    assert abs(_p(r) - want) <= 1e-10 * abs(want), (_p(r), want)
    assert r.rel_err_bound <= 1e-10


@pytest.mark.parametrize("m,n,full", [(40, 20, False), (40, 20, True), (800, 28, False)])
def test_coherent_states_closed_form(ctx, m, n, full):
    """Coherent states through an interferometer stay coherent (beta = U alpha):
    p = prod_clicks (1 - e^{-|beta|^2}) prod_no_clicks e^{-|beta|^2}."""
    rng = np.random.default_rng(100 + n + m)
    clicks = sorted(rng.choice(m, n, replace=False).tolist())
    # amplitudes with |beta|^2 in [0.7, 3] on the clicked modes keep the
    # alternating sum's cancellation moderate; small ones elsewhere
    beta = 0.3 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    ph = np.exp(2j * np.pi * rng.random(n))
    beta[clicks] = np.sqrt(rng.uniform(0.7, 3.0, n)) * ph
    if m <= 40:
        U = gi.haar_unitary(m, rng)
        cov = gi.gbs_covariance(U, np.zeros(m))
    else:
        cov = 0.5 * np.eye(2 * m)
    pat = gi.full_pattern(m, clicks) if full else gi.marginal_pattern(m, clicks)
    want = _coherent_closed_form(beta, pat)
    r = ctx.probability_displaced(cov, gi.coherent_mean(beta), pat, prec="dd")
    assert _rel_mp(r, want) <= 1e-10, (_rel_mp(r, want), r.rel_err_bound)
    assert r.rel_err_bound <= 1e-10


def test_product_state_factorises(ctx):
    rng = np.random.default_rng(120)
    m = 12
    cov, blocks = gi.random_product_state(m, rng)
    mean = gi.random_mean(m, rng, scale=0.8)
    pat = np.array([1, 1, 0, 1, -1, 1, 1, 0, 1, 1, -1, 1], np.int8)
    whole = ctx.probability_displaced(cov, mean, pat, prec="dd")
    prod = 1.0
    for i in range(m):
        if pat[i] < 0:
            continue
        ri = ctx.probability_displaced(blocks[i], mean[2 * i:2 * i + 2], pat[i:i + 1], prec="dd")
        prod *= _p(ri)
    assert abs(_p(whole) - prod) <= 1e-13 * prod


def test_displaced_tmsv_closed_forms(ctx):
    """P_vac(a, b) = sech^2 r exp(-|a|^2 - |b|^2 + 2 tanh r Re(a b)) and
    P_vac(a) = exp(-|a|^2 / cosh^2 r) / cosh^2 r (Fock expansion of the
    displaced two-mode squeezed vacuum); click patterns by inclusion-exclusion."""
    r0 = 0.7
    a, b = 0.5 - 0.3j, -0.2 + 0.6j
    cov = gi.tmsv_covariance(r0)
    mean = gi.coherent_mean([a, b])
    c2 = np.cosh(r0) ** 2
    pa = np.exp(-abs(a) ** 2 / c2) / c2
    pb = np.exp(-abs(b) ** 2 / c2) / c2
    pab = np.exp(-abs(a) ** 2 - abs(b) ** 2 + 2 * np.tanh(r0) * (a * b).real) / c2
    want = {(0, 0): pab, (1, 0): pb - pab, (0, 1): pa - pab, (1, 1): 1 - pa - pb + pab,
            (1, -1): 1 - pa, (-1, 0): pb}
    for pat, w in want.items():
        r = ctx.probability_displaced(cov, mean, np.array(pat, np.int8), prec="dd")
        assert abs(_p(r) - w) <= 1e-14, (pat, _p(r), w)


def test_mean_validation(ctx):
    cov = 0.5 * np.eye(6)
    pat = np.array([1, -1, 0], np.int8)
    mean = np.zeros(6)
    mean[0] = 1.0     # |alpha|^2 = 1/2 on mode 0
    mean[2] = np.nan  # mode 1 is not observed: ignored
    r = ctx.probability_displaced(cov, mean, pat, prec="dd")
    assert abs(_p(r) - (1.0 - np.exp(-0.5))) <= 1e-15
    mean[0] = np.inf
    with pytest.raises(tg.TorError) as ei:
        ctx.probability_displaced(cov, mean, pat)
    assert ei.value.status == tg.TOR_EINVAL
    with pytest.raises(ValueError):
        ctx.probability_displaced(cov, np.zeros(5), pat)
    L = tg.lib()
    res = tg._CResult()
    st = L.tor_probability_displaced(ctx._h, tg._dptr(cov), None, 3, tg._i8ptr(pat), 0, 1e-10, ctypes.byref(res))
    assert st == tg.TOR_EINVAL


def test_displaced_not_positive_definite(ctx):
    cov = 0.5 * np.eye(4)
    cov[2, 2] = -3.0
    with pytest.raises(tg.TorError) as ei:
        ctx.probability_displaced(cov, np.ones(4), np.array([1, 1], np.int8))
    assert ei.value.status == tg.TOR_ENOTPD
    with pytest.raises(tg.TorError) as ei:  # the bad mode conditioned away as a no-click mode
        ctx.probability_displaced(cov, np.ones(4), np.array([1, 0], np.int8))
    assert ei.value.status == tg.TOR_ENOTPD


def test_batch_displaced_matches_single(ctx):
    """tor_batch_displaced: marginal and full patterns of uneven size share
    launches; every result is bitwise the single-query result, failures stay
    per query."""
    rng = np.random.default_rng(130)
    m = 40
    cov, _ = _haar_state(m, 131, r=0.5)
    mean = gi.random_mean(m, rng, 0.5)
    pats = []
    for n in (0, 3, 9, 12, 15):
        clicks = sorted(rng.choice(m, n, replace=False).tolist())
        pats.append(gi.marginal_pattern(m, clicks))
        pats.append(gi.full_pattern(m, clicks))
    bad = np.full(m, -1, np.int8)
    bad[0] = 2  # not a pattern value
    pats.append(bad)
    st = ctx.state(cov)
    res, status = ctx.batch_displaced(st, mean, np.stack(pats), prec="dd")
    assert status == tg.TOR_EINVAL
    for p, r in zip(pats[:-1], res[:-1]):
        s = ctx.probability_displaced(cov, mean, p, prec="dd")
        assert (r.p, r.p_lo, r.T, r.T_lo, r.abs_sum, r.rel_err_bound) == (s.p, s.p_lo, s.T, s.T_lo, s.abs_sum,
                                                                          s.rel_err_bound)
        assert r.status == s.status
    assert res[-1].status == tg.TOR_EINVAL
    # a zero-mean batch and a displaced batch on the same state differ
    z, _ = ctx.batch(st, np.stack(pats[:-1]), prec="dd")
    assert any(a.p != b.p for a, b in zip(z, res[:-1]))
    st.close()


def test_displaced_state_batch_and_server(ctx):
    """A state created with a mean: tor_batch and the continuous-batching
    server give bitwise the tor_probability_displaced results; the async batch
    gives bitwise tor_batch's results for its marginal patterns and EINVAL for
    patterns with no-click modes."""
    rng = np.random.default_rng(140)
    m = 30
    cov, _ = _haar_state(m, 141, r=0.5)
    mean = gi.random_mean(m, rng, 0.5)
    pats = []
    for n in (2, 6, 10, 13):
        clicks = sorted(rng.choice(m, n, replace=False).tolist())
        pats.append(gi.marginal_pattern(m, clicks))
        pats.append(gi.full_pattern(m, clicks))
    st = ctx.state(cov, mean=mean)
    res, status = ctx.batch(st, np.stack(pats), prec="dd")
    assert status >= 0
    singles = [ctx.probability_displaced(cov, mean, p, prec="dd") for p in pats]
    for r, s in zip(res, singles):
        assert (r.p, r.p_lo, r.T, r.abs_sum) == (s.p, s.p_lo, s.T, s.abs_sum)
    srv = tg.Server(ctx, workers=2, prec="dd")
    tickets = [srv.submit(st, p) for p in pats]
    for t, s in zip(tickets, singles):
        r, _lat = srv.wait(t)
        assert (r.p, r.p_lo, r.T) == (s.p, s.p_lo, s.T)
    srv.stop()
    import torch
    d_pat = torch.tensor(np.stack(pats), dtype=torch.int8, device="cuda")
    d_out = ctx.batch_async(st, d_pat, prec="dd")
    torch.cuda.synchronize()
    got = tg.results_from_device(d_out)
    for q, (g, r) in enumerate(zip(got, res)):
        if q % 2:  # full patterns are not taken by the async path
            assert g.status == tg.TOR_EINVAL
        else:
            assert (g.p, g.p_lo, g.T, g.T_lo, g.abs_sum, g.rel_err_bound, g.status) == (
                r.p, r.p_lo, r.T, r.T_lo, r.abs_sum, r.rel_err_bound, r.status)
    # quad-double terms: the per-query conditioning route with the mean row
    import mpmath as mp
    mp.mp.dps = 50
    q, _ = ctx.batch(st, np.stack(pats[:2]), prec="qd")
    for g, s in zip(q, singles[:2]):
        assert g.prec_used == tg.PREC_QD
        assert _rel_mp(g, mp.mpf(s.p) + mp.mpf(s.p_lo)) <= s.rel_err_bound + 1e-28
    st.close()
