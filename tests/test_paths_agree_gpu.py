"""Every evaluation path on the same seeded queries: single calls
(tor_probability), fused batches (tor_batch), the continuous-batching server,
stream-ordered batches (tor_batch_async) and the inverted-state route for full
patterns, on random states and random marginal, full and partial patterns.

Paths that build the same trees must agree bitwise (single = batch = server;
async = batch for p); the inverted-state route agrees within the error bounds;
every double-double result is checked against the binary128 oracle at 1e-10
and at its own bound.
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


def _mp(x, lo=0.0):
    import mpmath as mp
    mp.mp.dps = 60
    return mp.mpf(x) + mp.mpf(lo)


def _rel(a, b):
    return float(abs((a - b) / b)) if b != 0 else float(abs(a))


def _patterns(m, rng, count):
    pats = []
    for _ in range(count):
        kind = rng.integers(0, 3)
        n = int(rng.integers(0, min(m, 12) + 1))
        c = gi.random_click_set(m, n, rng)
        if kind == 0:
            p = gi.marginal_pattern(m, c)
        elif kind == 1:
            p = gi.full_pattern(m, c)
        else:
            p = gi.full_pattern(m, c)
            rest = np.setdiff1d(np.arange(m), c)
            if len(rest):
                p[rng.choice(rest, size=int(rng.integers(1, len(rest) + 1)), replace=False)] = -1
        pats.append(p)
    return np.stack(pats)


@pytest.mark.parametrize("m,seed", [(8, 170), (30, 171), (100, 172)])
def test_paths_agree(ctx, m, seed):
    import torch
    rng = np.random.default_rng(seed)
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.2, 0.9, m))
    pats = _patterns(m, rng, 20)
    st = ctx.state(cov)
    inv = ctx.state(cov).invert("dd")
    batch, _ = ctx.batch(st, pats, prec="dd")
    on_inv, _ = ctx.batch(inv, pats, prec="dd")
    srv = tg.Server(ctx, workers=2, prec="dd")
    tickets = [srv.submit(st, p) for p in pats]
    served = [srv.wait(t)[0] for t in tickets]
    srv.stop()
    d_out = ctx.batch_async(st, torch.from_numpy(pats).to("cuda"), prec="dd")
    torch.cuda.synchronize()
    asyn = tg.results_from_device(d_out)
    for pat, b, j, s, a in zip(pats, batch, on_inv, served, asyn):
        single = ctx.probability(cov, pat, prec="dd")
        key = lambda r: (r.p, r.p_lo, r.T, r.T_lo, r.abs_sum, r.status)
        assert key(single) == key(b) == key(s)
        full = (pat >= 0).all() and (pat == 0).any()
        if not (pat == 0).any():  # marginal: the async path builds the same trees
            assert (a.p, a.p_lo, a.T, a.T_lo) == (b.p, b.p_lo, b.T, b.T_lo)
        elif not full:
            assert a.status == tg.TOR_EINVAL
        if full:  # inverted state: complementary-minor route
            assert _rel(_mp(j.p, j.p_lo), _mp(b.p, b.p_lo)) <= j.rel_err_bound + b.rel_err_bound + 1e-28
        else:
            assert key(j) == key(b)
        o = oracle.prob(cov, pat)
        err = _rel(_mp(b.p, b.p_lo), _mp(o.p, o.p_lo))
        assert err <= 1e-10 and err <= b.rel_err_bound + 1e-28, (pat, err, b.rel_err_bound)
    st.close()
    inv.close()


@pytest.mark.parametrize("m,seed", [(10, 173), (40, 174)])
def test_displaced_paths_agree(ctx, m, seed):
    """The same for a displaced state: tor_probability_displaced, tor_batch on
    the state, the server and the async batch (marginal patterns) agree
    bitwise; the inverted state (information-form trees, dd and qd, also
    through the async batch) within the bounds; every result against the oracle's definition route with means."""
    import torch
    rng = np.random.default_rng(seed)
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.2, 0.8, m))
    mean = gi.random_mean(m, rng, 0.4)
    pats = _patterns(m, rng, 16)
    st = ctx.state(cov, mean=mean)
    inv = ctx.state(cov, mean=mean).invert("qd")
    batch, _ = ctx.batch(st, pats, prec="dd")
    on_inv, _ = ctx.batch(inv, pats, prec="dd")
    on_inv_qd, _ = ctx.batch(inv, pats, prec="qd")
    srv = tg.Server(ctx, workers=2, prec="dd")
    served = [srv.wait(t)[0] for t in [srv.submit(st, p) for p in pats]]
    srv.stop()
    d_out = ctx.batch_async(st, torch.from_numpy(pats).to("cuda"), prec="dd")
    d_inv = ctx.batch_async(inv, torch.from_numpy(pats).to("cuda"), prec="dd")
    torch.cuda.synchronize()
    asyn = tg.results_from_device(d_out)
    asyn_inv = tg.results_from_device(d_inv)
    for pat, b, j, jq, s, a, ai in zip(pats, batch, on_inv, on_inv_qd, served, asyn, asyn_inv):
        single = ctx.probability_displaced(cov, mean, pat, prec="dd")
        key = lambda r: (r.p, r.p_lo, r.T, r.T_lo, r.abs_sum, r.status)
        assert key(single) == key(b) == key(s)
        if not (pat == 0).any():
            assert (a.p, a.p_lo, a.T, a.T_lo) == (b.p, b.p_lo, b.T, b.T_lo)
        else:
            assert a.status == tg.TOR_EINVAL
        if (pat >= 0).all() or not (pat == 0).any():  # async on the inverted state
            assert (ai.p, ai.p_lo) == (j.p, j.p_lo)
        else:
            assert ai.status == tg.TOR_EINVAL
        pb = _mp(b.p, b.p_lo)
        assert _rel(_mp(j.p, j.p_lo), pb) <= j.rel_err_bound + b.rel_err_bound + 1e-27
        assert _rel(_mp(jq.p, jq.p_lo), pb) <= b.rel_err_bound + 1e-27
        if int((pat >= 0).sum()) <= 14:  # the definition route: 2^n Cholesky factorisations
            o = oracle.formP_mean(cov, mean, pat)
            err = _rel(pb, _mp(o.p, o.p_lo))
            assert err <= 1e-10 and err <= b.rel_err_bound + 1e-27, (pat, err, b.rel_err_bound)
    st.close()
    inv.close()
