"""GPU serving: continuous batching returns, for every query, bitwise the
same result as the query evaluated alone; memory admission splits batches;
a full queue refuses submissions with TOR_EAGAIN."""
import threading

import numpy as np
import pytest

import gbs_inputs as gi
import paper_1810_00900_amd as tg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tg.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def setup(ctx):
    covs = [gi.state_m800(30), gi.state_m800(31)]
    states = [ctx.state(c) for c in covs]
    rng = np.random.default_rng(3)
    qs = []
    for i in range(240):
        s = int(rng.integers(2))
        n = int(rng.integers(0, 17))
        qs.append((s, gi.marginal_pattern(800, gi.random_click_set(800, n, rng))))
    return covs, states, qs


def test_alone_vs_mix_identical(ctx, setup):
    covs, states, qs = setup
    alone = [ctx.probability(covs[s], p, prec="dd", tol=1e-10) for s, p in qs]
    with tg.Server(ctx, workers=3, prec="dd", tol=1e-10, max_batch=64) as srv:
        tickets = [None] * len(qs)

        def submit(part):
            for i in part:
                s, p = qs[i]
                tickets[i] = srv.submit(states[s], p)

        th = [threading.Thread(target=submit, args=(range(k, len(qs), 4),)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(qs)
    assert st["batches"] < len(qs)          # queries were fused
    for (r, lat), a in zip(got, alone):
        assert (r.p, r.p_lo, r.abs_sum, r.n_clicks) == (a.p, a.p_lo, a.abs_sum, a.n_clicks)
        assert lat >= 0.0


def test_memory_admission_splits_batches(ctx, setup):
    covs, states, qs = setup
    pats = [gi.config5_pattern(12, seed=s) for s in range(20)]
    # one n = 12 query needs about 17 KB (10-mode tasks) to 28 KB (9-mode)
    with tg.Server(ctx, workers=1, prec="dd", mem_budget_bytes=40 << 10) as srv:
        tickets = [srv.submit(states[0], p) for p in pats]
        res = [srv.wait(t)[0] for t in tickets]
        st = srv.stats()
    assert st["max_batch_seen"] <= 2
    assert st["batches"] >= 10
    for p, r in zip(pats, res):
        a = ctx.probability(covs[0], p, prec="dd")
        assert (r.p, r.p_lo) == (a.p, a.p_lo)


def test_queue_full_eagain(ctx, setup):
    covs, states, qs = setup
    refused = 0
    tickets = []
    pat = gi.config5_pattern(16, seed=1)
    with tg.Server(ctx, workers=1, max_pending=4, prec="dd", max_batch=4) as srv:
        for _ in range(2000):
            try:
                tickets.append(srv.submit(states[1], pat))
            except tg.TorError as e:
                assert e.status == tg.TOR_EAGAIN
                refused += 1
        vals = {srv.wait(t)[0].p for t in tickets}
    assert refused > 0
    assert len(vals) == 1


def test_poll_and_errors(ctx, setup):
    covs, states, qs = setup
    with tg.Server(ctx, workers=1) as srv:
        t = srv.submit(states[0], qs[0][1])
        out = None
        for _ in range(100000):
            out = srv.poll(t)
            if out is not None:
                break
        assert out is not None
        with pytest.raises(tg.TorError):
            srv.poll(t)                    # ticket already released
        bad = qs[1][1].copy()
        bad[0] = 7
        with pytest.raises(tg.TorError) as e:
            srv.submit(states[0], bad)
        assert e.value.status == tg.TOR_EINVAL


def test_concurrent_clients_conditioned_queries(ctx):
    """Patterns with no-click modes from four client threads on fresh states
    (plain and displaced): the workers gather each state's matrices on the
    device from one device copy, created once under the state's lock, and
    every result equals the query alone bitwise."""
    rng = np.random.default_rng(180)
    m = 60
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.8, m))
    mean = gi.random_mean(m, rng, 0.3)
    states = [ctx.state(cov), ctx.state(cov, mean=mean)]
    qs = []
    for i in range(160):
        s = i % 2
        c = gi.random_click_set(m, int(rng.integers(0, 11)), rng)
        p = gi.full_pattern(m, c)
        p[np.setdiff1d(np.arange(m), c)[: int(rng.integers(0, 20))]] = -1
        qs.append((s, p))
    tickets = [None] * len(qs)
    with tg.Server(ctx, workers=3, prec="dd", tol=1e-10, max_batch=16) as srv:
        def client(k):
            for i in range(k, len(qs), 4):
                tickets[i] = srv.submit(states[qs[i][0]], qs[i][1])
        th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        got = [srv.wait(t)[0] for t in tickets]
    for (s, p), g in zip(qs, got):
        w = ctx.probability(cov, p, prec="dd") if s == 0 else ctx.probability_displaced(cov, mean, p, prec="dd")
        assert (g.p, g.p_lo, g.T, g.T_lo, g.status) == (w.p, w.p_lo, w.T, w.T_lo, w.status)
    for st in states:
        st.close()


def test_quad_double_server(ctx):
    """A server with quad-double terms: each query (plain and displaced
    states, marginal and full patterns) is evaluated alone by a worker, and
    its result is bitwise the single quad-double query's."""
    rng = np.random.default_rng(181)
    m = 20
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.8, m))
    mean = gi.random_mean(m, rng, 0.3)
    states = [ctx.state(cov), ctx.state(cov, mean=mean)]
    qs = []
    for i in range(12):
        c = gi.random_click_set(m, int(rng.integers(0, 9)), rng)
        qs.append((i % 2, gi.full_pattern(m, c) if i % 3 else gi.marginal_pattern(m, c)))
    with tg.Server(ctx, workers=3, prec="qd") as srv:
        tickets = [srv.submit(states[s], p) for s, p in qs]
        got = [srv.wait(t)[0] for t in tickets]
    for (s, p), g in zip(qs, got):
        w = ctx.probability(cov, p, prec="qd") if s == 0 else ctx.probability_displaced(cov, mean, p, prec="qd")
        assert (g.p, g.p_lo, g.T, g.T_lo, g.prec_used) == (w.p, w.p_lo, w.T, w.T_lo, tg.PREC_QD)
    for st in states:
        st.close()
