"""Persistent request loop (tor_pserver_*): one long-running kernel takes
probability queries and sampling batches as they are submitted.

* every probability result equals tor_batch's on the same state and pattern
  (double-double terms) bitwise, in every field, whether the query ran alone
  or in a mix of concurrent submissions from several threads;
* sampling batches return gbs_trace's outcomes and statuses bitwise, also when
  they run beside probability queries;
* the kernel stops on the host's stop flag with an idle ring, exits as a
  whole after its idle limit and is launched again on demand, also when work
  arrives while it is closing;
* admission refuses a query whose partial sums do not fit (TOR_EAGAIN) and
  takes it once results are read; argument errors.
"""
import threading
import time

import numpy as np
import pytest

import gbs_inputs as gi
import paper_1810_00900_amd as tg

pytestmark = pytest.mark.gpu

FIELDS = ("p", "p_lo", "log_p", "tor", "T", "T_lo", "abs_sum", "cancel_ratio", "rel_err_bound", "log_pvac_n",
          "n_clicks", "prec_used", "status")


@pytest.fixture(scope="module")
def ctx():
    c = tg.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def states(ctx):
    covs = [gi.state_m800(30), gi.state_m800(31)]
    sts = [ctx.state(c) for c in covs]
    yield covs, sts
    for s in sts:
        s.close()


def _same(a, b):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x == y or (x != x and y != y), (f, x, y)


def _queries(seed, nq, nmax=20):
    rng = np.random.default_rng(seed)
    qs = []
    for _ in range(nq):
        s = int(rng.integers(2))
        n = int(rng.integers(0, nmax + 1))
        qs.append((s, gi.marginal_pattern(800, gi.random_click_set(800, n, rng))))
    return qs


def test_alone_equals_tor_batch(ctx, states):
    covs, sts = states
    qs = _queries(501, 24) + [(0, gi.marginal_pattern(800, list(range(0, 800, 36))[:22]))]
    want = [ctx.batch(sts[s], p[None, :], prec="dd")[0][0] for s, p in qs]
    with tg.PServer(ctx) as srv:
        for (s, p), w in zip(qs, want):
            print("alone n =", int((p == 1).sum()), flush=True)
            r, lat = srv.wait(srv.submit(sts[s], p))
            _same(r, w)
            assert lat > 0 if (p == 1).any() else lat >= 0  # no clicks: finished on the host
        st = srv.stats()
    assert st["completed"] == len(qs) and st["pending"] == 0


def test_mix_from_threads_equals_alone(ctx, states):
    covs, sts = states
    qs = _queries(502, 160, nmax=18)
    want = []
    for s in (0, 1):
        idx = [i for i, (ss, _) in enumerate(qs) if ss == s]
        res, _ = ctx.batch(sts[s], np.stack([qs[i][1] for i in idx]), prec="dd")
        want += list(zip(idx, res))
    want = dict(want)
    got = [None] * len(qs)
    with tg.PServer(ctx) as srv:
        tickets = [None] * len(qs)

        def submit(part):
            for i in part:
                s, p = qs[i]
                tickets[i] = srv.submit(sts[s], p)

        th = [threading.Thread(target=submit, args=(range(k, len(qs), 4),)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        print("mix: submitted", len(qs), flush=True)
        for i, t in enumerate(tickets):
            got[i] = srv.wait(t)[0]
    for i in range(len(qs)):
        _same(got[i], want[i])


def test_full_patterns_of_inverted_state(ctx):
    rng = np.random.default_rng(503)
    U = gi.haar_unitary(24, rng)
    cov = gi.gbs_covariance(U, rng.uniform(0.3, 0.9, 24))
    inv = ctx.state(cov).invert("dd")
    pats = [gi.full_pattern(24, gi.random_click_set(24, n, rng)) for n in (1, 4, 9, 13, 16)]
    pats += [gi.marginal_pattern(24, gi.random_click_set(24, n, rng)) for n in (5, 12)]
    want, _ = ctx.batch(inv, np.stack(pats), prec="dd")
    with tg.PServer(ctx) as srv:
        ts = [srv.submit(inv, p) for p in pats]
        for t, w in zip(ts, want):
            _same(srv.wait(t)[0], w)
        # a pattern with no-click and unobserved modes needs per-query conditioning
        bad = pats[0].copy()
        bad[np.nonzero(bad == 0)[0][0]] = -1
        with pytest.raises(tg.TorError) as ei:
            srv.submit(inv, bad)
        assert ei.value.status == tg.TOR_EINVAL
    inv.close()


def test_sampling_beside_probability(ctx, states):
    covs, sts = states
    cov2 = gi.state_config2()
    st2 = ctx.state(cov2)
    seed, n_post = 77, 12
    batches = [(0, 48), (48, 40), (88, 64)]
    qs = _queries(504, 30, nmax=16)
    want_p = {}
    for i, (s, p) in enumerate(qs):
        want_p[i] = ctx.batch(sts[s], p[None, :], prec="dd")[0][0]
    with tg.PServer(ctx) as srv:
        tickets = []
        for b, (c0, nc) in enumerate(batches):
            tickets.append(("c", b, srv.submit_chains(st2, n_post, seed, c0, nc)))
            for i in range(b * 10, b * 10 + 10):
                tickets.append(("p", i, srv.submit(sts[qs[i][0]], qs[i][1])))
        print("mixed: submitted", len(tickets), flush=True)
        got_c, got_p = {}, {}
        for kind, i, t in tickets:
            if kind == "c":
                got_c[i] = srv.wait_chains(t)
            else:
                got_p[i] = srv.wait(t)[0]
    for i, r in got_p.items():
        _same(r, want_p[i])
    for b, (c0, nc) in enumerate(batches):
        _, _, oc, stt = ctx.gbs_trace(cov2, n_post, seed, c0, nc)
        outcomes, status, lat = got_c[b]
        np.testing.assert_array_equal(outcomes, oc)
        np.testing.assert_array_equal(status, stt)
    st2.close()


def test_idle_ring_stop(ctx):
    srv = tg.PServer(ctx, idle_ms=60000)
    st = srv.stats()
    assert st["running"] == 1 and st["launches"] == 1
    t0 = time.perf_counter()
    srv.stop()
    assert time.perf_counter() - t0 < 5.0


def test_idle_exit_and_relaunch(ctx, states):
    covs, sts = states
    p = gi.marginal_pattern(800, list(range(3, 800, 61)))
    want = ctx.batch(sts[0], p[None, :], prec="dd")[0][0]
    def exit_seen(srv, limit=5.0):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < limit:
            if not srv.stats()["running"]:
                return time.perf_counter() - t0
            time.sleep(0.002)
        return None

    with tg.PServer(ctx, idle_ms=2) as srv:
        w = exit_seen(srv)
        print("idle exit seen after", w, srv.stats(), flush=True)
        assert w is not None  # exited without work
        _same(srv.wait(srv.submit(sts[0], p))[0], want)
        w = exit_seen(srv)
        print("idle exit seen after", w, srv.stats(), flush=True)
        assert w is not None
        _same(srv.wait(srv.submit(sts[0], p))[0], want)
        assert srv.stats()["launches"] >= 3


def test_relaunch_races(ctx, states):
    """Submissions at random moments around the kernel's idle exit (1 ms):
    some land while the launch is closing (the next launch is queued behind
    it), some after it has left; every result stays tor_batch's."""
    covs, sts = states
    rng = np.random.default_rng(508)
    pats = [gi.marginal_pattern(800, gi.random_click_set(800, int(n), rng)) for n in rng.integers(4, 15, 8)]
    want = [ctx.batch(sts[0], p[None, :], prec="dd")[0][0] for p in pats]
    with tg.PServer(ctx, idle_ms=1) as srv:
        for i in range(120):
            time.sleep(float(rng.uniform(0.0, 0.003)))
            k = i % len(pats)
            _same(srv.wait(srv.submit(sts[0], pats[k]))[0], want[k])
        st = srv.stats()
        print("relaunches:", st["launches"], flush=True)
    assert st["launches"] > 1


def test_full_ring_reuse(ctx, states):
    """A closed loop that keeps the request ring full (every slot reused three
    times while the completion watcher scans it): each result is its own
    query's, bitwise tor_batch's."""
    import collections
    covs, sts = states
    rng = np.random.default_rng(509)
    pats = [gi.marginal_pattern(800, gi.random_click_set(800, int(n), rng)) for n in rng.integers(1, 7, 16)]
    want = [ctx.batch(sts[1], p[None, :], prec="dd")[0][0] for p in pats]
    total = 3 * tg.PS_SLOTS + 100
    done = 0
    with tg.PServer(ctx) as srv:
        pending = collections.deque()
        for i in range(total):
            while True:
                try:
                    pending.append((i % len(pats), srv.submit(sts[1], pats[i % len(pats)])))
                    break
                except tg.TorError as e:
                    assert e.status == tg.TOR_EAGAIN and pending
                    k, t = pending.popleft()
                    _same(srv.wait(t)[0], want[k])
                    done += 1
        while pending:
            k, t = pending.popleft()
            _same(srv.wait(t)[0], want[k])
            done += 1
    assert done == total
    print("full ring: queries", total, flush=True)


def test_admission_by_memory(ctx, states):
    covs, sts = states
    rng = np.random.default_rng(505)
    big = gi.marginal_pattern(800, gi.random_click_set(800, 22, rng))
    small = gi.marginal_pattern(800, gi.random_click_set(800, 12, rng))
    # a query needs its 2^(n - J) task partials and the reduction stages' (32 bytes each)
    tasks = 2 ** (22 - ctx.tuning("dd", 22))
    parts = tasks
    while tasks > 1:
        tasks = -(-tasks // 1024)
        parts += tasks
    budget = int(1.5 * parts * 32)  # one big query and a small one, not two big ones
    with tg.PServer(ctx, mem_budget_bytes=budget) as srv:
        t1 = srv.submit(sts[0], big)
        with pytest.raises(tg.TorError) as ei:
            srv.submit(sts[1], big)
        assert ei.value.status == tg.TOR_EAGAIN
        t2 = srv.submit(sts[1], small)  # still fits
        srv.wait(t1)
        srv.wait(t2)
        t3 = srv.submit(sts[1], big)  # admitted once the first result is read
        _same(srv.wait(t3)[0], ctx.batch(sts[1], big[None, :], prec="dd")[0][0])


def test_errors(ctx, states):
    covs, sts = states
    rng = np.random.default_rng(506)
    disp = ctx.state(covs[0][:20, :20], mean=gi.random_mean(10, rng))
    with tg.PServer(ctx) as srv:
        with pytest.raises(tg.TorError) as ei:
            srv.submit(disp, gi.marginal_pattern(10, [1, 2]))
        assert ei.value.status == tg.TOR_EINVAL
        with pytest.raises(tg.TorError) as ei:
            srv.submit_chains(sts[0], 16, 1, 0, 4)
        assert ei.value.status == tg.TOR_ETOOBIG
        part = gi.marginal_pattern(800, [1, 5])
        part[9] = 0  # a no-click mode on a state that is not inverted
        with pytest.raises(tg.TorError) as ei:
            srv.submit(sts[0], part)
        assert ei.value.status == tg.TOR_EINVAL
        with pytest.raises(tg.TorError):
            srv.poll(123456789)
    disp.close()


def test_autotune_unit_depth(ctx, states, tmp_path):
    """The persistent autotuner picks a unit depth per n, writes it with the
    task sizes, and results stay bitwise tor_batch's (the task size is the
    batched path's)."""
    import json
    covs, sts = states
    path = tmp_path / "tune.json"
    rng = np.random.default_rng(507)
    pats = [gi.marginal_pattern(800, gi.random_click_set(800, n, rng)) for n in (14, 15, 16)]
    want = [ctx.batch(sts[0], p[None, :], prec="dd")[0][0] for p in pats]
    with tg.PServer(ctx) as srv:
        srv.autotune(14, 16, path)
        for p, w in zip(pats, want):
            _same(srv.wait(srv.submit(sts[0], p))[0], w)
    d = json.load(open(path))
    assert {f"pst:{n}" for n in (14, 15, 16)} <= set(d["persistent_unit_levels"])
    for n in (14, 15, 16):
        assert 0 <= d["persistent_unit_levels"][f"pst:{n}"] <= n - ctx.tuning("dd", n)
    with tg.Context(0) as c2:
        c2.load_tuning(path)
