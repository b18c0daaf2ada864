"""No-click conditioning on the GPU (Eq. MatrixUpdate over the no-click modes,
one in-place Schur step per mode, batched over queries).

* 400 two-mode squeezed pairs spread over 800 modes, hundreds of no-click
  modes: the probability against its exact value (mpmath, per independent
  pair, from the binary64 matrix entries) and the pair closed forms;
* a Haar-random 200-mode state, full patterns (every mode observed) against
  the binary128 oracle, which conditions with one Cholesky of sigma_Q[N];
* batches equal single calls bitwise; the conditioning of blocks of up to 16
  no-click modes per pair of launches equals one launch per mode bitwise
  (zero-mean and displaced, full 800-mode patterns, partial blocks).
"""
import itertools

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


def _mp_p(r):
    import mpmath as mp
    mp.mp.dps = 40
    return mp.mpf(r.p) + mp.mpf(r.p_lo)


def _rel(a, b):
    import mpmath as mp
    return abs(float((mp.mpf(a) - mp.mpf(b)) / mp.mpf(b)))


def _exact_pattern_blocks(cov, groups, pattern):
    """Exact probability (mpmath, 60 digits) of `pattern` for a covariance that
    is block diagonal over `groups`: per group the signed sum over subsets Y of
    its clicked modes of det(sigma_Q[Y + its no-click modes])^-1/2."""
    import mpmath as mp
    mp.mp.dps = 60
    P = mp.mpf(1)
    for g in groups:
        C = [i for i in g if pattern[i] == 1]
        N = [i for i in g if pattern[i] == 0]
        s = mp.mpf(0)
        for k in range(len(C) + 1):
            for Y in itertools.combinations(C, k):
                modes = list(Y) + N
                if not modes:
                    s += 1
                    continue
                idx = [q for mode in modes for q in (2 * mode, 2 * mode + 1)]
                M = mp.matrix([[mp.mpf(float(cov[a, b])) + (mp.mpf(1) / 2 if a == b else 0) for b in idx]
                               for a in idx])
                t = 1 / mp.sqrt(mp.det(M))
                s += -t if k % 2 else t
        P *= s
    return P


def _pairs_state(npair, seed):
    rng = np.random.default_rng(seed)
    rs = rng.uniform(0.3, 0.6, npair)
    perm = rng.permutation(2 * npair)
    m = 2 * npair
    cov = np.zeros((2 * m, 2 * m))
    pairs = []
    for k, r in enumerate(rs):
        a, b = int(perm[2 * k]), int(perm[2 * k + 1])
        idx = [2 * a, 2 * a + 1, 2 * b, 2 * b + 1]
        cov[np.ix_(idx, idx)] = gi.tmsv_covariance(r)
        pairs.append((a, b))
    return cov, pairs, rs


def test_tmsv_pairs_800_modes_hundreds_of_no_clicks(ctx):
    cov, pairs, rs = _pairs_state(400, 91)
    m = 800
    pat = -np.ones(m, np.int8)
    kinds = ["11"] * 8 + ["1-"] * 4 + ["00"] * 300 + ["--"] * 88
    closed = 1.0
    for (a, b), r, kd in zip(pairs, rs, kinds):
        if kd == "11":
            pat[a] = pat[b] = 1
            closed *= 1 - 1 / np.cosh(r) ** 2
        elif kd == "1-":
            pat[a] = 1
            closed *= np.tanh(r) ** 2
        elif kd == "00":
            pat[a] = pat[b] = 0
            closed *= 1 / np.cosh(r) ** 2
    assert int((pat == 1).sum()) == 20 and int((pat == 0).sum()) == 600
    want = _exact_pattern_blocks(cov, [list(p) for p in pairs], pat)
    assert abs(float((want - closed) / want)) < 1e-12
    ctx.reset_stats()
    r = ctx.probability(cov, pat, prec="dd")
    assert ctx.stats()["condition_launches"] == 2 * ((600 + 15) // 16)  # blocks of 16 modes, two launches each
    ctx.set_option(tg.OPT_COND_BLOCK, 1)
    try:
        ctx.reset_stats()
        r1 = ctx.probability(cov, pat, prec="dd")
        assert ctx.stats()["condition_launches"] == 600  # one launch per mode
    finally:
        ctx.set_option(tg.OPT_COND_BLOCK, 16)
    assert (r.p, r.p_lo, r.T, r.T_lo, r.abs_sum, r.log_pvac_n) == (r1.p, r1.p_lo, r1.T, r1.T_lo, r1.abs_sum,
                                                                 r1.log_pvac_n)
    assert r.n_clicks == 20
    err = _rel(_mp_p(r), want)
    assert err <= 1e-10
    # the vacuum factor of the 300 no-click pairs
    import mpmath as mp
    want_log_pvac = float(sum(-2 * mp.log(mp.cosh(mp.mpf(float(x)))) for x, kd in zip(rs, kinds) if kd == "00"))
    assert r.log_pvac_n == pytest.approx(want_log_pvac, rel=1e-9)


def test_full_patterns_m200_vs_oracle(ctx):
    rng = np.random.default_rng(200)
    m = 200
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.9, m))
    for n in (0, 6, 12):
        pat = np.zeros(m, np.int8)
        pat[rng.choice(m, n, replace=False)] = 1
        o = oracle.formS(cov, pat)
        r = ctx.probability(cov, pat, prec="dd")
        assert r.n_clicks == n
        err = _rel(_mp_p(r), o.p + o.p_lo)
        assert err <= 1e-10, (n, err)
        assert r.log_pvac_n == pytest.approx(np.log(o.pvac_n), rel=1e-12)


def test_mixed_patterns_batch_equals_single(ctx):
    rng = np.random.default_rng(7)
    m = 120
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.9, m))
    pats = []
    for q in range(9):
        p = rng.choice(np.array([-1, 0, 1], np.int8), m, p=[0.5, 0.42, 0.08])
        if q == 3:
            p[:] = -1          # marginal: nothing to condition
        if q == 5:
            p[p == 1] = 0      # no clicks at all: P(vacuum on N)
        pats.append(p)
    pats = np.stack(pats)
    st = ctx.state(cov)
    res, _ = ctx.batch(st, pats, prec="dd")
    for p, r in zip(pats, res):
        a = ctx.probability(cov, p, prec="dd")
        assert (r.p, r.p_lo, r.abs_sum, r.log_pvac_n) == (a.p, a.p_lo, a.abs_sum, a.log_pvac_n)
        o = oracle.formS(cov, p)
        assert _rel(_mp_p(r), o.p + o.p_lo) <= 1e-10


def test_single_call_device_gather_equals_host_packing(ctx):
    """tor_probability gathers the (C, N) matrix on the device from one copy
    of the covariance when the pattern observes at least half of the modes
    with 64 or more no-click modes, and packs it on the host otherwise; both
    give the words of a state's device gather, so single calls on either side
    of the threshold equal the batched queries of a state bitwise."""
    rng = np.random.default_rng(12)
    m = 120
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.9, m))
    st = ctx.state(cov)
    for k in (40, 63, 64, 100, 112):
        idx = rng.permutation(m)
        p = np.full(m, -1, np.int8)
        p[idx[:8]] = 1
        p[idx[8:8 + k]] = 0
        print("single-call gather, no-click modes", k, flush=True)
        a = ctx.probability(cov, p, prec="dd")
        r = ctx.batch(st, p[None, :], prec="dd")[0][0]
        assert (r.p, r.p_lo, r.abs_sum, r.log_pvac_n, r.rel_err_bound) == \
            (a.p, a.p_lo, a.abs_sum, a.log_pvac_n, a.rel_err_bound), k
        if k in (63, 64):
            o = oracle.formS(cov, p)
            assert _rel(_mp_p(a), o.p + o.p_lo) <= 1e-10
    st.close()


def test_single_call_device_screen_errors(ctx):
    """On the device-gather path of a single call the finiteness and symmetry
    checks of the observed block run on the device: a non-finite or
    asymmetric entry inside the block is reported as by the host scan
    (TOR_EINVAL, naming the entry), one outside it is not read at all."""
    rng = np.random.default_rng(13)
    m = 120
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.9, m))
    idx = rng.permutation(m)
    p = np.full(m, -1, np.int8)
    p[idx[:8]] = 1
    p[idx[8:108]] = 0
    good = ctx.probability(cov, p, prec="dd")
    a, b = 2 * int(idx[3]), 2 * int(idx[50]) + 1   # observed quadratures
    u = 2 * int(idx[115])                          # an unobserved one
    for what, val in (("not symmetric", None), ("non-finite", np.nan), ("non-finite", np.inf)):
        bad = cov.copy()
        if val is None:
            bad[a, b] += 1e-6
        else:
            bad[a, b] = bad[b, a] = val
        with pytest.raises(tg.TorError) as e:
            ctx.probability(bad, p, prec="dd")
        assert e.value.status == tg.TOR_EINVAL and what in str(e.value), str(e.value)
    outside = cov.copy()
    outside[u, a] += 1.0      # the row of an unobserved mode: asymmetric there,
    outside[u, u] = np.nan    # and not finite
    r = ctx.probability(outside, p, prec="dd")
    assert (r.p, r.p_lo, r.abs_sum) == (good.p, good.p_lo, good.abs_sum)


def test_condition_too_many_observed_modes(ctx):
    m = 1030
    cov = 0.5 * np.eye(2 * m)
    pat = np.zeros(m, np.int8)
    pat[:3] = 1
    with pytest.raises(tg.TorError) as e:
        ctx.probability(cov, pat, prec="dd")
    assert e.value.status == tg.TOR_ETOOBIG


FIELDS = ("p", "p_lo", "log_p", "tor", "T", "T_lo", "abs_sum", "log_pvac_n", "n_clicks", "status")


def _same(a, b):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x == y or (x != x and y != y), (f, x, y)


@pytest.mark.parametrize("block", [16, 5, 2])
def test_blocked_conditioning_equals_per_mode(ctx, block):
    """Each entry takes the same rank-2 updates in the same order, whatever the
    block: results are bitwise those of one launch per mode."""
    rng = np.random.default_rng(211)
    cov800 = gi.state_m800(30)
    cases = [(cov800, gi.full_pattern(800, gi.random_click_set(800, 20, rng)), None)]  # 780 no-click modes
    m = 90
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.9, m))
    mean = gi.random_mean(m, rng)
    for n, nz in ((6, m - 6), (0, m), (9, 7), (4, 16), (3, 17)):  # full patterns, and partial blocks
        pat = -np.ones(m, np.int8)
        idx = rng.permutation(m)
        pat[idx[:n]] = 1
        pat[idx[n:n + nz]] = 0
        cases.append((cov, pat, None))
        cases.append((cov, pat, mean))
    want = []
    ctx.set_option(tg.OPT_COND_BLOCK, 1)
    try:
        for c, p, mu in cases:
            want.append(ctx.probability(c, p, prec="dd") if mu is None else
                        ctx.probability_displaced(c, mu, p, prec="dd"))
        ctx.set_option(tg.OPT_COND_BLOCK, block)
        for (c, p, mu), w in zip(cases, want):
            r = ctx.probability(c, p, prec="dd") if mu is None else ctx.probability_displaced(c, mu, p, prec="dd")
            _same(r, w)
        # a batch mixing block counts (queries of a state, conditioned together)
        st = ctx.state(cov)
        pats = np.stack([p for c, p, mu in cases[1:] if mu is None])
        res, _ = ctx.batch(st, pats, prec="dd")
        for r, w in zip(res, [w for (c, p, mu), w in zip(cases[1:], want[1:]) if mu is None]):
            _same(r, w)
        st.close()
    finally:
        ctx.set_option(tg.OPT_COND_BLOCK, 16)
