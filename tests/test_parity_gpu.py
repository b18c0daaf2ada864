"""GPU parity: the HIP subset-tree kernels against the binary128 CPU oracle.

Tolerances: 1e-10 relative for n <= 16 and 1e-8 for n <= 24 (double-double
terms); every result must also lie within the library's own a-priori bound
rel_err_bound = 16 n u R.  Full-size cases (n = 28, 32) are checked against
closed forms that hold at any size (product states, independent two-mode
squeezed pairs).
"""
import json
import os

import numpy as np
import pytest

import gbs_inputs as gi
import oracle
import paper_1810_00900_amd as tg

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rel(a, b):
    """Relative error of a against b; mpmath values keep both double-double
    words (a binary64 sum of hi + lo would round at 1e-16)."""
    import mpmath as mp
    if b == 0:
        return abs(float(a))
    return abs(float((mp.mpf(a) - mp.mpf(b)) / mp.mpf(b)))


def _gpu_p(r):
    import mpmath as mp
    mp.mp.dps = 40
    return mp.mpf(r.p) + mp.mpf(r.p_lo)


def _orc_p(o):
    import mpmath as mp
    mp.mp.dps = 40
    return mp.mpf(o.p) + mp.mpf(o.p_lo)


@pytest.fixture(scope="module")
def ctx():
    c = tg.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def cov800():
    return gi.state_m800(50)


# ---------------------------------------------------------------- small states

@pytest.mark.parametrize("prec", ["dd", "f64"])
def test_config1_all_clicks(ctx, prec):
    cov = gi.state_config1()
    pat = np.ones(8, np.int8)
    o = oracle.formP(cov, pat)
    r = ctx.probability(cov, pat, prec=prec)
    assert r.n_clicks == 8
    assert _rel(_gpu_p(r), _orc_p(o)) <= 1e-10
    assert _rel(_gpu_p(r), _orc_p(o)) <= max(r.rel_err_bound, 1e-30)
    assert r.cancel_ratio == pytest.approx(o.cancel_ratio, rel=1e-9)


def test_config1_normalisation(ctx):
    """Sum over all 2^8 click patterns equals 1 (GPU, each pattern separately)."""
    cov = gi.state_config1()
    tot = 0.0
    for mask in range(256):
        pat = np.array([(mask >> i) & 1 for i in range(8)], np.int8)
        tot += _gpu_p(ctx.probability(cov, pat, prec="dd"))
    assert abs(tot - 1.0) <= 1e-13


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_mixed_patterns_small(ctx, seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(5, 11))
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 1.0, m))
    for _ in range(4):
        pat = rng.integers(-1, 2, size=m).astype(np.int8)
        o = oracle.formP(cov, pat)
        for prec in ("dd", "auto"):
            r = ctx.probability(cov, pat, prec=prec)
            assert _rel(_gpu_p(r), _orc_p(o)) <= 1e-10, (pat, prec)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4])
def test_few_clicks(ctx, n):
    """Tiny trees (fewer modes than one leaf block) and the no-click case."""
    rng = np.random.default_rng(7 + n)
    m = 12
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 1.0, m))
    pat = np.full(m, -1, np.int8)
    pat[rng.choice(m, n, replace=False)] = 1
    pat[0] = 0 if pat[0] != 1 else 1
    o = oracle.prob(cov, pat)
    r = ctx.probability(cov, pat, prec="dd")
    assert _rel(_gpu_p(r), _orc_p(o)) <= 1e-12


def test_vacuum_exact(ctx):
    cov = 0.5 * np.eye(20)
    assert ctx.probability(cov, np.zeros(10, np.int8)).p == 1.0
    for pat in ([1] + [0] * 9, [1] * 10, [1, -1] * 5):
        r = ctx.probability(cov, np.array(pat, np.int8), prec="dd")
        assert r.p == 0.0 and r.p_lo == 0.0


def test_full_patterns_m20(ctx):
    """Patterns with no-click modes: conditioning (Eq. MatrixUpdate over N)."""
    rng = np.random.default_rng(44)
    m = 20
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.9, m))
    for n in (4, 8, 10):
        clicks = gi.random_click_set(m, n, rng)
        pat = gi.full_pattern(m, clicks)
        if n == 8:
            rest = np.setdiff1d(np.arange(m), clicks)
            pat[rest[:3]] = -1          # some modes unobserved
        o = oracle.formS(cov, pat)
        r = ctx.probability(cov, pat, prec="dd")
        err = _rel(_gpu_p(r), _orc_p(o))
        assert err <= 1e-10
        assert err <= r.rel_err_bound


def test_subset_sum_of_oracle_sigma(ctx):
    """tor_subset_sum on the oracle's own conditioned matrix (hi/lo words)."""
    rng = np.random.default_rng(45)
    m = 14
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(0.3, 0.9, m))
    pat = gi.full_pattern(m, [1, 3, 4, 7, 9, 12])
    hi, lo, pv = oracle.conditioned(cov, pat)
    o = oracle.formS(cov, pat)
    r = ctx.subset_sum(hi, lo, prec="dd")
    import mpmath as mp
    want = mp.mpf(o.T) + mp.mpf(o.T_lo)
    assert _rel(_gpu_p(r), want) <= 1e-12
    assert _rel(_gpu_p(r), want) <= r.rel_err_bound


# ---------------------------------------------------------------- 800-mode states

@pytest.mark.parametrize("n", [8, 12, 14, 16])
def test_m800_marginal_1e10(ctx, cov800, n):
    pat = gi.config5_pattern(n)
    o = oracle.formS(cov800, pat)
    r = ctx.probability(cov800, pat, prec="dd")
    err = _rel(_gpu_p(r), _orc_p(o))
    assert err <= 1e-10
    assert err <= r.rel_err_bound
    assert r.cancel_ratio == pytest.approx(o.cancel_ratio, rel=1e-6)


def test_m800_marginal_n20(ctx, cov800):
    pat = gi.config5_pattern(20)
    o = oracle.formS(cov800, pat)
    r = ctx.probability(cov800, pat, prec="dd")
    assert _rel(_gpu_p(r), _orc_p(o)) <= 1e-8


def test_m800_golden_n24(ctx, cov800):
    """n = 24 against a stored oracle value (tests/golden/, written by
    tests/golden/make_golden.py which calls only the oracle)."""
    path = os.path.join(ROOT, "tests", "golden", "config5_marginal.json")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    gold = json.load(open(path))
    for case in gold["cases"]:
        pat = gi.config5_pattern(case["n"], seed=case["seed"])
        r = ctx.probability(cov800 if case["seed"] == 50 else gi.state_m800(case["seed"]), pat, prec="dd")
        import mpmath as mp
        want = mp.mpf(case["p_hi"]) + mp.mpf(case["p_lo"])
        tol = 1e-10 if case["n"] <= 16 else 1e-8
        assert _rel(_gpu_p(r), want) <= tol, case["n"]


def test_m800_bench_configuration_against_quad_double(ctx, cov800):
    """The timed configuration itself (n = 28 marginal on the 800-mode state,
    dd terms, default 10-mode tasks): too large for the oracle (~50 min on 16
    cores), checked against the quad-double tier, whose bound there is ~1e-40
    and which is pinned to the oracle and to exact closed forms in
    test_qd_gpu.py."""
    import mpmath as mp
    pat = gi.config5_pattern(28)
    r = ctx.probability(cov800, pat, prec="dd")
    q = ctx.probability(cov800, pat, prec="qd")
    assert q.rel_err_bound <= 1e-30
    want = mp.mpf(q.p) + mp.mpf(q.p_lo)
    err = _rel(_gpu_p(r), want)
    assert err <= r.rel_err_bound and err <= 1e-8, (err, r.rel_err_bound)
    assert r.cancel_ratio == pytest.approx(q.cancel_ratio, rel=1e-6)


def test_m800_largest_tree_against_quad_double(ctx, cov800):
    """The largest tree the library takes (n = 32 clicks, 2^32 subsets; a
    32-click marginal of the 800-mode state): double-double terms against the
    quad-double tier, within the dd bound."""
    import mpmath as mp
    pat = gi.config5_pattern(32)
    assert int((pat == 1).sum()) == 32
    r = ctx.probability(cov800, pat, prec="dd")
    big = tg.Context(0)  # the quad-double tree of 32 modes holds ~96 GB of HBM
    big.set_option(tg.OPT_MEM_BUDGET, 160 << 30)
    q = big.probability(cov800, pat, prec="qd")
    big.close()
    assert q.rel_err_bound <= 1e-30
    err = _rel(_gpu_p(r), mp.mpf(q.p) + mp.mpf(q.p_lo))
    print("n = 32: dd vs qd", err, "dd bound", r.rel_err_bound, "R", q.cancel_ratio)
    assert err <= r.rel_err_bound, (err, r.rel_err_bound)
    assert r.cancel_ratio == pytest.approx(q.cancel_ratio, rel=1e-4)


def test_auto_escalates(ctx, cov800):
    """AUTO starts with binary64 terms and repeats in double-double when the
    bound exceeds tol."""
    pat = gi.config5_pattern(14)
    r = ctx.probability(cov800, pat, prec="auto", tol=1e-10)
    assert r.prec_used == tg.PREC_DD
    r64 = ctx.probability(cov800, pat, prec="f64", tol=1e-10)
    assert r64.status == tg.TOR_WARN_PRECISION
    o = oracle.formS(cov800, pat)
    assert _rel(_gpu_p(r64), _orc_p(o)) <= r64.rel_err_bound


# ---------------------------------------------------------------- any size

def _target(n):
    return 1e-10 if n <= 16 else 1e-8


def _mp_rel(r, want):
    """Relative error of the library's double-double p against an mpmath value
    (both words of p enter; a binary64 sum would round at 1e-16)."""
    import mpmath as mp
    got = mp.mpf(r.p) + mp.mpf(r.p_lo)
    return abs(float((got - want) / want))


def _exact_blocks(cov, groups):
    """Exact probability (mpmath, 60 digits) that every mode clicks, for a
    covariance that is block diagonal over the given groups of modes: the
    product over groups of sum_{Y subset of group} (-1)^|Y| det(sigma_Q[Y])^-1/2,
    from the binary64 matrix entries themselves."""
    import itertools

    import mpmath as mp
    mp.mp.dps = 60
    P = mp.mpf(1)
    for g in groups:
        s = mp.mpf(0)
        for k in range(len(g) + 1):
            for Y in itertools.combinations(g, k):
                if not Y:
                    s += 1
                    continue
                idx = [q for mode in Y for q in (2 * mode, 2 * mode + 1)]
                M = mp.matrix([[mp.mpf(float(cov[a, b])) + (mp.mpf(1) / 2 if a == b else 0) for b in idx]
                               for a in idx])
                t = 1 / mp.sqrt(mp.det(M))
                s += -t if k % 2 else t
        P *= s
    return P


@pytest.mark.parametrize("n", [10, 20, 28, 32])
def test_product_state_closed_form(ctx, n):
    """Independent squeezed modes (r ~ U[0.8, 1.3], per-mode cancellation
    similar to the 800-mode workloads): p = prod (1 - q_i), exact in mpmath."""
    rng = np.random.default_rng(1000 + n)
    params = [(rng.uniform(0.8, 1.3), rng.uniform(0, np.pi), 0.0) for _ in range(n)]
    cov = gi.direct_sum([gi.single_mode_covariance(*p) for p in params])
    want = _exact_blocks(cov, [[i] for i in range(n)])
    closed = np.prod([1 - 1 / np.cosh(p[0]) for p in params])
    assert abs(float((want - closed) / want)) < 1e-13      # the matrix is that state
    r = ctx.probability(cov, np.ones(n, np.int8), prec="dd")
    assert r.cancel_ratio > 1e6
    err = _mp_rel(r, want)
    assert err <= r.rel_err_bound
    assert err <= (_target(n) if n <= 24 else 1e-8)


def test_tmsv_pairs_28(ctx):
    """14 independent two-mode squeezed pairs, all 28 modes clicked, the two
    modes of each pair far apart in the ordering: p = prod (1 - 1/cosh^2 r)."""
    rng = np.random.default_rng(77)
    npair = 14
    rs = rng.uniform(0.6, 1.0, npair)
    m = 2 * npair
    cov = np.zeros((2 * m, 2 * m))
    for k, r in enumerate(rs):
        a, b = k, k + npair
        idx = [2 * a, 2 * a + 1, 2 * b, 2 * b + 1]
        cov[np.ix_(idx, idx)] = gi.tmsv_covariance(r)
    want = _exact_blocks(cov, [[k, k + npair] for k in range(npair)])
    closed = np.prod(1 - 1 / np.cosh(rs) ** 2)
    assert abs(float((want - closed) / want)) < 1e-13
    r = ctx.probability(cov, np.ones(m, np.int8), prec="dd")
    err = _mp_rel(r, want)
    assert err <= r.rel_err_bound
    assert err <= 1e-8


# ---------------------------------------------------------------- plan and determinism

def test_tiling_independent(ctx, cov800):
    pat = gi.config5_pattern(16)
    vals = []
    c = tg.Context(0)
    for j in (3, 5, 7, 9, 10, 11):
        c.set_option(tg.OPT_TASK_MODES, j)
        vals.append(_gpu_p(c.probability(cov800, pat, prec="dd")))
    c.close()
    for v in vals[1:]:
        assert _rel(v, vals[0]) <= 1e-13


@pytest.mark.parametrize("J,n", [(10, 10), (10, 12), (10, 16), (11, 11), (11, 12), (11, 16)])
def test_top_level_tasks_vs_oracle(ctx, cov800, J, n):
    """10- and 11-mode wave tasks (top one or two decisions in LDS, then
    nine-mode trees): n = J is one task with no HBM level, larger n span
    2^(n-J) tasks."""
    pat = gi.config5_pattern(n)
    o = oracle.formS(cov800, pat)
    c = tg.Context(0)
    try:
        c.set_option(tg.OPT_TASK_MODES, J)
        r = c.probability(cov800, pat, prec="dd")
        c.set_option(tg.OPT_TASK_MODES, 9)
        r9 = c.probability(cov800, pat, prec="dd")
    finally:
        c.close()
    err = _rel(_gpu_p(r), _orc_p(o))
    assert err <= 1e-10
    assert err <= r.rel_err_bound
    assert _rel(_gpu_p(r), _gpu_p(r9)) <= 1e-13
    assert r.abs_sum == pytest.approx(r9.abs_sum, rel=1e-13)


@pytest.mark.parametrize("J", [10, 11])
def test_top_level_tasks_f64(ctx, cov800, J):
    pat = gi.config5_pattern(14)
    o = oracle.formS(cov800, pat)
    c = tg.Context(0)
    try:
        c.set_option(tg.OPT_TASK_MODES, J)
        r = c.probability(cov800, pat, prec="f64")
    finally:
        c.close()
    assert _rel(_gpu_p(r), _orc_p(o)) <= r.rel_err_bound


def test_deterministic(ctx, cov800):
    pat = gi.config5_pattern(18)
    a = ctx.probability(cov800, pat, prec="dd")
    b = ctx.probability(cov800, pat, prec="dd")
    assert (a.p, a.p_lo, a.abs_sum) == (b.p, b.p_lo, b.abs_sum)


def test_batch_matches_single(ctx, cov800):
    st = ctx.state(cov800)
    rng = np.random.default_rng(5)
    pats = np.stack([gi.marginal_pattern(800, gi.random_click_set(800, int(k), rng))
                     for k in (8, 11, 13, 9, 15)])
    res, status = ctx.batch(st, pats, prec="dd")
    assert status >= 0
    for p, r in zip(pats, res):
        s = ctx.probability(cov800, p, prec="dd")
        assert (r.p, r.p_lo) == (s.p, s.p_lo)


def test_batch_mixed_sizes_and_errors(ctx, cov800):
    """A batch mixing tree sizes (n = 0..20, J < 9 and J = 9 trees), an
    invalid pattern and duplicates: every valid result equals the same query
    run alone, bitwise; the invalid one reports its own status."""
    st = ctx.state(cov800)
    rng = np.random.default_rng(9)
    ns = [0, 1, 2, 5, 8, 9, 10, 13, 17, 20, 3, 9]
    pats = [gi.marginal_pattern(800, gi.random_click_set(800, n, rng)) for n in ns]
    bad = pats[3].copy()
    bad[7] = 5
    pats.insert(4, bad)
    pats.append(pats[7].copy())
    res, status = ctx.batch(st, np.stack(pats), prec="auto", tol=1e-10)
    assert status == tg.TOR_EINVAL
    assert res[4].status == tg.TOR_EINVAL
    for i, (p, r) in enumerate(zip(pats, res)):
        if i == 4:
            continue
        s = ctx.probability(cov800, p, prec="auto", tol=1e-10)
        assert (r.p, r.p_lo, r.abs_sum, r.prec_used) == (s.p, s.p_lo, s.abs_sum, s.prec_used), i
        o = oracle.prob(cov800, p) if r.n_clicks <= 14 else None
        if o is not None:
            assert _rel(_gpu_p(r), _orc_p(o)) <= 1e-10


# ---------------------------------------------------------------- errors

def test_errors(ctx):
    cov = 0.5 * np.eye(8)
    with pytest.raises(tg.TorError) as e:
        ctx.probability(cov, np.array([1, 2, 0, 0], np.int8))
    assert e.value.status == tg.TOR_EINVAL
    bad = cov.copy()
    bad[2, 2] = -1.0
    with pytest.raises(tg.TorError) as e:
        ctx.probability(bad, np.array([1, 1, 0, 0], np.int8))
    assert e.value.status == tg.TOR_ENOTPD
    asym = cov.copy()
    asym[3, 0] = 0.1
    with pytest.raises(tg.TorError) as e:
        ctx.probability(asym, np.array([1, 1, 0, 0], np.int8))
    assert e.value.status == tg.TOR_EINVAL
    big = 0.5 * np.eye(2 * 33)
    with pytest.raises(tg.TorError) as e:
        ctx.probability(big, np.ones(33, np.int8))
    assert e.value.status == tg.TOR_ETOOBIG
