"""Single-launch subset sums of small zero-mean trees (tor_fused.hip).

A group of trees with at most 22 modes runs in one launch: each workgroup
rebuilds its unit's node from Sigma_C with the expansion's Schur update
(Sec. II, Eq. MatrixUpdate), sums its tasks with the wave tier, and completion
counters order the two reduction stages.  The nodes, the tasks and the order
of every sum are those of the launch chain, so the two paths agree bitwise:

* every tree size 1..22 (every unit layout: a single task, one block, several
  blocks and the second stage, depth-first levels 0..4), both term precisions;
* every task size 1..11 at n = 20 (units of 2^0 .. 2^4 tasks);
* batches of small trees against single calls, repeated calls (the counters
  are left at zero), and the launch counts of both paths;
* the 800-mode marginal patterns of the n = 20 and 22 headline sizes against
  the oracle's exact sum (parity through the single-launch path).
"""
import numpy as np
import pytest

import gbs_inputs as gi
import oracle
import paper_1810_00900_amd as tg

pytestmark = pytest.mark.gpu

FIELDS = ("p", "p_lo", "tor", "log_p", "cancel_ratio", "rel_err_bound", "n_clicks", "prec_used", "status")


@pytest.fixture(scope="module")
def ctx():
    c = tg.Context(0)
    yield c
    c.set_option(tg.OPT_FUSED, 1)
    c.close()


@pytest.fixture(scope="module")
def cov():
    return gi.state_m800(50)


def _same(a, b):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x == y or (x != x and y != y), (f, x, y)


def _both(ctx, fn):
    ctx.set_option(tg.OPT_FUSED, 0)
    ctx.reset_stats()
    r0 = fn()
    s0 = ctx.stats()
    ctx.set_option(tg.OPT_FUSED, 1)
    ctx.reset_stats()
    r1 = fn()
    s1 = ctx.stats()
    return r0, r1, s0, s1


@pytest.mark.parametrize("prec", ["dd", "f64"])
def test_every_size_equals_chain(ctx, cov, prec):
    for n in range(1, 23):
        print("fused n =", n, prec, flush=True)
        pat = gi.config5_pattern(n).copy()
        r0, r1, s0, s1 = _both(ctx, lambda: ctx.probability(cov, pat, prec=prec, tol=1.0))
        _same(r0, r1)
        assert s0["fused_launches"] == 0 and s1["fused_launches"] == 1
        assert s1["expand_launches"] == 0 and s1["reduce_launches"] == 0


@pytest.mark.parametrize("J", list(range(1, 12)))
def test_every_task_size_equals_chain(cov, J):
    c = tg.Context(0)
    try:
        c.set_option(tg.OPT_TASK_MODES, J)
        for n in (J + 5, 20) if J + 5 < 20 else (20,):
            print("fused J =", J, "n =", n, flush=True)
            pat = gi.config5_pattern(n).copy()
            r0, r1, _, s1 = _both(c, lambda: c.probability(cov, pat, prec="dd", tol=1.0))
            _same(r0, r1)
            tasks = 2 ** (n - J)
            assert s1["fused_launches"] == (1 if tasks <= tg.FUSED_MAX_TASKS else 0)
    finally:
        c.close()


def test_batches_and_repeats(ctx, cov):
    st = ctx.state(cov)
    rng = np.random.default_rng(7)
    pats = []
    for n in (4, 9, 12, 15, 17, 18, 20, 0, 11):  # 1867 tasks: one launch
        p = np.full(800, -1, np.int8)
        p[rng.choice(800, n, replace=False)] = 1
        pats.append(p)
    pats = np.stack(pats)
    alone = [ctx.batch(st, p[None, :], prec="dd", tol=1.0)[0][0] for p in pats]
    for rep in range(3):
        print("fused batch rep", rep, flush=True)
        ctx.reset_stats()
        res, _ = ctx.batch(st, pats, prec="dd", tol=1.0)
        s = ctx.stats()
        assert s["fused_launches"] >= 1 and s["expand_launches"] == 0
        for a, b in zip(alone, res):
            _same(a, b)
    ctx.set_option(tg.OPT_FUSED, 0)
    try:
        res0, _ = ctx.batch(st, pats, prec="dd", tol=1.0)
    finally:
        ctx.set_option(tg.OPT_FUSED, 1)
    for a, b in zip(alone, res0):
        _same(a, b)
    st.close()


def test_large_group_takes_the_chain(ctx, cov):
    """A group beyond TOR_FUSED_MAX_TASKS tasks (here 17 trees of 2^10
    tasks) takes the launch chain, with the same results as the trees one at
    a time (each in one launch)."""
    st = ctx.state(cov)
    rng = np.random.default_rng(11)
    pats = []
    for _ in range(17):
        p = np.full(800, -1, np.int8)
        p[rng.choice(800, 20, replace=False)] = 1
        pats.append(p)
    pats = np.stack(pats)
    ctx.reset_stats()
    res, _ = ctx.batch(st, pats, prec="dd", tol=1.0)
    s = ctx.stats()
    assert s["fused_launches"] == 0 and s["expand_launches"] > 0
    for p, r in zip(pats, res):
        _same(ctx.batch(st, p[None, :], prec="dd", tol=1.0)[0][0], r)
    st.close()


def test_option_checked(ctx):
    with pytest.raises(tg.TorError):
        ctx.set_option(tg.OPT_FUSED, 2)
