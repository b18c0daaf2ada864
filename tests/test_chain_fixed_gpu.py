"""The paper's fixed-outcome benchmark chain (gbs_chain_fixed).

* every step probability against the paper's own mode-by-mode rule (the
  oracle's signed mixture of Gaussians, Sec. II, in 40-digit mpmath);
* the product of the steps equals the whole-pattern probability of
  tor_probability;
* P(click) + P(no click) = 1 at a step with a shared history;
* the worst case of the paper's runtime study (all clicks measured first,
  8 dB squeezing, Haar interferometer) at l = 200 modes, 10 clicks;
* quad-double terms (TOR_PREC_QD): the same rule checks, and the worst case
  at l = 512, 16 clicks, where the double-double bound is ~1e-7, against
  tor_probability in quad-double (a different conditioning order).
"""
import numpy as np
import pytest

import gbs_inputs as gi
import oracle
import paper_1810_00900_amd as tg

pytestmark = pytest.mark.gpu
R8DB = 8.0 / (20.0 * np.log10(np.e))     # 8 dB of squeezing


@pytest.fixture(scope="module")
def ctx():
    c = tg.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return abs(float(a) - float(b)) / abs(float(b))


@pytest.mark.parametrize("prec", ["dd", "qd"])
@pytest.mark.parametrize("pat", [
    [1, 0, 1, 1, 0, -1, 1, 0],
    [0, 0, 0, 1, 1, 1, 1, 0],
    [1, 1, 1, 1, 0, 0, 0, 0],
    [-1, 1, -1, 0, 1, -1, 0, 1],
])
def test_steps_match_paper_rule(ctx, pat, prec):
    cov = gi.state_config1()
    pat = np.array(pat, np.int8)
    tot, steps = ctx.chain_fixed(cov, pat, prec=prec)
    want_tot, want = oracle.prob_sequential(cov, pat, dps=40, steps=True)
    for j in range(8):
        if pat[j] < 0:
            assert steps[j] == 1.0
            continue
        assert _rel(steps[j], want[j]) <= 1e-12, (j, steps[j], float(want[j]))
    assert _rel(tot.p + tot.p_lo, want_tot) <= 1e-12
    assert tot.n_clicks == int((pat == 1).sum())


def test_total_equals_probability_and_complementary_steps(ctx):
    rng = np.random.default_rng(12)
    m = 14
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), np.full(m, R8DB))
    pat = rng.choice(np.array([0, 1], np.int8), m, p=[0.6, 0.4])
    tot, steps = ctx.chain_fixed(cov, pat, prec="dd")
    r = ctx.probability(cov, pat, prec="dd")
    assert _rel(tot.p + tot.p_lo, r.p + r.p_lo) <= 1e-12
    assert tot.log_pvac_n == pytest.approx(r.log_pvac_n, rel=1e-12)
    assert np.prod(steps) == pytest.approx(tot.p, rel=1e-12)
    # flip the outcome of the mode measured at step 5 (modes are measured from the last down)
    j = m - 1 - 5
    alt = pat.copy()
    alt[j] = 1 - alt[j]
    _, steps2 = ctx.chain_fixed(cov, alt, prec="dd")
    assert steps[j] + steps2[j] == pytest.approx(1.0, abs=1e-13)
    for k in range(j + 1, m):          # measured before j: same history, same steps
        assert steps[k] == steps2[k]


def test_worst_case_l200_m10(ctx):
    """All 10 clicks in the first 10 measured modes, then 190 no-click steps
    (the paper's worst case at l = 2 m^2)."""
    rng = np.random.default_rng(200)
    l, m = 200, 10
    cov = gi.gbs_covariance(gi.haar_unitary(l, rng), np.full(l, R8DB))
    pat = np.zeros(l, np.int8)
    pat[l - m:] = 1
    ctx.reset_stats()
    tot, steps = ctx.chain_fixed(cov, pat, prec="dd")
    assert ctx.stats()["condition_launches"] == l - m
    assert np.all((steps > 0) & (steps <= 1))
    r = ctx.probability(cov, pat, prec="dd")
    assert _rel(tot.p + tot.p_lo, r.p + r.p_lo) <= max(1e-10, 4 * (tot.rel_err_bound + r.rel_err_bound))
    assert np.prod(steps) == pytest.approx(tot.p, rel=1e-9)


def test_worst_case_l512_m16_quad_double(ctx):
    """All 16 clicks first, then 496 no-click steps: the double-double bound is
    ~1e-7 here; quad-double steps multiply to tor_probability in quad-double
    (conditioned in the opposite mode order) to 1e-25, and complementary
    outcomes at a late step sum to one."""
    rng = np.random.default_rng(512)
    l, m = 512, 16
    cov = gi.gbs_covariance(gi.haar_unitary(l, rng), np.full(l, R8DB))
    pat = np.zeros(l, np.int8)
    pat[l - m:] = 1
    ctx.reset_stats()
    tot, steps = ctx.chain_fixed(cov, pat, prec="qd")
    assert ctx.stats()["condition_launches"] == 2 * (l - m)
    assert tot.prec_used == tg.PREC_QD and tot.status == tg.TOR_OK
    assert tot.rel_err_bound <= 1e-25
    r = ctx.probability(cov, pat, prec="qd")
    assert _rel(tot.p + tot.p_lo, r.p + r.p_lo) <= 1e-25
    d, _ = ctx.chain_fixed(cov, pat, prec="dd")
    assert _rel(d.p + d.p_lo, r.p + r.p_lo) <= max(d.rel_err_bound, 1e-30)
    j = 100  # measured at step l - 1 - j, after all clicks
    alt = pat.copy()
    alt[j] = 1
    _, steps2 = ctx.chain_fixed(cov, alt, prec="qd")
    assert steps[j] + steps2[j] == pytest.approx(1.0, abs=1e-15)


# ---------------------------------------------------------------- displaced states

@pytest.mark.parametrize("pat", [
    [1, 0, 1, 1, 0, -1, 1, 0],
    [0, 0, 0, 1, 1, 1, 1, 0],
    [-1, 1, -1, 0, 1, -1, 0, 1],
])
def test_displaced_steps_match_paper_rule(ctx, pat):
    """gbs_chain_fixed_displaced against the oracle's mode-by-mode rule with
    means (the no-click update moves the mean; 40-digit mpmath)."""
    cov = gi.state_config1()
    pat = np.array(pat, np.int8)
    mu = gi.random_mean(8, np.random.default_rng(300), 0.5)
    tot, steps = ctx.chain_fixed(cov, pat, prec="dd", mean=mu)
    want_tot, want = oracle.prob_sequential(cov, pat, dps=40, steps=True, mean=mu)
    for j in range(8):
        if pat[j] < 0:
            assert steps[j] == 1.0
            continue
        assert _rel(steps[j], want[j]) <= 1e-12, (j, steps[j], float(want[j]))
    assert _rel(tot.p + tot.p_lo, want_tot) <= 1e-12
    r = ctx.probability_displaced(cov, mu, pat, prec="dd")
    assert _rel(tot.p + tot.p_lo, r.p + r.p_lo) <= 1e-12


def test_displaced_coherent_chain_closed_form(ctx):
    """Coherent states through an interferometer stay a product of coherent
    states beta = U alpha: every step is independent of the history,
    P(click) = 1 - exp(-|beta_j|^2)."""
    rng = np.random.default_rng(301)
    m = 24
    U = gi.haar_unitary(m, rng)
    beta = U @ (0.8 * (rng.standard_normal(m) + 1j * rng.standard_normal(m)))
    cov = gi.gbs_covariance(U, np.zeros(m))
    pat = rng.choice(np.array([0, 1], np.int8), m)
    tot, steps = ctx.chain_fixed(cov, pat, prec="dd", mean=gi.coherent_mean(beta))
    pv = np.exp(-np.abs(beta) ** 2)
    want = np.where(pat == 1, 1 - pv, pv)
    assert np.allclose(steps, want, rtol=1e-12, atol=0)
    assert tot.p == pytest.approx(float(np.prod(want)), rel=1e-12)


def test_displaced_chain_zero_mean_is_the_zero_mean_chain(ctx):
    rng = np.random.default_rng(302)
    m = 14
    cov = gi.gbs_covariance(gi.haar_unitary(m, rng), np.full(m, R8DB))
    pat = rng.choice(np.array([-1, 0, 1], np.int8), m, p=[0.2, 0.5, 0.3])
    a, sa = ctx.chain_fixed(cov, pat, prec="dd")
    b, sb = ctx.chain_fixed(cov, pat, prec="dd", mean=np.zeros(2 * m))
    assert np.array_equal(sa, sb)
    assert (a.p, a.p_lo, a.T, a.T_lo) == (b.p, b.p_lo, b.T, b.T_lo)


@pytest.mark.parametrize("pat", [
    [1, 0, 1, 1, 0, -1, 1, 0],
    [-1, 1, -1, 0, 1, -1, 0, 1],
])
def test_displaced_chain_quad_double(ctx, pat):
    """gbs_chain_fixed_displaced with quad-double terms (mean row in the qd
    conditioning snapshots and trees): every step against the oracle's rule
    with means, the whole pattern against tor_probability_displaced in qd."""
    import mpmath as mp
    mp.mp.dps = 50
    cov = gi.state_config1()
    pat = np.array(pat, np.int8)
    mu = gi.random_mean(8, np.random.default_rng(303), 0.5)
    tot, steps = ctx.chain_fixed(cov, pat, prec="qd", mean=mu)
    assert tot.prec_used == tg.PREC_QD
    want_tot, want = oracle.prob_sequential(cov, pat, dps=40, steps=True, mean=mu)
    for j in range(8):
        if pat[j] >= 0:
            assert _rel(steps[j], want[j]) <= 1e-14, (j, steps[j], float(want[j]))
    r = ctx.probability_displaced(cov, mu, pat, prec="qd")
    assert abs(mp.mpf(tot.p) + mp.mpf(tot.p_lo) - (mp.mpf(r.p) + mp.mpf(r.p_lo))) <= 1e-28 * abs(mp.mpf(r.p))
