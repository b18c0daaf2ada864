"""GPU chain-rule sampler: coins, per-mode probabilities and sample
distributions against the CPU oracle.

* the device coin equals the reference Philox4x32-10 draw for (seed, chain, mode);
* replayed per-mode click probabilities equal the oracle's ratio
  p(C + j, N) / p(C, N + j unobserved) to the binary64-term bound 16 n u R
  (R from the oracle's own sum);
* outcomes follow the coins (click iff u < P(click));
* empirical distributions over all patterns of small states match the exact
  (oracle) distribution by a chi-square test, with and without postselection.
"""
import itertools

import numpy as np
import pytest
from scipy import stats as sps

import gbs_inputs as gi
import oracle
import paper_1810_00900_amd as tg
from philox_ref import uniform as philox_uniform

pytestmark = pytest.mark.gpu
U53 = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    c = tg.Context(0)
    yield c
    c.close()


def _small_state(m, seed, lo=0.3, hi=1.0):
    rng = np.random.default_rng(seed)
    return gi.gbs_covariance(gi.haar_unitary(m, rng), rng.uniform(lo, hi, m))


def test_coins_are_philox(ctx):
    cov = _small_state(6, 1)
    seed = 0x1234_5678_9ABC_DEF0
    pc, un, oc, st = ctx.gbs_trace(cov, -1, seed, 1000, 8)
    for c in range(8):
        for j in range(6):
            assert un[c, j] == philox_uniform(seed, 1000 + c, j)
            assert oc[c, j] == (1 if un[c, j] < pc[c, j] else 0)
    assert (st == 1).all()


def _oracle_click_prob(cov, m, hist, j):
    """P(click at j | outcomes hist[0..j-1]) from two oracle probabilities."""
    base = np.full(m, -1, np.int8)
    base[:j] = hist[:j]
    num = base.copy()
    num[j] = 1
    den = base
    a = oracle.formS(cov, num)
    b = oracle.formS(cov, den)
    R = max(a.cancel_ratio, b.cancel_ratio)
    return (a.p + a.p_lo) / (b.p + b.p_lo), R


def test_replay_small_all_steps(ctx):
    m = 7
    cov = _small_state(m, 2)
    pc, un, oc, st = ctx.gbs_trace(cov, -1, 99, 0, 6)
    for c in range(6):
        for j in range(m):
            want, R = _oracle_click_prob(cov, m, oc[c], j)
            n = int(oc[c, :j].sum()) + 1
            tol = 16 * n * U53 * max(R, 1.0) * 4 + 1e-14
            assert abs(pc[c, j] - want) <= tol * max(abs(want), 1e-300), (c, j, pc[c, j], want)


def test_replay_config2_postselected(ctx):
    """m = 100, r = 0.6 (the postselected sampling workload): replay chains and
    check sampled steps, including steps with up to 12 clicks, against the
    oracle."""
    m = 100
    cov = gi.state_config2()
    pc, un, oc, st = ctx.gbs_trace(cov, 12, 2, 0, 24)
    rng = np.random.default_rng(0)
    checked = 0
    deep = 0
    for c in range(24):
        evaluated = np.nonzero(~np.isnan(pc[c]))[0]
        if len(evaluated) == 0:
            continue
        # the last evaluated step (deepest click count) plus a random earlier one
        for j in {int(evaluated[-1]), int(rng.choice(evaluated))}:
            want, R = _oracle_click_prob(cov, m, oc[c], j)
            n = int(oc[c, :j].sum()) + 1
            deep = max(deep, n - 1)
            tol = 16 * n * U53 * max(R, 1.0) * 4 + 1e-14
            assert abs(pc[c, j] - want) <= tol * abs(want), (c, j, pc[c, j], want, R)
            checked += 1
        if checked >= 16:
            break
    assert deep >= 8


def test_postselection_stops(ctx):
    """A rejected chain stops as soon as n_post can no longer be met; accepted
    chains have exactly n_post clicks."""
    m = 100
    cov = gi.state_config2()
    pc, un, oc, st = ctx.gbs_trace(cov, 12, 2, 0, 64)
    for c in range(64):
        ev = ~np.isnan(pc[c])
        clicks = int(oc[c].sum())
        if st[c] == 1:
            assert clicks == 12 and ev.all()
        else:
            assert st[c] == 0
            last = int(np.nonzero(ev)[0][-1])
            # stopped right after the 13th click, or when too few modes remained
            assert clicks == 13 or clicks + (m - last - 1) < 12


def _chi2_pvalue(samples, probs):
    m = samples.shape[1]
    keys = samples @ (1 << np.arange(m))
    counts = np.bincount(keys, minlength=1 << m).astype(float)
    n = samples.shape[0]
    exp = n * probs
    mask = exp > 5
    chi2 = float(((counts[mask] - exp[mask]) ** 2 / exp[mask]).sum())
    # lump the rare cells
    rare_o, rare_e = counts[~mask].sum(), exp[~mask].sum()
    k = int(mask.sum())
    if rare_e > 5:
        chi2 += (rare_o - rare_e) ** 2 / rare_e
        k += 1
    return sps.chi2.sf(chi2, k - 1)


def test_distribution_m5(ctx):
    m = 5
    cov = _small_state(m, 3, 0.5, 1.2)
    probs = np.array([oracle.formP(cov, np.array([(k >> i) & 1 for i in range(m)], np.int8)).p
                      for k in range(1 << m)])
    assert abs(probs.sum() - 1) < 1e-13
    samples, st = ctx.gbs_sample(cov, -1, 7, 200000)
    assert st["chains_started"] == 200000 and st["chains_accepted"] == 200000
    assert _chi2_pvalue(samples, probs) > 1e-4


def test_distribution_postselected(ctx):
    """m = 8 (the 8-mode state), postselected on 4 clicks: the accepted samples
    follow the conditional distribution over the 70 four-click patterns."""
    m, npost = 8, 4
    cov = gi.state_config1()
    pats = [np.array(b, np.int8) for b in itertools.product((0, 1), repeat=m) if sum(b) == npost]
    pk = np.array([oracle.formP(cov, p).p for p in pats])
    full = np.zeros(1 << m)
    for p, v in zip(pats, pk):
        full[int((p.astype(np.int64) << np.arange(m)).sum())] = v
    full /= full.sum()
    samples, st = ctx.gbs_sample(cov, npost, 11, 30000)
    assert (samples.sum(axis=1) == npost).all()
    acc = st["chains_accepted"] / st["chains_started"]
    assert acc == pytest.approx(pk.sum(), rel=0.05)
    assert _chi2_pvalue(samples, full) > 1e-4


def test_deterministic(ctx):
    cov = _small_state(6, 4)
    a, sa = ctx.gbs_sample(cov, 2, 5, 500)
    b, sb = ctx.gbs_sample(cov, 2, 5, 500)
    assert (a == b).all() and sa["chains_started"] == sb["chains_started"]
    c, _ = ctx.gbs_sample(cov, 2, 6, 500)
    assert not (a == c).all()


def test_resume_from_chain_index(ctx):
    """Chain k's outcome is a pure function of (seed, k): replaying a window of
    chains reproduces the accepted samples found there."""
    cov = _small_state(6, 5)
    samples, st = ctx.gbs_sample(cov, 3, 8, 40)
    pc, un, oc, stt = ctx.gbs_trace(cov, 3, 8, 0, int(st["chains_started"]))
    acc = oc[stt == 1]
    assert (acc[:40] == samples).all()


def test_sampler_errors(ctx):
    cov = _small_state(6, 6)
    with pytest.raises(tg.TorError):
        ctx.gbs_sample(cov, 21, 1, 10)
    with pytest.raises(tg.TorError):
        ctx.set_option(tg.OPT_CHAIN_CLICKS, 21)
    bad = cov.copy()
    bad[0, 1] += 1.0
    with pytest.raises(tg.TorError):
        ctx.gbs_sample(bad, 2, 1, 10)


def test_many_clicks_product_state(ctx):
    """Chains carrying up to 20 clicks (the large sampler kernel): on a
    product of squeezed modes the click probability of mode j is
    1 - 1/cosh(r_j) whatever the history, at any click count; the replayed
    probabilities must match it within the binary64-term bound."""
    rng = np.random.default_rng(31)
    m = 30
    rs = rng.uniform(1.4, 1.8, m)
    cov = gi.direct_sum([gi.single_mode_covariance(r, rng.uniform(0, np.pi)) for r in rs])
    pc, un, oc, st = ctx.gbs_trace(cov, 18, 4, 0, 16)
    want = 1.0 - 1.0 / np.cosh(rs)
    deep = 0
    for c in range(16):
        for j in np.nonzero(~np.isnan(pc[c]))[0]:
            n = int(oc[c, :j].sum())
            deep = max(deep, n)
            R = np.prod([(1 + 1 / np.cosh(rs[i])) / (1 - 1 / np.cosh(rs[i])) for i in np.nonzero(oc[c, :j])[0]])
            tol = 16 * (n + 1) * U53 * R * 4 + 1e-14
            assert abs(pc[c, j] - want[j]) <= tol * want[j], (c, j, n, pc[c, j], want[j])
    assert deep >= 16
    samples, s2 = ctx.gbs_sample(cov, 18, 4, 20)
    assert (samples.sum(axis=1) == 18).all()


def test_chain_click_cap_option(ctx):
    rng = np.random.default_rng(32)
    m = 24
    rs = rng.uniform(1.2, 1.6, m)
    cov = gi.direct_sum([gi.single_mode_covariance(r) for r in rs])
    with tg.Context(0) as c:
        _, s15 = c.gbs_sample(cov, -1, 9, 200)
        c.set_option(tg.OPT_CHAIN_CLICKS, 20)
        smp, s20 = c.gbs_sample(cov, -1, 9, 200)
    # the expected click count is sum(1 - 1/cosh r) ~ 15: the 15-click cap drops
    # many chains, the 20-click cap fewer
    assert s20["chains_capped"] < s15["chains_capped"]
    assert smp.sum(axis=1).max() <= 20


# ---------------------------------------------------------------- displaced states

def _oracle_click_prob_displaced(cov, mean, m, hist, j):
    """P(click at j | outcomes hist[0..j-1]) of a displaced state from two
    oracle probabilities with mean factors (form P)."""
    base = np.full(m, -1, np.int8)
    base[:j] = hist[:j]
    num = base.copy()
    num[j] = 1
    a = oracle.formP_mean(cov, mean, num)
    b = oracle.formP_mean(cov, mean, base)
    R = max(a.cancel_ratio, b.cancel_ratio)
    return (a.p + a.p_lo) / (b.p + b.p_lo), R


def test_displaced_replay_small_all_steps(ctx):
    """gbs_trace_displaced: every step's click probability against the oracle's
    ratio of displaced probabilities (the information-form tree with mean row
    h = K_j mu and pivot factors exp(+|w|^2 / 2))."""
    m = 7
    cov = _small_state(m, 40)
    mean = gi.random_mean(m, np.random.default_rng(41), 0.6)
    pc, un, oc, st = ctx.gbs_trace(cov, -1, 123, 0, 8, mean=mean)
    for c in range(8):
        for j in range(m):
            want, R = _oracle_click_prob_displaced(cov, mean, m, oc[c], j)
            n = int(oc[c, :j].sum()) + 1
            tol = 16 * n * U53 * max(R, 1.0) * 32 + 1e-14
            assert abs(pc[c, j] - want) <= tol * max(abs(want), 1e-300), (c, j, pc[c, j], want)
            assert oc[c, j] == (1 if un[c, j] < pc[c, j] else 0)


def test_displaced_coherent_many_clicks(ctx):
    """Coherent states through an interferometer (a product of coherent states
    beta = U alpha): P(click at j) = 1 - exp(-|beta_j|^2) whatever the
    history, up to 20 clicks (the large kernel and the LDS Schur loop above
    nine modes, with the mean row)."""
    rng = np.random.default_rng(42)
    m = 32
    U = gi.haar_unitary(m, rng)
    beta = np.sqrt(rng.uniform(0.4, 1.4, m)) * np.exp(2j * np.pi * rng.random(m))
    alpha = U.conj().T @ beta
    cov = gi.gbs_covariance(U, np.zeros(m))
    want = 1 - np.exp(-np.abs(U @ alpha) ** 2)
    with tg.Context(0) as c:
        c.set_option(tg.OPT_CHAIN_CLICKS, 20)
        pc, un, oc, st = c.gbs_trace(cov, -1, 17, 0, 12, mean=gi.coherent_mean(U @ alpha))
    deep = 0
    for ch in range(12):
        for j in np.nonzero(~np.isnan(pc[ch]))[0]:
            n = int(oc[ch, :j].sum())
            deep = max(deep, n)
            assert abs(pc[ch, j] - want[j]) <= 1e-8 * want[j], (ch, j, n, pc[ch, j], want[j])
    assert deep >= 12


def test_displaced_zero_mean_is_the_zero_mean_sampler(ctx):
    cov = _small_state(9, 43)
    a = ctx.gbs_trace(cov, 3, 21, 0, 32)
    b = ctx.gbs_trace(cov, 3, 21, 0, 32, mean=np.zeros(18))
    assert np.array_equal(a[0], b[0], equal_nan=True)
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(x, y, equal_nan=True)


def test_displaced_distribution_m5(ctx):
    m = 5
    cov = _small_state(m, 44, 0.5, 1.0)
    mean = gi.random_mean(m, np.random.default_rng(45), 0.7)
    probs = np.array([oracle.formP_mean(cov, mean, np.array([(k >> i) & 1 for i in range(m)], np.int8)).p
                      for k in range(1 << m)])
    assert abs(probs.sum() - 1) < 1e-13
    samples, st = ctx.gbs_sample(cov, -1, 8, 200000, mean=mean)
    assert st["chains_accepted"] == 200000
    assert _chi2_pvalue(samples, probs) > 1e-4
    with pytest.raises(tg.TorError) as ei:
        bad = mean.copy()
        bad[3] = np.nan
        ctx.gbs_sample(cov, -1, 8, 10, mean=bad)
    assert ei.value.status == tg.TOR_EINVAL
