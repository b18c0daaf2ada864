"""Chain-rule sampler with double-double terms (TOR_OPT_CHAIN_PREC) and the
per-step cancellation ratio and error bound of gbs_trace_steps.

Each step's coin has bias P(click) = 1 - X0 / X1 (Sec. II: the ratio of the
probabilities with and without the new click), evaluated from a split subset
sum whose cancellation grows with the clicks so far.  With binary64 terms its
error is about 16 k u R; with double-double terms (and K_j in double-double
words) the binary64 rounding of the final ratio dominates.

* config 2 (m = 100, r = 0.6, postselected on 12 clicks): replayed steps with
  8..12 clicks so far match the oracle's ratio of exact probabilities to
  1e-10 relative, and the reported bound covers the observed error;
* the binary64 chains' reported bound covers their observed error on the same
  steps, and the two precisions draw the same coins wherever |u - P(click)|
  exceeds the binary64 bound;
* small states, every step, zero-mean and displaced: double-double steps match
  the oracle to 1e-13;
* samples of a 5-mode state follow the exact distribution (chi-square).
"""
import numpy as np
import pytest

import gbs_inputs as gi
import oracle
import paper_1810_00900_amd as tg
from test_sampler_gpu import (_chi2_pvalue, _oracle_click_prob, _oracle_click_prob_displaced,
                              _small_state)

pytestmark = pytest.mark.gpu


def _trace(cov, n_post, seed, nchains, prec, mean=None):
    with tg.Context(0) as c:
        c.set_option(tg.OPT_CHAIN_PREC, prec)
        return c.gbs_trace(cov, n_post, seed, 0, nchains, mean=mean, steps=True)


@pytest.fixture(scope="module")
def config2():
    cov = gi.state_config2()
    dd = _trace(cov, 12, 2, 24, tg.PREC_DD)
    f64 = _trace(cov, 12, 2, 24, tg.PREC_F64)
    # steps with 8..12 clicks so far, up to three per click count
    picks, seen = [], {}
    pc, _, oc = dd[0], dd[1], dd[2]
    for c in range(pc.shape[0]):
        for j in np.nonzero(~np.isnan(pc[c]))[0]:
            k = int(oc[c, :j].sum())
            if 8 <= k <= 12 and seen.get(k, 0) < 3:
                seen[k] = seen.get(k, 0) + 1
                picks.append((c, int(j), k))
    want = {(c, j): _oracle_click_prob(cov, 100, oc[c], j) for c, j, _ in picks}
    return cov, dd, f64, picks, want


def test_dd_replay_config2_clicks_8_to_12(config2):
    cov, dd, _, picks, want = config2
    pc, _, oc, _, R, B = dd
    assert {k for _, _, k in picks} == {8, 9, 10, 11, 12}
    worst = 0.0
    for c, j, k in picks:
        w, Ro = want[(c, j)]
        err = abs(pc[c, j] - w)
        print(f"dd chain {c} mode {j} clicks {k}: p {pc[c, j]:.6e} rel err {err / w:.2e} "
              f"bound {B[c, j]:.2e} R {R[c, j]:.3e} (oracle R {Ro:.3e})", flush=True)
        assert err <= 1e-10 * w, (c, j, k, err / w)
        assert err <= B[c, j], (c, j, k, err, B[c, j])
        assert B[c, j] <= 1e-12 * max(w, 1e-3)
        assert R[c, j] >= 1.0
        worst = max(worst, err / w)
    print("largest relative error", worst, flush=True)


def test_f64_bound_covers_error_and_coins_agree(config2):
    cov, dd, f64, picks, want = config2
    pc, un, oc, st, R, B = f64
    # the chains of the two precisions agree while no coin falls within the
    # binary64 bound (every coin is the same Philox draw)
    for c in range(pc.shape[0]):
        for j in range(pc.shape[1]):
            if np.isnan(pc[c, j]) or np.isnan(dd[0][c, j]):
                break
            assert abs(pc[c, j] - dd[0][c, j]) <= B[c, j] + dd[5][c, j], (c, j)
            if abs(un[c, j] - pc[c, j]) > B[c, j]:
                assert oc[c, j] == dd[2][c, j]
            else:
                break
    for c, j, k in picks:
        if np.isnan(pc[c, j]) or not np.array_equal(oc[c, :j], dd[2][c, :j]):
            continue  # a coin within the bound took this chain elsewhere
        w, _ = want[(c, j)]
        assert abs(pc[c, j] - w) <= B[c, j], (c, j, k, abs(pc[c, j] - w), B[c, j])


def test_dd_small_states_every_step():
    m = 7
    cov = _small_state(m, 2)
    pc, un, oc, st, R, B = _trace(cov, -1, 99, 6, tg.PREC_DD)
    for c in range(6):
        for j in range(m):
            w, _ = _oracle_click_prob(cov, m, oc[c], j)
            assert abs(pc[c, j] - w) <= 1e-13 * max(w, 1e-300) + 1e-16, (c, j, pc[c, j], w)
            assert abs(pc[c, j] - w) <= B[c, j]
            assert oc[c, j] == (1 if un[c, j] < pc[c, j] else 0)
    cov = _small_state(m, 40)
    mean = gi.random_mean(m, np.random.default_rng(41), 0.6)
    pc, un, oc, st, R, B = _trace(cov, -1, 123, 8, tg.PREC_DD, mean=mean)
    for c in range(8):
        for j in range(m):
            w, _ = _oracle_click_prob_displaced(cov, mean, m, oc[c], j)
            assert abs(pc[c, j] - w) <= 1e-13 * max(w, 1e-300) + 1e-16, (c, j, pc[c, j], w)


def test_dd_distribution_m5():
    m = 5
    cov = _small_state(m, 3, 0.5, 1.2)
    probs = np.array([oracle.formP(cov, np.array([(k >> i) & 1 for i in range(m)], np.int8)).p
                      for k in range(1 << m)])
    with tg.Context(0) as c:
        c.set_option(tg.OPT_CHAIN_PREC, tg.PREC_DD)
        samples, st = c.gbs_sample(cov, -1, 7, 100000)
    assert st["chains_accepted"] == 100000
    assert _chi2_pvalue(samples, probs) > 1e-4


def test_chain_prec_option_checked():
    with tg.Context(0) as c:
        with pytest.raises(tg.TorError):
            c.set_option(tg.OPT_CHAIN_PREC, tg.PREC_QD)
