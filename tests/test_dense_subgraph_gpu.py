"""Dense-subgraph search with GBS (Sec. IV) on a synthetic planted-clique
graph: the encoded state's mean click number from the library equals the
oracle's, samples postselected on k clicks have k clicks, and their induced
subgraphs are denser than uniform random k-subsets (the baseline), with and
without loss."""
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


def _mean_clicks_lib(ctx, cov, n):
    single = -np.ones((n, n), np.int8)
    np.fill_diagonal(single, 1)
    st = ctx.state(cov)
    res, _ = ctx.batch(st, single, prec="dd")
    st.close()
    return sum(r.p for r in res)


def test_mean_clicks_match_oracle(ctx):
    A, _ = gi.planted_clique_graph(40, 0.5, 10, 8)
    U, lam = gi.takagi_real_symmetric(A)
    cov = gi.graph_covariance(A, 0.7 / lam.max(), eta=0.5)
    got = _mean_clicks_lib(ctx, cov, 40)
    want = 0.0
    for i in range(40):
        pat = -np.ones(40, np.int8)
        pat[i] = 1
        o = oracle.formS(cov, pat)
        want += o.p + o.p_lo
    assert got == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("eta", [1.0, 0.5])
def test_gbs_finds_denser_subgraphs_than_uniform(ctx, eta):
    n, k = 40, 6
    A, clique = gi.planted_clique_graph(n, 0.5, 10, 8)
    c = gi.calibrate_scale(A, 6.0, lambda cov: _mean_clicks_lib(ctx, cov, n), iters=40)
    cov = gi.graph_covariance(A, c, eta)
    samples, st = ctx.gbs_sample(cov, k, 123, 300)
    assert samples.shape == (300, n) and (samples.sum(axis=1) == k).all()
    dens = np.array([gi.subgraph_density(A, np.nonzero(s)[0]) for s in samples])
    rng = np.random.default_rng(5)
    uni = np.array([gi.subgraph_density(A, rng.choice(n, k, replace=False)) for _ in range(3000)])
    # the uniform mean is the graph density (~0.5 plus the clique's share)
    assert dens.mean() > uni.mean() + 0.05, (dens.mean(), uni.mean())
    assert dens.max() == 1.0
