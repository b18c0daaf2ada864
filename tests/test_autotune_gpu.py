"""Autotuner: per-n task sizes are chosen, cached, reloaded, and do not change
results beyond rounding (and never make a query depend on its batch)."""
import json

import numpy as np
import pytest

import gbs_inputs as gi
import paper_1810_00900_amd as tg

pytestmark = pytest.mark.gpu


def test_autotune_cache_roundtrip(tmp_path):
    path = tmp_path / "tune.json"
    cov = gi.state_m800(50)
    with tg.Context(0) as ctx:
        base = {n: ctx.probability(cov, gi.config5_pattern(n), prec="dd") for n in (10, 12, 14)}
        ctx.autotune("dd", 10, 14, path)
        table = {n: ctx.tuning("dd", n) for n in range(10, 15)}
        assert all(6 <= j <= 11 for j in table.values())
        assert ctx.tuning("dd", 5) == 5            # small trees use one task
        for n, r0 in base.items():
            r = ctx.probability(cov, gi.config5_pattern(n), prec="dd")
            assert abs((r.p + r.p_lo) - (r0.p + r0.p_lo)) <= 1e-13 * abs(r0.p)
        st = ctx.state(cov)
        pats = np.stack([gi.config5_pattern(n) for n in (14, 10, 12)])
        res, _ = ctx.batch(st, pats, prec="dd")
        for p, r in zip(pats, res):
            a = ctx.probability(cov, p, prec="dd")
            assert (r.p, r.p_lo) == (a.p, a.p_lo)
    d = json.load(open(path))
    assert d["arch"].startswith("gfx950")
    assert {f"dd:{n}" for n in range(10, 15)} <= set(d["task_modes"])
    with tg.Context(0) as ctx2:
        ctx2.load_tuning(path)
        assert {n: ctx2.tuning("dd", n) for n in range(10, 15)} == table


def test_autotune_rejects_bad_args():
    with tg.Context(0) as ctx:
        with pytest.raises(tg.TorError):
            ctx.autotune("auto", 10, 12)
        with pytest.raises(tg.TorError):
            ctx.autotune("dd", 12, 10)
