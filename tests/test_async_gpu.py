"""tor_batch_async: patterns and results in device memory, plan made on the
device, stream-ordered.

The device planner builds the same trees, task sizes and reduction order as
the host planner, so p, p_lo, T, T_lo and abs_sum must equal tor_batch's
bitwise (log_p and tor go through device log/exp: last-bit tolerance).
"""
import numpy as np
import pytest

import gbs_inputs as gi
import paper_1810_00900_amd as tg

pytestmark = pytest.mark.gpu

EXACT = ("p", "p_lo", "T", "T_lo", "abs_sum", "cancel_ratio", "rel_err_bound", "n_clicks", "prec_used", "status")


@pytest.fixture(scope="module")
def ctx():
    c = tg.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def st800(ctx):
    cov = gi.state_m800(30)
    st = ctx.state(cov)
    yield cov, st
    st.close()


def _patterns(m, ns, seed):
    rng = np.random.default_rng(seed)
    pats = -np.ones((len(ns), m), np.int8)
    for q, n in enumerate(ns):
        pats[q, rng.choice(m, n, replace=False)] = 1
    return pats


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _same(a, b):
    for f in EXACT:
        assert getattr(a, f) == getattr(b, f), (f, getattr(a, f), getattr(b, f))
    if a.status >= 0:
        assert a.log_p == pytest.approx(b.log_p, rel=1e-14, abs=1e-300)
        assert a.tor == pytest.approx(b.tor, rel=1e-13)


@pytest.mark.parametrize("prec", ["dd", "f64"])
def test_async_equals_batch(ctx, st800, prec):
    import torch
    cov, st = st800
    ns = [0, 1, 2, 5, 9, 10, 11, 12, 14, 16, 18, 20] + list(np.random.default_rng(3).integers(0, 21, 36))
    pats = _patterns(400 * 2, ns, 11)
    want, _ = ctx.batch(st, pats, prec=prec)
    d_out = ctx.batch_async(st, _dev(pats), prec=prec)
    torch.cuda.synchronize()
    got = tg.results_from_device(d_out)
    assert len(got) == len(ns)
    for g, w in zip(got, want):
        _same(g, w)


@pytest.mark.parametrize("prec", ["dd", "f64"])
def test_async_displaced_equals_batch(ctx, prec):
    """A displaced state (800 modes, mean 0.3 x N(0, 1) per quadrature): the
    device planner lays out matrices with the mean row, and the results equal
    tor_batch's on the same state bitwise, error bound included."""
    import torch
    cov = gi.state_m800(30)
    mean = gi.random_mean(800, np.random.default_rng(53), 0.3)
    st = ctx.state(cov, mean=mean)
    ns = [0, 1, 2, 9, 10, 11, 12, 16, 20] + list(np.random.default_rng(4).integers(0, 21, 15))
    pats = _patterns(800, ns, 12)
    want, _ = ctx.batch(st, pats, prec=prec)
    d_out = ctx.batch_async(st, _dev(pats), prec=prec)
    torch.cuda.synchronize()
    got = tg.results_from_device(d_out)
    assert len(got) == len(ns)
    for g, w in zip(got, want):
        _same(g, w)
    # the mean matters: the zero-mean state gives other probabilities
    st0 = ctx.state(cov)
    d0 = ctx.batch_async(st0, _dev(pats), prec=prec)
    torch.cuda.synchronize()
    z = tg.results_from_device(d0)
    assert all(a.p != b.p for a, b, n in zip(z, got, ns) if n > 0)
    st0.close()
    st.close()


def test_async_statuses_in_a_mixed_batch(ctx, st800):
    import torch
    cov, st = st800
    pats = _patterns(800, [6, 8, 7, 33, 12], 5)
    pats[1, 17] = 0                 # a no-click mode: host planning only
    pats[2, 3] = 2                  # not a pattern value
    out = ctx.batch_async(st, _dev(pats), prec="dd")  # on the context's own stream
    torch.cuda.synchronize()
    got = tg.results_from_device(out)
    assert [r.status for r in got][1:4] == [tg.TOR_EINVAL, tg.TOR_EINVAL, tg.TOR_ETOOBIG]
    want, _ = ctx.batch(st, pats[[0, 4]], prec="dd")
    _same(got[0], want[0])
    _same(got[4], want[1])


def test_async_admission_by_pool(st800):
    """A 1 MiB pool (65536 double-doubles) holds four n = 16 trees of
    16377 entries each; the later queries get TOR_ENOMEM, the first four equal
    tor_batch."""
    import torch
    cov, _ = st800
    with tg.Context(0) as c:
        st = c.state(cov)
        c.set_option(tg.OPT_TASK_MODES, 10)  # the tree sizes below (not the tuning table's choice)
        c.set_option(tg.OPT_ASYNC_POOL, 1 << 20)
        pats = _patterns(800, [16] * 7, 9)
        out = c.batch_async(st, _dev(pats), prec="dd")
        torch.cuda.synchronize()
        got = tg.results_from_device(out)
        assert [r.status for r in got] == [0, 0, 0, 0, tg.TOR_ENOMEM, tg.TOR_ENOMEM, tg.TOR_ENOMEM]
        want, _ = c.batch(st, pats[:4], prec="dd")
        for g, w in zip(got[:4], want):
            _same(g, w)
        st.close()


def test_async_on_a_torch_stream_and_workspace_reuse(ctx, st800):
    """Patterns produced on a side stream, the batch enqueued on the same
    stream, twice in a row (the second batch smaller) before any wait."""
    import torch
    cov, st = st800
    s = torch.cuda.Stream()
    p1 = _patterns(800, [10, 17, 3, 20, 12, 9], 21)
    p2 = _patterns(800, [15, 4], 22)
    h1 = torch.from_numpy(p1).pin_memory()
    h2 = torch.from_numpy(p2).pin_memory()
    with torch.cuda.stream(s):
        d1 = h1.to("cuda", non_blocking=True)
        o1 = ctx.batch_async(st, d1, prec="dd", stream=s)
        r1 = o1.to("cpu", non_blocking=True)
        d2 = h2.to("cuda", non_blocking=True)
        o2 = ctx.batch_async(st, d2, prec="dd", stream=s)
    s.synchronize()
    g1 = tg.results_from_device(r1)
    g2 = tg.results_from_device(o2)
    w1, _ = ctx.batch(st, p1, prec="dd")
    w2, _ = ctx.batch(st, p2, prec="dd")
    for g, w in zip(g1 + g2, w1 + w2):
        _same(g, w)


def test_async_empty_and_bad_arguments(ctx, st800):
    import torch
    cov, st = st800
    out = ctx.batch_async(st, torch.empty((0, 800), dtype=torch.int8, device="cuda"))
    assert out.shape[0] == 0
    with pytest.raises(ValueError):
        ctx.batch_async(st, torch.zeros((2, 799), dtype=torch.int8, device="cuda"))
    import ctypes
    d = torch.zeros((2, 800), dtype=torch.int8, device="cuda")
    o = torch.empty((2, 96), dtype=torch.uint8, device="cuda")
    L = tg.lib()
    assert L.tor_batch_async(ctx.handle, st.handle, 2, ctypes.c_void_p(d.data_ptr()), 7, 1e-10,
                             ctypes.c_void_p(o.data_ptr()), None) == tg.TOR_EINVAL
    assert L.tor_batch_async(ctx.handle, st.handle, 2, None, 2, 1e-10, ctypes.c_void_p(o.data_ptr()),
                             None) == tg.TOR_EINVAL
    assert L.tor_batch_async(ctx.handle, st.handle, -1, ctypes.c_void_p(d.data_ptr()), 2, 1e-10,
                             ctypes.c_void_p(o.data_ptr()), None) == tg.TOR_EINVAL
