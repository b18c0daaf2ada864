"""tor_batch_async_noalloc: the allocation-free form of tor_batch_async.

Its workspace is a static device array, so its results must equal those of
tor_batch_async on a zero-mean state with the same covariance (same kernels,
trees and reduction order): p, p_lo, T, T_lo, abs_sum, cancel_ratio,
rel_err_bound, n_clicks, prec_used and status bitwise; log_p and tor to the
last bits.  Two calls in a row, the second with fewer queries (the workspace
keeps the first call's contents), then a query whose tree does not fit the
workspace (TOR_ENOMEM in its result) and a pattern with a no-click mode
(TOR_EINVAL).
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


def _patterns(m, ns, seed):
    rng = np.random.default_rng(seed)
    pats = -np.ones((len(ns), m), np.int8)
    for q, n in enumerate(ns):
        pats[q, rng.choice(m, n, replace=False)] = 1
    return pats


def _same(a, b):
    for f in EXACT:
        assert getattr(a, f) == getattr(b, f), (f, getattr(a, f), getattr(b, f))
    if a.status >= 0:
        assert a.log_p == pytest.approx(b.log_p, rel=1e-14, abs=1e-300)
        assert a.tor == pytest.approx(b.tor, rel=1e-13)


def _run_noalloc(ctx, d_cov, pats, prec):
    import torch
    d_pats = torch.from_numpy(pats).to("cuda")
    rec = tg.ctypes.sizeof(tg._CResult)
    d_out = torch.zeros((pats.shape[0], rec), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    tg.batch_async_noalloc(ctx, d_cov, d_pats, d_out, prec=prec, tol=1e-10, stream=stream)
    torch.cuda.synchronize()
    return tg.results_from_device(d_out)


def _run_async(ctx, st, pats, prec):
    import torch
    d_out = ctx.batch_async(st, torch.from_numpy(pats).to("cuda"), prec=prec)
    torch.cuda.synchronize()
    return tg.results_from_device(d_out)


@pytest.mark.parametrize("prec", ["dd", "f64"])
def test_noalloc_equals_async_two_calls(ctx, prec):
    import torch
    cov = gi.state_m800(30)
    d_cov = torch.from_numpy(np.ascontiguousarray(cov)).to("cuda")
    st = ctx.state(cov)
    ns1 = [0, 1, 2, 5, 9, 10, 11, 12, 16, 20, 22] + list(np.random.default_rng(5).integers(0, 19, 53))
    first = _patterns(800, ns1, 21)
    print("noalloc first call:", prec, "nq", len(ns1), flush=True)
    got1 = _run_noalloc(ctx, d_cov, first, prec)
    want1 = _run_async(ctx, st, first, prec)
    for g, w in zip(got1, want1):
        _same(g, w)
    # second call, fewer queries: the workspace still holds the first call's plan
    ns2 = [3, 14, 8, 0, 17, 6, 24]
    second = _patterns(800, ns2, 22)
    print("noalloc second call:", prec, "nq", len(ns2), flush=True)
    got2 = _run_noalloc(ctx, d_cov, second, prec)
    want2 = _run_async(ctx, st, second, prec)
    assert len(got2) == len(ns2)
    for g, w in zip(got2, want2):
        _same(g, w)
    assert all(g.status in (tg.TOR_OK, tg.TOR_WARN_PRECISION) for g in got2)
    st.close()


def test_noalloc_admission_and_errors(ctx):
    import torch
    cov = gi.state_m800(31)
    d_cov = torch.from_numpy(np.ascontiguousarray(cov)).to("cuda")
    pats = _patterns(800, [6, 26, 7], 23)  # a 26-click double-double tree needs ~260 MB of pool
    bad = pats[2].copy()
    bad[np.nonzero(bad == -1)[0][0]] = 0  # a no-click mode: not a marginal pattern
    pats = np.stack([pats[0], pats[1], bad])
    print("noalloc admission call", flush=True)
    got = _run_noalloc(ctx, d_cov, pats, "dd")
    assert got[0].status == tg.TOR_OK
    assert got[1].status == tg.TOR_ENOMEM
    assert got[2].status == tg.TOR_EINVAL
    st = ctx.state(cov)
    want = _run_async(ctx, st, pats[:1], "dd")
    _same(got[0], want[0])
    st.close()
    # host-side argument errors
    d_pats = torch.from_numpy(pats).to("cuda")
    d_out = torch.zeros((3, tg.ctypes.sizeof(tg._CResult)), dtype=torch.uint8, device="cuda")
    L = tg.lib()
    assert L.tor_batch_async_noalloc(ctx.handle, None, 800, 3, tg.ctypes.c_void_p(d_pats.data_ptr()), 2, 1e-10,
                                     tg.ctypes.c_void_p(d_out.data_ptr()), None) == tg.TOR_EINVAL
    assert L.tor_batch_async_noalloc(ctx.handle, tg.ctypes.c_void_p(d_cov.data_ptr()), 800,
                                     tg.NOALLOC_MAX_QUERIES + 1, tg.ctypes.c_void_p(d_pats.data_ptr()), 2, 1e-10,
                                     tg.ctypes.c_void_p(d_out.data_ptr()), None) == tg.TOR_ETOOBIG
    assert L.tor_batch_async_noalloc(ctx.handle, tg.ctypes.c_void_p(d_cov.data_ptr()), 800, 3,
                                     tg.ctypes.c_void_p(d_pats.data_ptr()), 3, 1e-10,
                                     tg.ctypes.c_void_p(d_out.data_ptr()), None) == tg.TOR_EINVAL  # qd
