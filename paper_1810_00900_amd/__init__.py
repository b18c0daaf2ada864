"""Python binding of libtorgbs (include/tor.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
numpy arrays to pointers, calls the C ABI and turns results into dataclasses.
PyTorch is used only to hand a stream (``torch.cuda.Stream``) to a context.

The library must have been built (``python -m paper_1810_00900_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtorgbs.so")

TOR_OK = 0
TOR_WARN_PRECISION = 1
TOR_EINVAL = -1
TOR_ENOTPD = -2
TOR_ETOOBIG = -3
TOR_ENOMEM = -4
TOR_EDEVICE = -5
TOR_EAGAIN = -6
FUSED_MAX_TASKS = 4096  # tor.h TOR_FUSED_MAX_TASKS
PS_SLOTS = 4096  # TOR_PS_SLOTS: request slots of the persistent loop's ring

PREC_AUTO, PREC_F64, PREC_DD, PREC_QD = 0, 1, 2, 3
_PREC = {"auto": PREC_AUTO, "f64": PREC_F64, "dd": PREC_DD, "qd": PREC_QD,
         PREC_AUTO: PREC_AUTO, PREC_F64: PREC_F64, PREC_DD: PREC_DD, PREC_QD: PREC_QD}

(OPT_TIMING, OPT_TASK_MODES, OPT_WAVE_GRID, OPT_MEM_BUDGET, OPT_ASYNC_POOL, OPT_CHAIN_CLICKS, OPT_COND_BLOCK,
 OPT_FUSED, OPT_CHAIN_PREC) = (0, 1, 2, 3, 4, 5, 6, 7, 8)

_STATUS_NAMES = {0: "TOR_OK", 1: "TOR_WARN_PRECISION", -1: "TOR_EINVAL", -2: "TOR_ENOTPD",
                 -3: "TOR_ETOOBIG", -4: "TOR_ENOMEM", -5: "TOR_EDEVICE", -6: "TOR_EAGAIN"}


class TorError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _CResult(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double), ("p_lo", ctypes.c_double), ("log_p", ctypes.c_double),
                ("tor", ctypes.c_double), ("T", ctypes.c_double), ("T_lo", ctypes.c_double),
                ("abs_sum", ctypes.c_double), ("cancel_ratio", ctypes.c_double),
                ("rel_err_bound", ctypes.c_double), ("log_pvac_n", ctypes.c_double),
                ("n_clicks", ctypes.c_int32), ("prec_used", ctypes.c_int32),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _CStats(ctypes.Structure):
    _fields_ = [("wave_ms", ctypes.c_double), ("expand_ms", ctypes.c_double),
                ("reduce_ms", ctypes.c_double), ("wave_launches", ctypes.c_int64),
                ("expand_launches", ctypes.c_int64), ("reduce_launches", ctypes.c_int64),
                ("subsets", ctypes.c_double), ("condition_launches", ctypes.c_int64),
                ("fused_launches", ctypes.c_int64)]


class _CGbsStats(ctypes.Structure):
    _fields_ = [("chains_started", ctypes.c_int64), ("chains_accepted", ctypes.c_int64),
                ("chains_evaluated", ctypes.c_int64), ("chains_capped", ctypes.c_int64),
                ("seconds", ctypes.c_double), ("subsets", ctypes.c_double)]


class _CServerOpts(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("max_pending", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_size_t), ("prec", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_batch", ctypes.c_int32)]


class _CServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("max_batch_seen", ctypes.c_int64), ("pending", ctypes.c_int64)]


class _CPServerOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("mem_budget_bytes", ctypes.c_size_t),
                ("chain_buffer_bytes", ctypes.c_size_t), ("grid", ctypes.c_int32), ("idle_ms", ctypes.c_int32)]


class _CPServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("units", ctypes.c_int64), ("launches", ctypes.c_int64), ("device_cursor", ctypes.c_int64),
                ("device_published", ctypes.c_int64), ("running", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("workgroups_started", ctypes.c_int32), ("workgroups_peak", ctypes.c_int32)]


@dataclass
class Result:
    p: float
    p_lo: float
    log_p: float
    tor: float
    T: float
    T_lo: float
    abs_sum: float
    cancel_ratio: float
    rel_err_bound: float
    log_pvac_n: float
    n_clicks: int
    prec_used: int
    status: int

    @classmethod
    def _from(cls, r: _CResult) -> "Result":
        return cls(*(getattr(r, f) for f, _ in _CResult._fields_[:-1]))


_lib = None


def lib():
    """Load libtorgbs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1810_00900_amd.build")
    # PyTorch ships its own HIP runtime (same soname, libamdhip64.so.7).  Load
    # torch first so that the library binds to that already-loaded runtime and
    # one process holds a single HIP runtime: torch's streams and device
    # tensors are then valid in the library, and torch can still initialise.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    i8p = ctypes.POINTER(ctypes.c_int8)
    sig = {
        "tor_ctx_create": ([ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int32),
        "tor_ctx_destroy": ([vp], None),
        "tor_ctx_set_stream": ([vp, vp], ctypes.c_int32),
        "tor_ctx_set_option": ([vp, ctypes.c_int, ctypes.c_int64], ctypes.c_int32),
        "tor_ctx_get_stats": ([vp, ctypes.POINTER(_CStats)], ctypes.c_int32),
        "tor_ctx_reset_stats": ([vp], ctypes.c_int32),
        "tor_last_error": ([], ctypes.c_char_p),
        "tor_probability": ([vp, dp, ctypes.c_int32, i8p, ctypes.c_int, ctypes.c_double,
                             ctypes.POINTER(_CResult)], ctypes.c_int32),
        "tor_probability_displaced": ([vp, dp, dp, ctypes.c_int32, i8p, ctypes.c_int, ctypes.c_double,
                                       ctypes.POINTER(_CResult)], ctypes.c_int32),
        "tor_subset_sum": ([vp, dp, dp, ctypes.c_int32, ctypes.c_int, ctypes.c_double,
                            ctypes.POINTER(_CResult)], ctypes.c_int32),
        "tor_state_create": ([vp, dp, ctypes.c_int32, ctypes.POINTER(vp)], ctypes.c_int32),
        "tor_state_create_displaced": ([vp, dp, dp, ctypes.c_int32, ctypes.POINTER(vp)], ctypes.c_int32),
        "tor_state_destroy": ([vp], None),
        "tor_state_invert": ([vp, ctypes.c_int], ctypes.c_int32),
        "tor_batch": ([vp, vp, ctypes.c_int32, i8p, ctypes.c_int, ctypes.c_double,
                       ctypes.POINTER(_CResult)], ctypes.c_int32),
        "tor_batch_displaced": ([vp, vp, dp, ctypes.c_int32, i8p, ctypes.c_int, ctypes.c_double,
                                 ctypes.POINTER(_CResult)], ctypes.c_int32),
        "tor_batch_async": ([vp, vp, ctypes.c_int32, vp, ctypes.c_int, ctypes.c_double, vp, vp], ctypes.c_int32),
        "tor_batch_async_noalloc": ([vp, vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int, ctypes.c_double, vp,
                                     vp], ctypes.c_int32),
        "tor_server_start": ([vp, ctypes.POINTER(_CServerOpts), ctypes.POINTER(vp)], ctypes.c_int32),
        "tor_pserver_start": ([vp, ctypes.POINTER(_CPServerOpts), ctypes.POINTER(vp)], ctypes.c_int32),
        "tor_pserver_submit": ([vp, vp, i8p, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
        "tor_pserver_submit_chains": ([vp, vp, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
        "tor_pserver_poll": ([vp, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(_CResult), dp], ctypes.c_int32),
        "tor_pserver_poll_chains": ([vp, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8), i8p, dp],
                                    ctypes.c_int32),
        "tor_pserver_get_stats": ([vp, ctypes.POINTER(_CPServerStats)], ctypes.c_int32),
        "tor_pserver_autotune": ([vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p], ctypes.c_int32),
        "tor_pserver_stop": ([vp], ctypes.c_int32),
        "tor_submit": ([vp, vp, i8p, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
        "tor_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(_CResult), dp], ctypes.c_int32),
        "tor_wait": ([vp, ctypes.c_uint64, ctypes.POINTER(_CResult), dp], ctypes.c_int32),
        "tor_server_get_stats": ([vp, ctypes.POINTER(_CServerStats)], ctypes.c_int32),
        "tor_server_stop": ([vp], ctypes.c_int32),
        "tor_autotune": ([vp, ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p], ctypes.c_int32),
        "tor_load_tuning": ([vp, ctypes.c_char_p], ctypes.c_int32),
        "tor_get_tuning": ([vp, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int32),
        "gbs_sample": ([vp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                        ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(_CGbsStats)], ctypes.c_int32),
        "gbs_chain_fixed": ([vp, dp, ctypes.c_int32, i8p, ctypes.c_int, ctypes.c_double, dp,
                             ctypes.POINTER(_CResult)], ctypes.c_int32),
        "gbs_chain_fixed_displaced": ([vp, dp, dp, ctypes.c_int32, i8p, ctypes.c_int, ctypes.c_double, dp,
                                       ctypes.POINTER(_CResult)], ctypes.c_int32),
        "gbs_trace": ([vp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                       dp, dp, ctypes.POINTER(ctypes.c_uint8), i8p], ctypes.c_int32),
        "gbs_sample_displaced": ([vp, dp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(_CGbsStats)], ctypes.c_int32),
        "gbs_trace_displaced": ([vp, dp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                 ctypes.c_int32, dp, dp, ctypes.POINTER(ctypes.c_uint8), i8p], ctypes.c_int32),
        "gbs_trace_steps": ([vp, dp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                             ctypes.c_int32, dp, dp, ctypes.POINTER(ctypes.c_uint8), i8p, dp, dp], ctypes.c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def last_error() -> str:
    return lib().tor_last_error().decode()


def _check(status: int, allow_warn: bool = True) -> int:
    if status < 0 or (status == TOR_WARN_PRECISION and not allow_warn):
        raise TorError(status, last_error())
    return status


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int8)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i8ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))


class Context:
    """A library context on one HIP device (tor_ctx)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().tor_ctx_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = device
        self._stream_ref = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tor_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream=None):
        """Run on a torch.cuda.Stream (or a raw hipStream_t int); None = own stream."""
        raw = None
        if stream is not None:
            raw = getattr(stream, "cuda_stream", stream)
        self._stream_ref = stream
        _check(lib().tor_ctx_set_stream(self._h, ctypes.c_void_p(raw)))

    def set_option(self, opt: int, value: int):
        _check(lib().tor_ctx_set_option(self._h, int(opt), int(value)))

    def stats(self) -> dict:
        s = _CStats()
        _check(lib().tor_ctx_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _CStats._fields_}

    def reset_stats(self):
        _check(lib().tor_ctx_reset_stats(self._h))

    def probability(self, cov, pattern, prec="auto", tol: float = 1e-10) -> Result:
        cov = _f64(cov)
        pattern = _i8(pattern)
        m = pattern.shape[0]
        if cov.shape != (2 * m, 2 * m):
            raise ValueError("cov must be 2m x 2m for a pattern of length m")
        r = _CResult()
        _check(lib().tor_probability(self._h, _dptr(cov), m, _i8ptr(pattern), _PREC[prec], float(tol),
                                     ctypes.byref(r)))
        return Result._from(r)

    def probability_displaced(self, cov, mean, pattern, prec="auto", tol: float = 1e-10) -> Result:
        """Click-pattern probability of a displaced Gaussian state (mean: 2m
        entries, hbar = 1, interleaved like cov) -- tor_probability_displaced."""
        cov = _f64(cov)
        mean = _f64(mean)
        pattern = _i8(pattern)
        m = pattern.shape[0]
        if cov.shape != (2 * m, 2 * m):
            raise ValueError("cov must be 2m x 2m for a pattern of length m")
        if mean.shape != (2 * m,):
            raise ValueError("mean must have 2m entries")
        r = _CResult()
        _check(lib().tor_probability_displaced(self._h, _dptr(cov), _dptr(mean), m, _i8ptr(pattern), _PREC[prec],
                                               float(tol), ctypes.byref(r)))
        return Result._from(r)

    def subset_sum(self, sigma, sigma_lo=None, prec="dd", tol: float = 1e-10) -> Result:
        sigma = _f64(sigma)
        n = sigma.shape[0] // 2
        lo = None if sigma_lo is None else _f64(sigma_lo)
        r = _CResult()
        _check(lib().tor_subset_sum(self._h, _dptr(sigma), None if lo is None else _dptr(lo), n, _PREC[prec],
                                    float(tol), ctypes.byref(r)))
        return Result._from(r)

    def autotune(self, prec="dd", n_lo=10, n_hi=24, cache_path=None):
        """Time the wave-tier task sizes per n and keep the fastest (tor_autotune)."""
        _check(lib().tor_autotune(self._h, _PREC[prec], int(n_lo), int(n_hi),
                                  None if cache_path is None else str(cache_path).encode()))

    def load_tuning(self, cache_path):
        _check(lib().tor_load_tuning(self._h, str(cache_path).encode()))

    def tuning(self, prec, n) -> int:
        v = ctypes.c_int32()
        _check(lib().tor_get_tuning(self._h, _PREC[prec], int(n), ctypes.byref(v)))
        return v.value

    def chain_fixed(self, cov, outcomes, prec="dd", tol: float = 1e-10, mean=None):
        """The paper's fixed-outcome benchmark chain (gbs_chain_fixed, or
        gbs_chain_fixed_displaced with a mean vector of 2m entries): modes
        measured from the last down; returns (Result for the whole pattern,
        step probabilities per mode, 1 for unmeasured modes)."""
        cov = _f64(cov)
        outcomes = _i8(outcomes)
        m = cov.shape[0] // 2
        if outcomes.shape != (m,):
            raise ValueError("outcomes must have m entries")
        steps = np.empty(m, np.float64)
        out = _CResult()
        if mean is None:
            _check(lib().gbs_chain_fixed(self._h, _dptr(cov), m, _i8ptr(outcomes), _PREC[prec], float(tol),
                                         _dptr(steps), ctypes.byref(out)))
        else:
            mean = _f64(mean)
            if mean.shape != (2 * m,):
                raise ValueError("mean must have 2m entries")
            _check(lib().gbs_chain_fixed_displaced(self._h, _dptr(cov), _dptr(mean), m, _i8ptr(outcomes),
                                                   _PREC[prec], float(tol), _dptr(steps), ctypes.byref(out)))
        return Result._from(out), steps

    def gbs_sample(self, cov, n_post: int, seed: int, n_samples: int, mean=None):
        """Exact chain-rule threshold samples (gbs_sample, or
        gbs_sample_displaced with a mean vector of 2m entries); returns
        (samples uint8[n_samples, m], stats dict)."""
        cov = _f64(cov)
        m = cov.shape[0] // 2
        out = np.zeros((n_samples, m), dtype=np.uint8)
        st = _CGbsStats()
        op = out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        if mean is None:
            _check(lib().gbs_sample(self._h, _dptr(cov), m, int(n_post), int(seed) & (2**64 - 1), int(n_samples),
                                    op, ctypes.byref(st)))
        else:
            mean = _f64(mean)
            if mean.shape != (2 * m,):
                raise ValueError("mean must have 2m entries")
            _check(lib().gbs_sample_displaced(self._h, _dptr(cov), _dptr(mean), m, int(n_post),
                                              int(seed) & (2**64 - 1), int(n_samples), op, ctypes.byref(st)))
        return out, {f: getattr(st, f) for f, _ in _CGbsStats._fields_}

    def gbs_trace(self, cov, n_post: int, seed: int, chain_begin: int, nchains: int, mean=None,
                  steps: bool = False):
        """Replay chains of gbs_sample (gbs_trace_displaced with a mean):
        (p_click, uniform, outcome, status); with steps=True also the per-step
        cancellation ratio and absolute error bound of p_click
        (gbs_trace_steps)."""
        cov = _f64(cov)
        m = cov.shape[0] // 2
        pc = np.zeros((nchains, m))
        un = np.zeros((nchains, m))
        oc = np.zeros((nchains, m), dtype=np.uint8)
        stt = np.zeros(nchains, dtype=np.int8)
        op = oc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        if steps:
            rr = np.zeros((nchains, m))
            bb = np.zeros((nchains, m))
            if mean is not None:
                mean = _f64(mean)
                if mean.shape != (2 * m,):
                    raise ValueError("mean must have 2m entries")
            _check(lib().gbs_trace_steps(self._h, _dptr(cov), None if mean is None else _dptr(mean), m,
                                         int(n_post), int(seed) & (2**64 - 1), int(chain_begin), int(nchains),
                                         _dptr(pc), _dptr(un), op, _i8ptr(stt), _dptr(rr), _dptr(bb)))
            return pc, un, oc, stt, rr, bb
        if mean is None:
            _check(lib().gbs_trace(self._h, _dptr(cov), m, int(n_post), int(seed) & (2**64 - 1), int(chain_begin),
                                   int(nchains), _dptr(pc), _dptr(un), op, _i8ptr(stt)))
        else:
            mean = _f64(mean)
            if mean.shape != (2 * m,):
                raise ValueError("mean must have 2m entries")
            _check(lib().gbs_trace_displaced(self._h, _dptr(cov), _dptr(mean), m, int(n_post),
                                             int(seed) & (2**64 - 1), int(chain_begin), int(nchains), _dptr(pc),
                                             _dptr(un), op, _i8ptr(stt)))
        return pc, un, oc, stt

    def state(self, cov, mean=None) -> "State":
        """A state kept by the library; with a mean vector a displaced state."""
        return State(self, cov, mean)

    def batch(self, state: "State", patterns, prec="auto", tol: float = 1e-10):
        patterns = _i8(patterns)
        if patterns.ndim != 2 or patterns.shape[1] != state.m:
            raise ValueError("patterns must be nq x m")
        nq = patterns.shape[0]
        out = (_CResult * max(nq, 1))()
        st = lib().tor_batch(self._h, state.handle, nq, _i8ptr(patterns), _PREC[prec], float(tol), out)
        res = [Result._from(out[i]) for i in range(nq)]
        if st < 0 and all(r.status < 0 for r in res):
            raise TorError(st, last_error())
        return res, st

    def batch_displaced(self, state: "State", mean, patterns, prec="auto", tol: float = 1e-10):
        """tor_batch_displaced: nq patterns on the state's covariance with the
        given mean (2m entries); returns (results, status)."""
        patterns = _i8(patterns)
        mean = _f64(mean)
        if patterns.ndim != 2 or patterns.shape[1] != state.m:
            raise ValueError("patterns must be nq x m")
        if mean.shape != (2 * state.m,):
            raise ValueError("mean must have 2m entries")
        nq = patterns.shape[0]
        out = (_CResult * max(nq, 1))()
        st = lib().tor_batch_displaced(self._h, state.handle, _dptr(mean), nq, _i8ptr(patterns), _PREC[prec],
                                       float(tol), out)
        res = [Result._from(out[i]) for i in range(nq)]
        if st < 0 and all(r.status < 0 for r in res):
            raise TorError(st, last_error())
        return res, st

    def batch_async(self, state: "State", d_patterns, prec="dd", tol: float = 1e-10, d_out=None, stream=None):
        """Stream-ordered batch (tor_batch_async).  d_patterns: contiguous
        int8 device tensor, nq x m.  Returns d_out, a uint8 device tensor of
        nq result records, written when `stream` (a torch.cuda.Stream, a raw
        hipStream_t int, or None for the context's stream) reaches the call;
        decode it with results_from_device() after synchronising."""
        import torch
        if d_patterns.dtype != torch.int8 or not d_patterns.is_cuda or not d_patterns.is_contiguous():
            raise ValueError("d_patterns must be a contiguous int8 device tensor")
        if d_patterns.ndim != 2 or d_patterns.shape[1] != state.m:
            raise ValueError("d_patterns must be nq x m")
        nq = int(d_patterns.shape[0])
        rec = ctypes.sizeof(_CResult)
        if d_out is None:
            d_out = torch.empty((nq, rec), dtype=torch.uint8, device=d_patterns.device)
        elif d_out.dtype != torch.uint8 or not d_out.is_cuda or d_out.numel() < nq * rec or not d_out.is_contiguous():
            raise ValueError("d_out must be a contiguous uint8 device tensor of nq result records")
        raw = None if stream is None else getattr(stream, "cuda_stream", stream)
        _check(lib().tor_batch_async(self._h, state.handle, nq, ctypes.c_void_p(d_patterns.data_ptr()),
                                     _PREC[prec], float(tol), ctypes.c_void_p(d_out.data_ptr()),
                                     ctypes.c_void_p(raw)))
        return d_out


NOALLOC_MAX_QUERIES = 4096


def batch_async_noalloc(ctx: "Context", d_cov, d_patterns, d_out, prec="dd", tol: float = 1e-10, stream=None):
    """tor_batch_async_noalloc: marginal patterns of the zero-mean covariance
    d_cov (contiguous float64 device tensor, 2m x 2m), results into d_out (a
    contiguous uint8 device tensor of nq result records, caller-allocated: the
    call itself allocates nothing).  Stream-ordered like Context.batch_async."""
    import torch
    if d_cov.dtype != torch.float64 or not d_cov.is_cuda or not d_cov.is_contiguous():
        raise ValueError("d_cov must be a contiguous float64 device tensor")
    if d_patterns.dtype != torch.int8 or not d_patterns.is_cuda or not d_patterns.is_contiguous():
        raise ValueError("d_patterns must be a contiguous int8 device tensor")
    m = int(d_patterns.shape[1])
    if tuple(d_cov.shape) != (2 * m, 2 * m):
        raise ValueError("d_cov must be 2m x 2m for patterns of length m")
    nq = int(d_patterns.shape[0])
    rec = ctypes.sizeof(_CResult)
    if d_out.dtype != torch.uint8 or not d_out.is_cuda or d_out.numel() < nq * rec or not d_out.is_contiguous():
        raise ValueError("d_out must be a contiguous uint8 device tensor of nq result records")
    raw = None if stream is None else getattr(stream, "cuda_stream", stream)
    _check(lib().tor_batch_async_noalloc(ctx.handle, ctypes.c_void_p(d_cov.data_ptr()), m, nq,
                                         ctypes.c_void_p(d_patterns.data_ptr()), _PREC[prec], float(tol),
                                         ctypes.c_void_p(d_out.data_ptr()), ctypes.c_void_p(raw)))
    return d_out


def results_from_device(d_out) -> list:
    """Decode the records written by Context.batch_async (copies to the host)."""
    buf = d_out.detach().cpu().contiguous().numpy().tobytes()
    rec = ctypes.sizeof(_CResult)
    return [Result._from(_CResult.from_buffer_copy(buf, i * rec)) for i in range(len(buf) // rec)]


class State:
    """A validated covariance kept by the library (tor_state)."""

    def __init__(self, ctx: Context, cov, mean=None):
        cov = _f64(cov)
        self.m = cov.shape[0] // 2
        h = ctypes.c_void_p()
        if mean is None:
            _check(lib().tor_state_create(ctx.handle, _dptr(cov), self.m, ctypes.byref(h)))
        else:
            mean = _f64(mean)
            if mean.shape != (2 * self.m,):
                raise ValueError("mean must have 2m entries")
            _check(lib().tor_state_create_displaced(ctx.handle, _dptr(cov), _dptr(mean), self.m, ctypes.byref(h)))
        self._h = h
        self.ctx = ctx

    @property
    def handle(self):
        return self._h

    def invert(self, prec="dd"):
        """tor_state_invert: sigma_Q^-1 of this (zero-mean) state, after which
        full patterns are evaluated from its clicked block (no per-query
        conditioning).  prec "qd" keeps quad-double words."""
        _check(lib().tor_state_invert(self._h, _PREC[prec]))
        return self

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tor_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (tor_server_*): submit from any thread, poll or
    wait for results; each result carries the submit-to-completion latency."""

    def __init__(self, ctx: Context, workers=2, max_pending=1 << 16, mem_budget_bytes=16 << 30, prec="dd",
                 tol=1e-10, max_batch=4096):
        o = _CServerOpts(int(workers), int(max_pending), int(mem_budget_bytes), _PREC[prec], float(tol),
                         int(max_batch))
        h = ctypes.c_void_p()
        _check(lib().tor_server_start(ctx.handle, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx

    def submit(self, state: State, pattern) -> int:
        """Returns a ticket, or raises TorError (status TOR_EAGAIN when not admitted)."""
        pattern = _i8(pattern)
        t = ctypes.c_uint64()
        _check(lib().tor_submit(self._h, state.handle, _i8ptr(pattern), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """(Result, latency_s) if done, else None."""
        r = _CResult()
        lat = ctypes.c_double()
        st = lib().tor_poll(self._h, ticket, ctypes.byref(r), ctypes.byref(lat))
        if st == TOR_EAGAIN:
            return None
        _check(st)
        return Result._from(r), lat.value

    def wait(self, ticket: int):
        r = _CResult()
        lat = ctypes.c_double()
        _check(lib().tor_wait(self._h, ticket, ctypes.byref(r), ctypes.byref(lat)))
        return Result._from(r), lat.value

    def stats(self) -> dict:
        s = _CServerStats()
        _check(lib().tor_server_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _CServerStats._fields_}

    def stop(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().tor_server_stop(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()


class PServer:
    """Persistent request loop (tor_pserver_*): one long-running kernel takes
    probability queries and sampling batches as they are submitted.  Submit
    from any thread; poll or wait for results (each with its submit-to-result
    latency)."""

    def __init__(self, ctx: Context, tol=1e-10, mem_budget_bytes=1 << 30, chain_buffer_bytes=64 << 20, grid=0,
                 idle_ms=50):
        o = _CPServerOpts(float(tol), int(mem_budget_bytes), int(chain_buffer_bytes), int(grid), int(idle_ms))
        h = ctypes.c_void_p()
        _check(lib().tor_pserver_start(ctx.handle, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx

    def submit(self, state: State, pattern) -> int:
        """Ticket of a probability query; raises TorError (TOR_EAGAIN: not admitted)."""
        pattern = _i8(pattern)
        if pattern.shape != (state.m,):
            raise ValueError("pattern must have m entries")
        t = ctypes.c_uint64()
        _check(lib().tor_pserver_submit(self._h, state.handle, _i8ptr(pattern), ctypes.byref(t)))
        return t.value

    def submit_chains(self, state: State, n_post: int, seed: int, chain_begin: int, nchains: int) -> int:
        """Ticket of a sampling batch (chains chain_begin .. + nchains - 1 of gbs_sample)."""
        t = ctypes.c_uint64()
        _check(lib().tor_pserver_submit_chains(self._h, state.handle, int(n_post), int(seed), int(chain_begin),
                                               int(nchains), ctypes.byref(t)))
        self._chains = getattr(self, "_chains", {})
        self._chains[t.value] = (state.m, int(nchains))
        return t.value

    def poll(self, ticket: int, wait: bool = False):
        """(Result, latency_s) once done, else None (wait=False)."""
        r = _CResult()
        lat = ctypes.c_double()
        st = lib().tor_pserver_poll(self._h, ticket, 1 if wait else 0, ctypes.byref(r), ctypes.byref(lat))
        if st == TOR_EAGAIN:
            return None
        _check(st)
        return Result._from(r), lat.value

    def wait(self, ticket: int):
        return self.poll(ticket, wait=True)

    def poll_chains(self, ticket: int, wait: bool = False):
        """(outcomes nchains x m uint8, status nchains int8, latency_s) once done, else None."""
        m, nchains = self._chains[ticket]
        outcomes = np.zeros((nchains, m), np.uint8)
        status = np.zeros(nchains, np.int8)
        lat = ctypes.c_double()
        st = lib().tor_pserver_poll_chains(self._h, ticket, 1 if wait else 0,
                                           outcomes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _i8ptr(status),
                                           ctypes.byref(lat))
        if st == TOR_EAGAIN:
            return None
        _check(st)
        del self._chains[ticket]
        return outcomes, status, lat.value

    def wait_chains(self, ticket: int):
        return self.poll_chains(ticket, wait=True)

    def autotune(self, n_lo=14, n_hi=24, cache_path=None):
        """Tune the unit depth per n (tor_pserver_autotune); optionally write the table."""
        _check(lib().tor_pserver_autotune(self._h, int(n_lo), int(n_hi),
                                          None if cache_path is None else str(cache_path).encode()))

    def stats(self) -> dict:
        s = _CPServerStats()
        _check(lib().tor_pserver_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _CPServerStats._fields_}

    def stop(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            h, self._h = self._h, None
            _check(lib().tor_pserver_stop(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()

