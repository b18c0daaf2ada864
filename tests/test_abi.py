"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/tor.h declares; host validation paths need no GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1810_00900_amd as tg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:tor_status|void|const char \*|int)\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_built():
    assert os.path.exists(tg.LIB_PATH), "build the library first (__graft_entry__.build())"


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(tg.LIB_PATH)
    names = _declared("tor.h")
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_signatures_match_header():
    names = _declared("tor.h")
    L = tg.lib()
    for n in names:
        assert getattr(L, n).restype is not None or n.endswith("destroy"), n


def test_no_gpu_fails_loudly():
    """Without a GPU the context cannot be created and the error says why."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(tg.TorError) as ei:
        tg.Context(0)
    assert ei.value.status in (tg.TOR_EDEVICE, tg.TOR_EINVAL)
    assert tg.last_error()


def test_last_error_is_a_string():
    assert isinstance(tg.last_error(), str)


def test_null_context_rejected():
    L = tg.lib()
    r = tg._CResult()
    cov = np.eye(2) * 0.5
    pat = np.ones(1, np.int8)
    st = L.tor_probability(None, tg._dptr(cov), 1, tg._i8ptr(pat), 0, 1e-10, ctypes.byref(r))
    assert st == tg.TOR_EINVAL


def test_null_context_rejected_displaced():
    L = tg.lib()
    r = tg._CResult()
    cov = np.eye(2) * 0.5
    mean = np.zeros(2)
    pat = np.ones(1, np.int8)
    st = L.tor_probability_displaced(None, tg._dptr(cov), tg._dptr(mean), 1, tg._i8ptr(pat), 0, 1e-10,
                                     ctypes.byref(r))
    assert st == tg.TOR_EINVAL


def test_null_state_rejected_by_invert():
    assert tg.lib().tor_state_invert(None, tg.PREC_DD) == tg.TOR_EINVAL


def test_binding_constants_match_header():
    src = open(os.path.join(ROOT, "include", "tor.h")).read()
    consts = dict(re.findall(r"^#define (TOR_[A-Z_]+) \(?(-?\d+)\)?", src, flags=re.M))
    for name in ("TOR_OK", "TOR_WARN_PRECISION", "TOR_EINVAL", "TOR_ENOTPD", "TOR_ETOOBIG", "TOR_ENOMEM",
                 "TOR_EDEVICE", "TOR_EAGAIN"):
        assert getattr(tg, name) == int(consts[name]), name
    assert tg.PS_SLOTS == int(consts["TOR_PS_SLOTS"])
    assert tg.FUSED_MAX_TASKS == int(consts["TOR_FUSED_MAX_TASKS"])
    opts = dict(re.findall(r"^\s+TOR_OPT_([A-Z_]+) = (\d+)", src, flags=re.M))
    assert len(opts) == 9
    for name, v in opts.items():
        assert getattr(tg, "OPT_" + name) == int(v), name
