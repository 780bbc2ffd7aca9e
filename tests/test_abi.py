"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side validation rejects bad inputs without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1510_08628_amd as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(wlda_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(W.LIB_PATH):
        pytest.fail("libwarplda_hip.so is not built (run __graft_entry__.build())")
    return W.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(W.EXPORTS) <= set(names)


def test_strerror(lib):
    assert lib.wlda_strerror(0) == b"ok"
    assert lib.wlda_strerror(-4) == b"call out of order"


def _ws(lib, **kw):
    p = dict(V=3, D=2, K=4, M=2, alpha=0.1, beta=0.1, seed=1)
    p.update(kw)
    w = np.array(kw.pop("words", [0, 1, 2]), np.uint32)
    d = np.array(kw.pop("docs", [0, 1, 1]), np.uint32)
    params = W.Params(p["V"], p["D"], p["K"], p["M"], p["alpha"], p["beta"], p["seed"])
    out = C.c_uint64(0)
    rc = lib.wlda_workspace_bytes(C.byref(params), w.ctypes.data_as(C.c_void_p),
                                  d.ctypes.data_as(C.c_void_p), len(w), C.byref(out))
    return rc, out.value


def test_workspace_bytes_and_validation(lib):
    rc, n = _ws(lib)
    assert rc == 0 and n > 0
    for bad in [dict(K=0), dict(M=0), dict(M=5), dict(alpha=0.0), dict(beta=-1.0),
                dict(K=1 << 21), dict(V=2)]:     # V=2 makes word id 2 out of range
        rc, _ = _ws(lib, **bad)
        assert rc == -1, bad
    # null output pointer
    params = W.Params(3, 2, 4, 2, 0.1, 0.1, 1)
    assert lib.wlda_workspace_bytes(C.byref(params), None, None, 0, None) == -1


def test_create_rejects_bad_workspace(lib):
    params = W.Params(3, 2, 4, 2, 0.1, 0.1, 1)
    w = np.array([0, 1, 2], np.uint32)
    d = np.array([0, 1, 1], np.uint32)
    h = C.c_void_p()
    # misaligned / null workspace is rejected before any device call
    rc = lib.wlda_create(C.byref(params), w.ctypes.data_as(C.c_void_p),
                         d.ctypes.data_as(C.c_void_p), 3, C.c_void_p(0), 1 << 20, None,
                         C.byref(h))
    assert rc == -2
    rc = lib.wlda_create(C.byref(params), w.ctypes.data_as(C.c_void_p),
                         d.ctypes.data_as(C.c_void_p), 3, C.c_void_p(4096 + 8), 1 << 20, None,
                         C.byref(h))
    assert rc == -2


def test_null_handle_calls(lib):
    for fn in ("wlda_init", "wlda_word_phase", "wlda_doc_phase", "wlda_destroy"):
        assert getattr(lib, fn)(None) == -1


def test_workspace_grows_with_long_segments(lib):
    # one very long column triggers the multi-workgroup path and its table
    T = 20000
    rc1, small = _ws(lib, V=64, D=64, K=100000, words=list(np.arange(T) % 64),
                     docs=list(np.arange(T) % 64))
    rc2, big = _ws(lib, V=64, D=64, K=100000, words=[0] * T, docs=list(np.arange(T) % 64))
    assert rc1 == rc2 == 0
    assert big > small


def test_option_flags(lib):
    """wlda_workspace_bytes_ex: flag 0 is wlda_workspace_bytes; the alias-table
    word proposal moves the words with L_w > K to the long-word kernels (their
    count tables enter the workspace); unknown bits are refused."""
    K = 300
    w = np.array([0] * 1000 + [1, 2], np.uint32)  # word 0: L_w = 1000 > K
    d = np.array([0, 1] * 501, np.uint32)
    params = W.Params(3, 2, K, 2, 0.1, 0.1, 1)
    out = C.c_uint64(0)

    def ws(flags):
        rc = lib.wlda_workspace_bytes_ex(C.byref(params), w.ctypes.data_as(C.c_void_p),
                                         d.ctypes.data_as(C.c_void_p), len(w), flags,
                                         C.byref(out))
        return rc, out.value

    rc0, plain = ws(0)
    assert rc0 == 0 and (0, plain) == _ws(lib, V=3, D=2, K=K, words=list(w), docs=list(d))
    rc1, alias = ws(W.WORD_ALIAS)
    assert rc1 == 0 and alias > plain
    assert ws(2)[0] == -1 and ws(0x80000000)[0] == -1
    h = C.c_void_p()
    rc = lib.wlda_create_ex(C.byref(params), w.ctypes.data_as(C.c_void_p),
                            d.ctypes.data_as(C.c_void_p), len(w), 4, C.c_void_p(0), 1 << 20, None,
                            C.byref(h))
    assert rc == -1
