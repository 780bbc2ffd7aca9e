"""CPU oracle for the WarpLDA sweep -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it.

``warplda_oracle.c`` is a plain, single-threaded C implementation written from
the paper (Algorithm 2, Eq. (5)-(7), the log joint likelihood of Section 6.1);
this module loads it with ctypes.  The exact (binary64) enumerators that pin it
live with the tests (``tests/enum_chain.py``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "warplda_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

PH_WORD, PH_DOC = 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary32 arithmetic without contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
             "-fexcess-precision=standard", "-shared", "-fPIC", SRC, "-o", tmp,
             "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("V", C.c_uint32), ("D", C.c_uint32), ("K", C.c_uint32),
                ("M", C.c_uint32), ("alpha", C.c_double), ("beta", C.c_double),
                ("seed", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
        L.oracle_create.restype = vp
        L.oracle_create.argtypes = [C.POINTER(_Params), vp, vp, u64]
        L.oracle_destroy.argtypes = [vp]
        for f in ("oracle_init", "oracle_word_phase", "oracle_doc_phase"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = C.c_int
        L.oracle_iterate.argtypes = [vp, u32]
        L.oracle_iterate.restype = C.c_int
        L.oracle_log_likelihood.argtypes = [vp]
        L.oracle_log_likelihood.restype = C.c_double
        L.oracle_log_joint.argtypes = [u64, u32, u32, u32, C.c_double, C.c_double, vp, vp, vp]
        L.oracle_log_joint.restype = C.c_double
        L.oracle_num_tokens.argtypes = [vp]
        L.oracle_num_tokens.restype = u64
        L.oracle_iteration.argtypes = [vp]
        L.oracle_iteration.restype = u32
        L.oracle_accepted.argtypes = [vp, C.c_int]
        L.oracle_accepted.restype = u64
        L.oracle_set_visit_reversed.argtypes = [vp, C.c_int]
        L.oracle_copy_assignments.argtypes = [vp, vp, vp]
        L.oracle_copy_csc.argtypes = [vp, vp, vp]
        L.oracle_copy_layout.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_copy_topic_counts.argtypes = [vp, vp]
        L.oracle_state_bytes.argtypes = [vp]
        L.oracle_state_bytes.restype = u64
        L.oracle_save_state.argtypes = [vp, vp, u64]
        L.oracle_save_state.restype = C.c_int
        L.oracle_load_state.argtypes = [vp, vp, u64]
        L.oracle_load_state.restype = C.c_int
        L.oracle_set_csc_state.argtypes = [vp, vp, vp]
        L.oracle_frozen_chain.argtypes = [vp, u32, u32, C.c_int, vp]
        L.oracle_frozen_chain.restype = C.c_int
        L.oracle_philox4x32_10.argtypes = [vp, vp, vp]
        L.oracle_theta.argtypes = [vp, u32, u32, vp]
        L.oracle_theta.restype = C.c_int
        L.oracle_phi.argtypes = [vp, u32, u32, vp]
        L.oracle_phi.restype = C.c_int
        L.oracle_set_token_offsets.argtypes = [vp, u32, u32]
        L.oracle_set_phase_state.argtypes = [vp, vp, C.c_int, u32]
        L.oracle_set_phase_state.restype = C.c_int
        L.oracle_set_alpha.argtypes = [vp, vp]
        L.oracle_set_alpha.restype = C.c_int
        L.oracle_set_word_alias.argtypes = [vp, C.c_int]
        L.oracle_set_word_alias.restype = C.c_int
        L.oracle_alias_table.argtypes = [vp, u32, u64, vp, vp]
        L.oracle_alias_table.restype = C.c_int
        L.oracle_instant_iterate.argtypes = [vp, u32]
        L.oracle_instant_iterate.restype = C.c_int
        L.oracle_foldin.argtypes = [u32, u32, u32, C.c_double, C.c_double, u64, vp, vp, vp,
                                    u32, vp, vp, vp, u32, u32, vp, u32, vp, vp]
        L.oracle_foldin.restype = C.c_int
        L.oracle_heldout_ll.argtypes = [u32, u32, C.c_double, C.c_double, vp, vp, vp, u32, vp, vp,
                                        vp, vp]
        L.oracle_heldout_ll.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(key, ctr) -> np.ndarray:
    k = np.ascontiguousarray(key, dtype=np.uint32)
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(k), _ptr(c), _ptr(out))
    return out


def log_joint(word_ids, doc_ids, z, V, D, K, alpha, beta) -> float:
    w = np.ascontiguousarray(word_ids, dtype=np.uint32)
    d = np.ascontiguousarray(doc_ids, dtype=np.uint32)
    zz = np.ascontiguousarray(z, dtype=np.int32)
    return lib().oracle_log_joint(len(w), V, D, K, alpha, beta, _ptr(w), _ptr(d), _ptr(zz))


def alias_table(counts):
    """Walker's alias table of oracle_alias_table over integer counts (one
    per topic, summing to L < 2^31): (thr, alias) as uint32 arrays."""
    c = np.ascontiguousarray(counts, dtype=np.int64)
    K = c.shape[0]
    thr = np.zeros(K, np.uint32)
    al = np.zeros(K, np.uint32)
    rc = lib().oracle_alias_table(_ptr(c), K, int(c.sum()), _ptr(thr), _ptr(al))
    if rc != 0:
        raise ValueError("counts must be non-negative and sum to 0 < L < 2^31")
    return thr, al


class FrozenModel:
    """A trained model as the oracle's fold-in sees it: the canonical column
    layout of the training corpus, its assignments and c_k."""

    def __init__(self, word_ids, doc_ids, z, V, D, K, M, alpha, beta, seed=1):
        o = Oracle(word_ids, doc_ids, V, D, K, M, alpha, beta, seed)
        colptr, _, _, inv = o.layout()
        zc = np.empty(len(z), np.int32)
        zc[inv] = np.asarray(z, np.int32)
        self.colptr = colptr
        self.z_csc = zc
        self.ck = np.bincount(zc, minlength=K).astype(np.int64)
        self.V, self.K, self.M, self.alpha, self.beta, self.seed = V, K, M, alpha, beta, seed

    def foldin(self, docptr, words, req_ids, sweeps, weights=None, learned_steps=0,
               first_sweep=0, z=None, pd=None):
        docptr = np.ascontiguousarray(docptr, np.uint64)
        words = np.ascontiguousarray(words, np.uint32)
        req = np.ascontiguousarray(req_ids, np.uint32)
        T = int(docptr[-1])
        z = np.zeros(T, np.int32) if z is None else np.ascontiguousarray(z, np.int32).copy()
        pd = np.zeros(self.M * T, np.int32) if pd is None else np.ascontiguousarray(pd, np.int32).copy()
        w = None if weights is None else np.ascontiguousarray(weights, np.uint32)
        rc = lib().oracle_foldin(self.V, self.K, self.M, self.alpha, self.beta, self.seed,
                                 _ptr(self.colptr), _ptr(self.z_csc), _ptr(self.ck),
                                 len(req), _ptr(docptr), _ptr(words), _ptr(req), first_sweep,
                                 sweeps, None if w is None else _ptr(w), learned_steps,
                                 _ptr(z), _ptr(pd))
        if rc != 0:
            raise RuntimeError("oracle_foldin failed")
        return z, pd

    def heldout_ll(self, docptr, z, hoptr, ho_words) -> float:
        docptr = np.ascontiguousarray(docptr, np.uint64)
        hoptr = np.ascontiguousarray(hoptr, np.uint64)
        z = np.ascontiguousarray(z, np.int32)
        how = np.ascontiguousarray(ho_words, np.uint32)
        return lib().oracle_heldout_ll(self.V, self.K, self.alpha, self.beta, _ptr(self.colptr),
                                       _ptr(self.z_csc), _ptr(self.ck), len(docptr) - 1,
                                       _ptr(docptr), _ptr(z), _ptr(hoptr), _ptr(how))


class Oracle:
    """Handle around the C oracle; mirrors the library's sampler calls."""

    def __init__(self, word_ids, doc_ids, V, D, K, M, alpha, beta, seed=1):
        self.word_ids = np.ascontiguousarray(word_ids, dtype=np.uint32)
        self.doc_ids = np.ascontiguousarray(doc_ids, dtype=np.uint32)
        self.V, self.D, self.K, self.M = V, D, K, M
        self.alpha, self.beta, self.seed = alpha, beta, seed
        p = _Params(V, D, K, M, alpha, beta, seed)
        self.h = lib().oracle_create(C.byref(p), _ptr(self.word_ids), _ptr(self.doc_ids),
                                     len(self.word_ids))
        if not self.h:
            raise ValueError("oracle_create rejected the inputs")
        self.T = len(self.word_ids)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().oracle_destroy(h)
            self.h = None

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError(f"oracle call failed ({rc})")

    def init(self):
        self._check(lib().oracle_init(self.h))

    def word_phase(self):
        self._check(lib().oracle_word_phase(self.h))

    def doc_phase(self):
        self._check(lib().oracle_doc_phase(self.h))

    def iterate(self, n=1):
        self._check(lib().oracle_iterate(self.h, n))

    def log_likelihood(self) -> float:
        return lib().oracle_log_likelihood(self.h)

    @property
    def iteration(self) -> int:
        return lib().oracle_iteration(self.h)

    def accepted(self, phase: int) -> int:
        return lib().oracle_accepted(self.h, phase)

    def set_visit_reversed(self, rev: bool):
        lib().oracle_set_visit_reversed(self.h, int(rev))

    def assignments(self):
        z = np.empty(self.T, dtype=np.int32)
        p = np.empty((self.M, self.T), dtype=np.int32)
        lib().oracle_copy_assignments(self.h, _ptr(z), _ptr(p))
        return z, p

    def csc(self):
        z = np.empty(self.T, dtype=np.int32)
        p = np.empty((self.M, self.T), dtype=np.int32)
        lib().oracle_copy_csc(self.h, _ptr(z), _ptr(p))
        return z, p

    def layout(self):
        colptr = np.empty(self.V + 1, dtype=np.uint64)
        rowptr = np.empty(self.D + 1, dtype=np.uint64)
        row = np.empty(self.T, dtype=np.uint32)
        inv = np.empty(self.T, dtype=np.uint32)
        lib().oracle_copy_layout(self.h, _ptr(colptr), _ptr(rowptr), _ptr(row), _ptr(inv))
        return colptr, rowptr, row, inv

    def topic_counts(self):
        ck = np.empty(self.K, dtype=np.int64)
        lib().oracle_copy_topic_counts(self.h, _ptr(ck))
        return ck

    def save_state(self) -> bytes:
        n = lib().oracle_state_bytes(self.h)
        buf = np.empty(n, dtype=np.uint8)
        self._check(lib().oracle_save_state(self.h, _ptr(buf), n))
        return buf.tobytes()

    def load_state(self, blob: bytes):
        buf = np.frombuffer(blob, dtype=np.uint8).copy()
        self._check(lib().oracle_load_state(self.h, _ptr(buf), len(buf)))

    def set_csc_state(self, z_csc, props_csc=None):
        z = np.ascontiguousarray(z_csc, dtype=np.int32)
        if props_csc is not None:
            p = np.ascontiguousarray(props_csc, dtype=np.int32)
            lib().oracle_set_csc_state(self.h, _ptr(z), _ptr(p))
        else:
            lib().oracle_set_csc_state(self.h, _ptr(z), None)

    def theta(self, d0: int = 0, nd: int | None = None) -> np.ndarray:
        """theta_hat of Eq. (4) for documents d0 .. d0+nd-1 (nd x K, binary64)."""
        nd = self.D - d0 if nd is None else nd
        out = np.empty((nd, self.K), dtype=np.float64)
        self._check(lib().oracle_theta(self.h, d0, nd, _ptr(out)))
        return out

    def phi(self, w0: int = 0, nw: int | None = None) -> np.ndarray:
        """phi_hat of Eq. (4) for words w0 .. w0+nw-1 (nw x K, binary64)."""
        nw = self.V - w0 if nw is None else nw
        out = np.empty((nw, self.K), dtype=np.float64)
        self._check(lib().oracle_phi(self.h, w0, nw, _ptr(out)))
        return out

    def set_token_offsets(self, csc_off: int, csr_off: int):
        """Test harness: this corpus is one column (row) of a larger one whose
        canonical positions start at csc_off (csr_off)."""
        lib().oracle_set_token_offsets(self.h, csc_off, csr_off)

    def set_phase_state(self, ck, next_phase: int, iteration: int):
        """Test harness: the larger corpus's c_k at the start of the next
        phase, that phase (PH_WORD or PH_DOC) and the completed iterations."""
        c = np.ascontiguousarray(ck, dtype=np.int64)
        assert c.shape == (self.K,)
        self._check(lib().oracle_set_phase_state(self.h, _ptr(c), next_phase, iteration))

    def set_alpha(self, alpha):
        """Asymmetric document-topic prior alpha_k (K positive values, taken
        as binary32), or None for the symmetric alpha; before init()."""
        if alpha is None:
            self._check(lib().oracle_set_alpha(self.h, None))
            self.alpha_k = None
            return
        a = np.ascontiguousarray(alpha, dtype=np.float32)
        if a.shape != (self.K,):
            raise ValueError("alpha must hold K values")
        self._check(lib().oracle_set_alpha(self.h, _ptr(a)))
        self.alpha_k = a

    def set_word_alias(self, on: bool):
        """Word proposals of columns with L_w > K from Walker's alias table
        over the updated c_w (True) or its inverse CDF (False, default)."""
        self._check(lib().oracle_set_word_alias(self.h, int(bool(on))))

    def instant_iterate(self, n: int = 1):
        """n iterations of the instant-update (collapsed Gibbs-MH) variant."""
        self._check(lib().oracle_instant_iterate(self.h, n))

    def frozen_chain(self, t: int, rounds: int, mode: int) -> np.ndarray:
        hist = np.zeros(self.K, dtype=np.uint64)
        self._check(lib().oracle_frozen_chain(self.h, t, rounds, mode, _ptr(hist)))
        return hist
