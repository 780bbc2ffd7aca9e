"""Python binding of the MI355X WarpLDA library (include/warplda.h).

Argument marshalling only: every step of the sweep runs in the HIP kernels of
``libwarplda_hip.so``.  PyTorch provides the device workspace and the stream.
There is no CPU fallback: if the library is not built, loading fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwarplda_hip.so")

WLDA_OK = 0
WORD_ALIAS = 1          # WLDA_WORD_ALIAS: alias-table word proposals for L_w > K
STATUS = {0: "ok", -1: "invalid argument", -2: "workspace too small or misaligned",
          -3: "HIP runtime error", -4: "call out of order", -5: "unsupported by this build",
          -6: "host memory exhausted"}


class WldaError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)} ({code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [("V", C.c_uint32), ("D", C.c_uint32), ("K", C.c_uint32), ("M", C.c_uint32),
                ("alpha", C.c_double), ("beta", C.c_double), ("seed", C.c_uint64)]


# Every symbol declared in include/warplda.h (checked by the CPU tests).
EXPORTS = [
    "wlda_workspace_bytes", "wlda_create", "wlda_workspace_bytes_ex", "wlda_create_ex",
    "wlda_set_alpha", "wlda_init", "wlda_word_phase",
    "wlda_doc_phase",
    "wlda_iterate", "wlda_log_likelihood", "wlda_copy_assignments",
    "wlda_copy_assignments_csc", "wlda_copy_topic_counts", "wlda_accepted", "wlda_iteration",
    "wlda_state_bytes", "wlda_save_state", "wlda_load_state", "wlda_set_assignments",
    "wlda_destroy", "wlda_strerror", "wlda_profile", "wlda_profile_read",
    "wlda_model_workspace_bytes", "wlda_model_create", "wlda_model_destroy",
    "wlda_foldin_batch_bytes", "wlda_foldin_batch", "wlda_foldin_batch_static",
    "wlda_encoder_workspace_bytes", "wlda_encoder_create", "wlda_encoder_destroy",
    "wlda_encoder_set_weights", "wlda_encoder_get_weights", "wlda_encoder_features",
    "wlda_encoder_forward", "wlda_encoder_proposal", "wlda_encoder_gradients",
    "wlda_encoder_train_step", "wlda_theta", "wlda_phi", "wlda_encoder_features_batch",
    "wlda_server_workspace_bytes", "wlda_server_create", "wlda_server_now", "wlda_server_submit",
    "wlda_server_step", "wlda_server_poll", "wlda_server_take_z", "wlda_server_destroy",
]


class ServerParams(C.Structure):
    _fields_ = [("max_docs", C.c_uint32), ("pool_tokens", C.c_uint64),
                ("pool_heldout", C.c_uint64), ("sweeps", C.c_uint32),
                ("learned_steps", C.c_uint32), ("eps", C.c_float)]


class Result(C.Structure):
    _fields_ = [("req_id", C.c_uint32), ("n_tokens", C.c_uint32), ("n_heldout", C.c_uint32),
                ("sweeps", C.c_uint32), ("learned", C.c_uint32), ("arrival_s", C.c_double),
                ("admit_s", C.c_double), ("done_s", C.c_double), ("heldout_ll", C.c_double)]


class EncoderParams(C.Structure):
    _fields_ = [("buckets", C.c_uint32), ("hidden", C.c_uint32), ("K", C.c_uint32),
                ("max_batch", C.c_uint32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char_p), ("launches", C.c_uint64),
                ("tokens_per_launch", C.c_uint64), ("total_ms", C.c_double)]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libwarplda_hip.so (raises if it is missing: no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build()")
    # torch first: its bundled HIP runtime must be the one this library binds
    # to, or device pointers and streams from torch would belong to another
    # runtime instance in the same process
    import torch  # noqa: F401
    L = C.CDLL(path)
    vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    P = C.POINTER(Params)
    sig = {
        "wlda_workspace_bytes": [P, vp, vp, u64, C.POINTER(u64)],
        "wlda_create": [P, vp, vp, u64, vp, u64, vp, C.POINTER(vp)],
        "wlda_workspace_bytes_ex": [P, vp, vp, u64, u32, C.POINTER(u64)],
        "wlda_create_ex": [P, vp, vp, u64, u32, vp, u64, vp, C.POINTER(vp)],
        "wlda_init": [vp], "wlda_word_phase": [vp], "wlda_doc_phase": [vp],
        "wlda_set_alpha": [vp, vp],
        "wlda_iterate": [vp, u32],
        "wlda_log_likelihood": [vp, C.POINTER(C.c_double)],
        "wlda_copy_assignments": [vp, vp, vp],
        "wlda_copy_assignments_csc": [vp, vp, vp],
        "wlda_copy_topic_counts": [vp, vp],
        "wlda_accepted": [vp, i32, C.POINTER(u64)],
        "wlda_iteration": [vp, C.POINTER(u32)],
        "wlda_state_bytes": [vp, C.POINTER(u64)],
        "wlda_save_state": [vp, vp, u64], "wlda_load_state": [vp, vp, u64],
        "wlda_set_assignments": [vp, vp, vp],
        "wlda_destroy": [vp],
        "wlda_profile": [vp, i32],
        "wlda_model_workspace_bytes": [P, u64, C.POINTER(u64)],
        "wlda_model_create": [P, vp, vp, vp, u64, vp, u64, vp, C.POINTER(vp)],
        "wlda_model_destroy": [vp],
        "wlda_foldin_batch_bytes": [vp, u32, u64, i32, u64, C.POINTER(u64)],
        "wlda_foldin_batch": [vp, u32, vp, vp, vp, vp, u32, u32, vp, vp, vp, u64, vp, vp],
        "wlda_foldin_batch_static": [vp, u32, vp, vp, vp, vp, u32, u32, vp, vp, vp, vp],
        "wlda_encoder_workspace_bytes": [C.POINTER(EncoderParams), C.POINTER(u64)],
        "wlda_encoder_create": [C.POINTER(EncoderParams), vp, u64, vp, C.POINTER(vp)],
        "wlda_encoder_destroy": [vp],
        "wlda_encoder_set_weights": [vp, vp],
        "wlda_encoder_get_weights": [vp, vp],
        "wlda_encoder_features": [u32, vp, u32, vp, vp, C.POINTER(u32)],
        "wlda_encoder_forward": [vp, u32, vp, vp, vp, vp],
        "wlda_encoder_proposal": [vp, u32, vp, C.c_float, vp],
        "wlda_encoder_gradients": [vp, u32, vp, vp, vp, vp, C.POINTER(C.c_float), vp],
        "wlda_encoder_train_step": [vp, u32, vp, vp, vp, vp, C.POINTER(C.c_float)],
        "wlda_theta": [vp, u32, u32, vp],
        "wlda_phi": [vp, u32, u32, vp],
        "wlda_encoder_features_batch": [u32, u32, vp, vp, vp, vp, vp],
        "wlda_server_workspace_bytes": [vp, vp, C.POINTER(ServerParams), C.POINTER(u64)],
        "wlda_server_create": [vp, vp, C.POINTER(ServerParams), vp, u64, vp, C.POINTER(vp)],
        "wlda_server_now": [vp, C.POINTER(C.c_double)],
        "wlda_server_submit": [vp, u32, vp, u32, vp, u32, C.c_double, vp],
        "wlda_server_step": [vp, C.POINTER(u32), C.POINTER(u32)],
        "wlda_server_poll": [vp, C.POINTER(Result), u32, C.POINTER(u32)],
        "wlda_server_take_z": [vp, u32, vp, u32],
        "wlda_server_destroy": [vp],
        "wlda_profile_read": [vp, C.POINTER(KernelStat), u32, C.POINTER(u32)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i32
    L.wlda_strerror.argtypes = [i32]
    L.wlda_strerror.restype = C.c_char_p
    _lib = L
    return L


def _check(fn, rc):
    if rc != WLDA_OK:
        raise WldaError(fn, rc)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Sampler:
    """One WarpLDA sampler on one GPU (mirrors the wlda_* calls).

    word_alias=True creates it with WLDA_WORD_ALIAS: the word proposals of
    words with L_w > K come from Walker's alias table over the updated c_w
    (Algorithm 2's BuildAlias / urn.Draw) instead of its inverse CDF."""

    def __init__(self, word_ids, doc_ids, V, D, K, M, alpha, beta, seed=1, device="cuda:0",
                 stream=None, word_alias=False):
        import torch
        L = load_library()
        self.word_ids = np.ascontiguousarray(word_ids, dtype=np.uint32)
        self.doc_ids = np.ascontiguousarray(doc_ids, dtype=np.uint32)
        self.T = int(self.word_ids.shape[0])
        self.V, self.D, self.K, self.M = V, D, K, M
        self.params = Params(V, D, K, M, float(alpha), float(beta), int(seed))
        self.flags = WORD_ALIAS if word_alias else 0
        nbytes = C.c_uint64(0)
        _check("wlda_workspace_bytes_ex",
               L.wlda_workspace_bytes_ex(C.byref(self.params), _ptr(self.word_ids),
                                         _ptr(self.doc_ids), self.T, self.flags, C.byref(nbytes)))
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p(0)
        _check("wlda_create_ex",
               L.wlda_create_ex(C.byref(self.params), _ptr(self.word_ids), _ptr(self.doc_ids),
                                self.T, self.flags, C.c_void_p(self.workspace.data_ptr()),
                                int(nbytes.value), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    @property
    def workspace_bytes(self) -> int:
        return int(self.workspace.numel())

    def close(self):
        if getattr(self, "h", None):
            load_library().wlda_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_alpha(self, alpha):
        """Asymmetric document-topic prior alpha_k (K positive values, taken as
        binary32), or None for the symmetric alpha; before the first init()."""
        if alpha is None:
            _check("wlda_set_alpha", load_library().wlda_set_alpha(self.h, None))
            return
        a = np.ascontiguousarray(alpha, dtype=np.float32)
        if a.shape != (self.K,):
            raise ValueError("alpha must hold K values")
        _check("wlda_set_alpha", load_library().wlda_set_alpha(self.h, a.ctypes.data))

    def init(self):
        _check("wlda_init", load_library().wlda_init(self.h))

    def word_phase(self):
        _check("wlda_word_phase", load_library().wlda_word_phase(self.h))

    def doc_phase(self):
        _check("wlda_doc_phase", load_library().wlda_doc_phase(self.h))

    def iterate(self, n=1):
        _check("wlda_iterate", load_library().wlda_iterate(self.h, n))

    def log_likelihood(self) -> float:
        v = C.c_double(0)
        _check("wlda_log_likelihood", load_library().wlda_log_likelihood(self.h, C.byref(v)))
        return v.value

    def assignments(self, csc=False):
        z = np.empty(self.T, dtype=np.int32)
        p = np.empty((self.M, self.T), dtype=np.int32)
        fn = "wlda_copy_assignments_csc" if csc else "wlda_copy_assignments"
        _check(fn, getattr(load_library(), fn)(self.h, _ptr(z), _ptr(p)))
        return z, p

    def topic_counts(self):
        ck = np.empty(self.K, dtype=np.int64)
        _check("wlda_copy_topic_counts", load_library().wlda_copy_topic_counts(self.h, _ptr(ck)))
        return ck

    def accepted(self, phase: int) -> int:
        v = C.c_uint64(0)
        _check("wlda_accepted", load_library().wlda_accepted(self.h, phase, C.byref(v)))
        return int(v.value)

    @property
    def iteration(self) -> int:
        v = C.c_uint32(0)
        _check("wlda_iteration", load_library().wlda_iteration(self.h, C.byref(v)))
        return int(v.value)

    def save_state(self) -> bytes:
        n = C.c_uint64(0)
        _check("wlda_state_bytes", load_library().wlda_state_bytes(self.h, C.byref(n)))
        buf = np.empty(int(n.value), dtype=np.uint8)
        _check("wlda_save_state", load_library().wlda_save_state(self.h, _ptr(buf), int(n.value)))
        return buf.tobytes()

    def load_state(self, blob: bytes):
        buf = np.frombuffer(blob, dtype=np.uint8).copy()
        _check("wlda_load_state", load_library().wlda_load_state(self.h, _ptr(buf), len(buf)))

    def profile(self, enable: bool):
        _check("wlda_profile", load_library().wlda_profile(self.h, int(enable)))

    def profile_read(self):
        """{kernel kind: (launches, tokens per launch, total ms)}"""
        arr = (KernelStat * 32)()
        n = C.c_uint32(0)
        _check("wlda_profile_read", load_library().wlda_profile_read(self.h, arr, 32, C.byref(n)))
        return {arr[i].name.decode(): (int(arr[i].launches), int(arr[i].tokens_per_launch),
                                       float(arr[i].total_ms)) for i in range(n.value)}

    def theta(self, d0, nd, out=None):
        """theta_hat rows of documents d0..d0+nd-1 as a device tensor (nd x K)."""
        import torch
        if out is None:
            out = torch.empty((nd, self.K), dtype=torch.float32, device=self.device)
        _check("wlda_theta", load_library().wlda_theta(self.h, d0, nd, C.c_void_p(out.data_ptr())))
        return out

    def phi(self, w0, nw, out=None):
        """phi_hat rows of words w0..w0+nw-1 as a device tensor (nw x K)."""
        import torch
        if out is None:
            out = torch.empty((nw, self.K), dtype=torch.float32, device=self.device)
        _check("wlda_phi", load_library().wlda_phi(self.h, w0, nw, C.c_void_p(out.data_ptr())))
        return out

    def set_assignments(self, z, props=None):
        zz = np.ascontiguousarray(z, dtype=np.int32)
        pp = None if props is None else np.ascontiguousarray(props, dtype=np.int32)
        _check("wlda_set_assignments",
               load_library().wlda_set_assignments(self.h, _ptr(zz),
                                                   None if pp is None else _ptr(pp)))


class Model:
    """A frozen model on the GPU (wlda_model_create): trained corpus + z."""

    def __init__(self, word_ids, doc_ids, z, V, D, K, M, alpha, beta, seed=1, device="cuda:0",
                 stream=None):
        import torch
        L = load_library()
        self.params = Params(V, D, K, M, float(alpha), float(beta), int(seed))
        self.K, self.M, self.V = K, M, V
        w = np.ascontiguousarray(word_ids, dtype=np.uint32)
        d = np.ascontiguousarray(doc_ids, dtype=np.uint32)
        zz = np.ascontiguousarray(z, dtype=np.int32)
        n = C.c_uint64(0)
        _check("wlda_model_workspace_bytes",
               L.wlda_model_workspace_bytes(C.byref(self.params), len(w), C.byref(n)))
        self.device = torch.device(device)
        self.workspace = torch.empty(int(n.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p(0)
        _check("wlda_model_create",
               L.wlda_model_create(C.byref(self.params), _ptr(w), _ptr(d), _ptr(zz), len(w),
                                   C.c_void_p(self.workspace.data_ptr()), int(n.value),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load_library().wlda_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def foldin(self, docptr, words, req_ids, sweeps, weights=None, learned_steps=0,
               hoptr=None, ho_words=None):
        """Batch fold-in; returns (z, heldout_ll per doc or None)."""
        import torch
        L = load_library()
        docptr = np.ascontiguousarray(docptr, np.uint64)
        words = np.ascontiguousarray(words, np.uint32)
        req = np.ascontiguousarray(req_ids, np.uint32)
        nd = len(req)
        T = int(docptr[-1])
        w = None if weights is None else np.ascontiguousarray(weights, np.uint32)
        hp = None if hoptr is None else np.ascontiguousarray(hoptr, np.uint64)
        hw = None if ho_words is None else np.ascontiguousarray(ho_words, np.uint32)
        n_ho = 0 if hp is None else int(hp[-1])
        nb = C.c_uint64(0)
        _check("wlda_foldin_batch_bytes",
               L.wlda_foldin_batch_bytes(self.h, nd, T, int(w is not None), n_ho, C.byref(nb)))
        ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        z = np.empty(T, np.int32)
        ho = np.empty(nd, np.float64) if hp is not None else None
        _check("wlda_foldin_batch",
               L.wlda_foldin_batch(self.h, nd, _ptr(docptr), _ptr(words), _ptr(req),
                                   None if w is None else _ptr(w), learned_steps, sweeps,
                                   None if hp is None else _ptr(hp),
                                   None if hw is None else _ptr(hw),
                                   C.c_void_p(ws.data_ptr()), int(nb.value), _ptr(z),
                                   None if ho is None else _ptr(ho)))
        del ws
        return z, ho

    def foldin_static(self, docptr, words, req_ids, sweeps, weights=None, learned_steps=0,
                      hoptr=None, ho_words=None):
        """The same batch through wlda_foldin_batch_static (no workspace: the
        library's static device array of WLDA_FOLDIN_STATIC_BYTES)."""
        L = load_library()
        docptr = np.ascontiguousarray(docptr, np.uint64)
        words = np.ascontiguousarray(words, np.uint32)
        req = np.ascontiguousarray(req_ids, np.uint32)
        nd = len(req)
        T = int(docptr[-1])
        w = None if weights is None else np.ascontiguousarray(weights, np.uint32)
        hp = None if hoptr is None else np.ascontiguousarray(hoptr, np.uint64)
        hw = None if ho_words is None else np.ascontiguousarray(ho_words, np.uint32)
        z = np.empty(T, np.int32)
        ho = np.empty(nd, np.float64) if hp is not None else None
        _check("wlda_foldin_batch_static",
               L.wlda_foldin_batch_static(self.h, nd, _ptr(docptr), _ptr(words), _ptr(req),
                                          None if w is None else _ptr(w), learned_steps, sweeps,
                                          None if hp is None else _ptr(hp),
                                          None if hw is None else _ptr(hw), _ptr(z),
                                          None if ho is None else _ptr(ho)))
        return z, ho


def encoder_features(buckets: int, words) -> tuple:
    """Sparse hashed bag of words of one document (library host helper)."""
    w = np.ascontiguousarray(words, np.uint32)
    idx = np.empty(max(1, len(w)), np.uint32)
    val = np.empty(max(1, len(w)), np.float32)
    n = C.c_uint32(0)
    _check("wlda_encoder_features",
           load_library().wlda_encoder_features(buckets, _ptr(w), len(w), _ptr(idx), _ptr(val),
                                                C.byref(n)))
    return idx[:n.value].copy(), val[:n.value].copy()


def features_csr(buckets: int, docptr, words) -> tuple:
    """CSR (rowptr, idx, val) of documents words[docptr[d]:docptr[d+1]]."""
    dp = np.ascontiguousarray(docptr, np.uint64)
    w = np.ascontiguousarray(words, np.uint32)
    n = len(dp) - 1
    rowptr = np.empty(n + 1, np.uint32)
    idx = np.empty(max(1, len(w)), np.uint32)
    val = np.empty(max(1, len(w)), np.float32)
    _check("wlda_encoder_features_batch",
           load_library().wlda_encoder_features_batch(buckets, n, _ptr(dp), _ptr(w), _ptr(rowptr),
                                                      _ptr(idx), _ptr(val)))
    return rowptr, idx[:rowptr[-1]].copy(), val[:rowptr[-1]].copy()


def batch_features(buckets: int, docs) -> tuple:
    """CSR (rowptr, idx, val) of a list of documents (word-id arrays)."""
    rows, idxs, vals = [0], [], []
    for words in docs:
        i, v = encoder_features(buckets, words)
        idxs.append(i)
        vals.append(v)
        rows.append(rows[-1] + len(i))
    return (np.array(rows, np.uint32),
            np.concatenate(idxs) if idxs else np.zeros(0, np.uint32),
            np.concatenate(vals) if vals else np.zeros(0, np.float32))


class Encoder:
    """The learned-proposal MLP on the GPU (wlda_encoder_*)."""

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")

    def __init__(self, buckets, hidden, K, max_batch=256, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, device="cuda:0", stream=None):
        import torch
        L = load_library()
        self.p = EncoderParams(buckets, hidden, K, max_batch, lr, beta1, beta2, eps)
        self.buckets, self.hidden, self.K, self.max_batch = buckets, hidden, K, max_batch
        n = C.c_uint64(0)
        _check("wlda_encoder_workspace_bytes",
               L.wlda_encoder_workspace_bytes(C.byref(self.p), C.byref(n)))
        self.device = torch.device(device)
        self.workspace = torch.empty(int(n.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p(0)
        _check("wlda_encoder_create",
               L.wlda_encoder_create(C.byref(self.p), C.c_void_p(self.workspace.data_ptr()),
                                     int(n.value), C.c_void_p(self.stream.cuda_stream),
                                     C.byref(h)))
        self.h = h

    def shapes(self):
        H, Hd, K = self.buckets, self.hidden, self.K
        return [(H, Hd), (Hd,), (Hd, Hd), (Hd,), (Hd, K), (K,)]

    def close(self):
        if getattr(self, "h", None):
            load_library().wlda_encoder_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, ws):
        arrs = [np.ascontiguousarray(w, np.float32) for w in ws]
        ptrs = (C.c_void_p * 6)(*[a.ctypes.data for a in arrs])
        _check("wlda_encoder_set_weights", load_library().wlda_encoder_set_weights(self.h, ptrs))

    def get_weights(self):
        arrs = [np.empty(s, np.float32) for s in self.shapes()]
        ptrs = (C.c_void_p * 6)(*[a.ctypes.data for a in arrs])
        _check("wlda_encoder_get_weights", load_library().wlda_encoder_get_weights(self.h, ptrs))
        return arrs

    @staticmethod
    def _dev(t):
        return C.c_void_p(t.data_ptr())

    def forward(self, rowptr, idx, val):
        """rowptr/idx/val: torch tensors on the device; returns probs (B x K)."""
        import torch
        B = rowptr.numel() - 1
        probs = torch.empty((B, self.K), dtype=torch.float32, device=self.device)
        _check("wlda_encoder_forward",
               load_library().wlda_encoder_forward(self.h, B, self._dev(rowptr), self._dev(idx),
                                                   self._dev(val), self._dev(probs)))
        return probs

    def proposal(self, probs, eps=0.01):
        import torch
        B = probs.shape[0]
        cdf = torch.empty((B, self.K), dtype=torch.int32, device=self.device)
        _check("wlda_encoder_proposal",
               load_library().wlda_encoder_proposal(self.h, B, self._dev(probs), eps,
                                                    self._dev(cdf)))
        return cdf

    def gradients(self, rowptr, idx, val, theta):
        B = rowptr.numel() - 1
        grads = [np.empty(s, np.float32) for s in self.shapes()]
        ptrs = (C.c_void_p * 6)(*[g.ctypes.data for g in grads])
        loss = C.c_float(0)
        _check("wlda_encoder_gradients",
               load_library().wlda_encoder_gradients(self.h, B, self._dev(rowptr), self._dev(idx),
                                                     self._dev(val), self._dev(theta),
                                                     C.byref(loss), ptrs))
        return float(loss.value), grads

    def train_step(self, rowptr, idx, val, theta, want_loss=True):
        B = rowptr.numel() - 1
        loss = C.c_float(0)
        _check("wlda_encoder_train_step",
               load_library().wlda_encoder_train_step(self.h, B, self._dev(rowptr), self._dev(idx),
                                                      self._dev(val), self._dev(theta),
                                                      C.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None


class Server:
    """Continuous-batching fold-in server (wlda_server_*)."""

    def __init__(self, model, encoder=None, max_docs=256, pool_tokens=1 << 20,
                 pool_heldout=1 << 20, sweeps=10, learned_steps=2, eps=0.01, stream=None):
        import torch
        L = load_library()
        self.model, self.encoder = model, encoder
        self.sp = ServerParams(max_docs, pool_tokens, pool_heldout, sweeps, learned_steps, eps)
        n = C.c_uint64(0)
        eh = encoder.h if encoder is not None else None
        _check("wlda_server_workspace_bytes",
               L.wlda_server_workspace_bytes(model.h, eh, C.byref(self.sp), C.byref(n)))
        self.workspace = torch.empty(int(n.value), dtype=torch.uint8, device=model.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(model.device)
        h = C.c_void_p(0)
        _check("wlda_server_create",
               L.wlda_server_create(model.h, eh, C.byref(self.sp),
                                    C.c_void_p(self.workspace.data_ptr()), int(n.value),
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load_library().wlda_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def now(self) -> float:
        t = C.c_double(0)
        _check("wlda_server_now", load_library().wlda_server_now(self.h, C.byref(t)))
        return t.value

    def submit(self, req_id, words, heldout=None, arrival=None, weights=None):
        w = np.ascontiguousarray(words, np.uint32)
        ho = np.ascontiguousarray(heldout if heldout is not None else [], np.uint32)
        wt = None if weights is None else np.ascontiguousarray(weights, np.uint32)
        t = self.now() if arrival is None else float(arrival)
        _check("wlda_server_submit",
               load_library().wlda_server_submit(self.h, req_id, _ptr(w), len(w),
                                                 _ptr(ho) if len(ho) else None, len(ho), t,
                                                 None if wt is None else _ptr(wt)))

    def step(self):
        a, p = C.c_uint32(0), C.c_uint32(0)
        _check("wlda_server_step", load_library().wlda_server_step(self.h, C.byref(a), C.byref(p)))
        return int(a.value), int(p.value)

    def poll(self, max_results=4096):
        arr = (Result * max_results)()
        n = C.c_uint32(0)
        _check("wlda_server_poll", load_library().wlda_server_poll(self.h, arr, max_results,
                                                                   C.byref(n)))
        return [dict(req_id=r.req_id, n_tokens=r.n_tokens, n_heldout=r.n_heldout,
                     sweeps=r.sweeps, learned=bool(r.learned), arrival_s=r.arrival_s,
                     admit_s=r.admit_s, done_s=r.done_s, heldout_ll=r.heldout_ll)
                for r in arr[:n.value]]

    def take_z(self, req_id, L):
        z = np.empty(L, np.int32)
        _check("wlda_server_take_z", load_library().wlda_server_take_z(self.h, req_id, _ptr(z), L))
        return z
