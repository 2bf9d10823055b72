"""ctypes binding of the FeLoG C ABI (include/felog.h).

Argument marshalling only: every step of the method runs in the HIP library
``_lib/libfelog.so``.  Loading fails loudly when the library has not been
built; there is no fallback.

The raw entry points keep the C names (``felog_walks_generate`` ...); the small
classes below own handles and free them.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfelog.so")

FELOG_OK, FELOG_EINVAL, FELOG_ENOMEM, FELOG_EDEVICE, FELOG_ESTATE, FELOG_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5
FELOG_EIO = -6
FELOG_EFAULT_INJECTED = -7
WALK_UNIFORM, WALK_NODE2VEC = 0, 1
NEG_DEGREE, NEG_UNIGRAM = 0, 1
TABLE_IN, TABLE_OUT = 0, 1
PREC_FP32, PREC_BF16 = 0, 1
FEEDBACK_MONOTONE, FEEDBACK_RECOMPUTE_ALL = 0, 1
FABC_MAX_SYMBOLS = 16
MAX_ROUNDS = 64

_STATUS = {0: "FELOG_OK", -1: "FELOG_EINVAL", -2: "FELOG_ENOMEM", -3: "FELOG_EDEVICE",
           -4: "FELOG_ESTATE", -5: "FELOG_EUNSUPPORTED", -6: "FELOG_EIO",
           -7: "FELOG_EFAULT_INJECTED"}


class FelogError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status
        self.message = message


class felog_walk_params(C.Structure):
    _fields_ = [("kind", C.c_int32), ("walks_per_node", C.c_int32), ("length", C.c_int32),
                ("p", C.c_float), ("q", C.c_float), ("seed", C.c_uint64),
                ("id_base", C.c_int64)]


class felog_model_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("neg_dist", C.c_int32), ("seed", C.c_uint64),
                ("precision", C.c_int32)]


class felog_train_params(C.Structure):
    _fields_ = [("window", C.c_int32), ("negatives", C.c_int32), ("lr_start", C.c_float),
                ("lr_end", C.c_float), ("minibatch_pairs", C.c_int64),
                ("chunk_walks", C.c_int64), ("seed", C.c_uint64),
                ("shared_negatives", C.c_int32)]


class felog_train_stats(C.Structure):
    _fields_ = [("minibatches", C.c_int64), ("pairs", C.c_int64),
                ("minibatches_total", C.c_int64), ("loss", C.c_double), ("ms", C.c_double),
                ("rows_in", C.c_int64), ("rows_out", C.c_int64),
                ("timed_launches", C.c_int64), ("ms_forward", C.c_double),
                ("ms_apply", C.c_double), ("ms_prep", C.c_double),
                ("ms_apply_first", C.c_double), ("rows_out_single", C.c_int64),
                ("path", C.c_int32), ("update_blocks", C.c_int32),
                ("timed_minibatches", C.c_int64), ("ms_update", C.c_double),
                ("us_phase", C.c_double * 4)]


class felog_feedback_params(C.Structure):
    _fields_ = [("mu", C.c_double), ("k_s", C.c_int32), ("mode", C.c_int32),
                ("seed", C.c_uint64), ("round", C.c_uint32)]


class felog_checkpoint_meta(C.Structure):
    _fields_ = [("round", C.c_uint32), ("walk_id_base", C.c_int64)]


class felog_run_params(C.Structure):
    _fields_ = [("walk", felog_walk_params), ("train", felog_train_params),
                ("feedback", felog_feedback_params), ("max_rounds", C.c_int32)]


class felog_run_stats(C.Structure):
    _fields_ = [("rounds", C.c_int32),
                ("active", C.c_int64 * MAX_ROUNDS), ("walks", C.c_int64 * MAX_ROUNDS),
                ("walk_steps", C.c_int64 * MAX_ROUNDS), ("ms_walk", C.c_double * MAX_ROUNDS),
                ("ms_feedback", C.c_double * MAX_ROUNDS),
                ("train", felog_train_stats * MAX_ROUNDS), ("final_active", C.c_int64)]


class felog_server_params(C.Structure):
    _fields_ = [("slots", C.c_int32), ("minibatch_pairs", C.c_int64), ("negatives", C.c_int32),
                ("lr_start", C.c_float), ("lr_end", C.c_float), ("update_mode", C.c_int32)]


class felog_job_desc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("nnz", C.c_int64), ("indptr", C.c_void_p),
                ("indices", C.c_void_p), ("dim", C.c_int32), ("walks_per_node", C.c_int32),
                ("walk_length", C.c_int32), ("window", C.c_int32), ("seed", C.c_uint64),
                ("arrival_time", C.c_double)]


class felog_job_state(C.Structure):
    _fields_ = [("state", C.c_int32), ("t_arrive", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("pairs", C.c_int64), ("loss", C.c_double),
                ("device_bytes", C.c_uint64), ("minibatch_pairs", C.c_int64),
                ("peak_bytes", C.c_uint64)]


JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3
SERVE_LAUNCHES, SERVE_PERSISTENT, SERVE_SHARED = 0, 1, 2

_p = C.c_void_p
_pp = C.POINTER(C.c_void_p)
_i32, _i64, _u32, _u64, _f32, _f64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float, C.c_double

# name -> (restype, argtypes); the names and order follow include/felog.h
SIGNATURES = {
    "felog_ctx_create": (_i32, [C.c_int, _p, _u64, _pp]),
    "felog_ctx_destroy": (None, [_p]),
    "felog_ctx_bytes_in_use": (_i32, [_p, C.POINTER(_u64)]),
    "felog_ctx_set_timing": (_i32, [_p, _i32]),
    "felog_ctx_set_sgns_path": (_i32, [_p, _i32, _i32]),
    "felog_ctx_set_single_stream": (_i32, [_p, _i32]),
    "felog_last_error": (C.c_char_p, []),
    "felog_graph_load_csr": (_i32, [_p, _i32, _i64, _p, _p, _p, _pp]),
    "felog_graph_destroy": (None, [_p]),
    "felog_graph_info": (_i32, [_p, C.POINTER(_i32), C.POINTER(_i64), C.POINTER(_i32)]),
    "felog_active_from_host": (_i32, [_p, _p, _i64, _pp]),
    "felog_active_all": (_i32, [_p, _pp]),
    "felog_active_count": (_i32, [_p, C.POINTER(_i64)]),
    "felog_active_read": (_i32, [_p, _p, _i64, C.POINTER(_i64)]),
    "felog_active_destroy": (None, [_p]),
    "felog_walks_generate": (_i32, [_p, C.POINTER(felog_walk_params), _p, _pp]),
    "felog_walks_info": (_i32, [_p, C.POINTER(_i64), C.POINTER(_i32), C.POINTER(_i64)]),
    "felog_walks_read": (_i32, [_p, _p, _i64]),
    "felog_walks_read_range": (_i32, [_p, _i64, _i64, _p, _i64]),
    "felog_walks_capped": (_i32, [_p, C.POINTER(_i64)]),
    "felog_walks_destroy": (None, [_p]),
    "felog_fabc_profile": (_i32, [_p, _i32, C.POINTER(_i32), _p, _p, C.POINTER(_i32),
                                  C.POINTER(C.c_uint64)]),
    "felog_walks_pack": (_i32, [_p, _i32, _p, C.POINTER(_p), _p]),
    "felog_packed_info": (_i32, [_p, C.POINTER(_i64), C.POINTER(_i32), C.POINTER(_i64),
                                 C.POINTER(_i32), C.POINTER(_i64)]),
    "felog_packed_read": (_i32, [_p, _p, _i64]),
    "felog_packed_from_host": (_i32, [_p, _p, _i64, C.POINTER(_p)]),
    "felog_packed_unpack": (_i32, [_p, C.POINTER(_p), _p]),
    "felog_packed_destroy": (None, [_p]),
    "felog_model_create": (_i32, [_p, C.POINTER(felog_model_params), _pp]),
    "felog_model_destroy": (None, [_p]),
    "felog_model_set_unigram": (_i32, [_p, _p]),
    "felog_model_read_cdf": (_i32, [_p, _p, _i64]),
    "felog_model_info": (_i32, [_p, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32),
                                C.POINTER(_i32)]),
    "felog_model_save": (_i32, [_p, _p, C.POINTER(felog_checkpoint_meta), C.c_char_p]),
    "felog_model_load": (_i32, [_p, C.c_char_p, _pp, _pp, C.POINTER(felog_checkpoint_meta)]),
    "felog_model_reset": (_i32, [_p, _u64]),
    "felog_embeddings_read": (_i32, [_p, _i32, _p, _i64]),
    "felog_embeddings_read_dev": (_i32, [_p, _i32, _p, _i64]),
    "felog_embeddings_read_bf16": (_i32, [_p, _i32, _p, _i64]),
    "felog_embeddings_write": (_i32, [_p, _i32, _p, _i64]),
    "felog_train_epoch": (_i32, [_p, _p, C.POINTER(felog_train_params),
                                 C.POINTER(felog_train_stats)]),
    "felog_train_steps": (_i32, [_p, _p, C.POINTER(felog_train_params), _i64, _i64,
                                 C.POINTER(felog_train_stats)]),
    "felog_train_delta": (_i32, [_p, _p, C.POINTER(felog_train_params), _i64,
                                 _p, _p, _i64, C.POINTER(_i64), _p, _p, _i64, C.POINTER(_i64),
                                 C.POINTER(_f64)]),
    "felog_feedback": (_i32, [_p, C.POINTER(felog_feedback_params), _p, _pp, _p, _i64]),
    "felog_feedback_noalloc": (_i32, [_p, C.POINTER(felog_feedback_params), _p, _i64, _p, _i64,
                                      _p, _i64, C.POINTER(_i64)]),
    "felog_run": (_i32, [_p, C.POINTER(felog_run_params), C.POINTER(felog_run_stats)]),
    "felog_server_create": (_i32, [C.c_int, _u64, C.POINTER(felog_server_params), _pp]),
    "felog_server_submit": (_i32, [_p, C.POINTER(felog_job_desc), C.POINTER(_u64)]),
    "felog_server_poll": (_i32, [_p, _u64, C.POINTER(felog_job_state)]),
    "felog_server_wait": (_i32, [_p, _u64, _f64, C.POINTER(felog_job_state)]),
    "felog_server_fetch": (_i32, [_p, _u64, _p, _i64]),
    "felog_server_release": (_i32, [_p, _u64]),
    "felog_server_stats": (_i32, [_p, C.POINTER(_f64), C.POINTER(_u64), C.POINTER(_i64)]),
    "felog_server_destroy": (None, [_p]),
}

_lib = None


def load() -> C.CDLL:
    """Load libfelog.so (built in-tree by paper_2606_22180_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfelog.so is not built (%s); run "
                              "`python -m paper_2606_22180_amd.build`" % LIB_PATH)
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != FELOG_OK:
        raise FelogError(status, load().felog_last_error().decode())


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


class Context:
    """A device + stream binding (felog_ctx).

    ``stream`` is a hipStream_t handle as an int (e.g. torch's
    ``torch.cuda.current_stream().cuda_stream``) or None for the null stream.
    A process that also uses torch on the GPU must import torch before this
    module loads the library, so that both share torch's HIP runtime."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        lib = load()
        self.handle = None
        self._live = 0                # objects created on this context, not yet destroyed
        self._close_pending = False
        h = C.c_void_p()
        _check(lib.felog_ctx_create(device, stream, hbm_budget, C.byref(h)))
        self.handle = h

    def set_timing(self, every: int):
        _check(load().felog_ctx_set_timing(self.handle, every))

    def set_sgns_path(self, path: int, blocks: int = 0):
        """0: persistent small-minibatch update where it applies; 1: per-minibatch
        launches always.  blocks: workgroups of the persistent launch (0 = the
        default, 64)."""
        _check(load().felog_ctx_set_sgns_path(self.handle, path, blocks))

    def set_single_stream(self, on: bool):
        """Every launch of the context on its one stream (for profilers)."""
        _check(load().felog_ctx_set_single_stream(self.handle, 1 if on else 0))

    def bytes_in_use(self) -> int:
        b = C.c_uint64()
        _check(load().felog_ctx_bytes_in_use(self.handle, C.byref(b)))
        return b.value

    def close(self):
        """Destroy the context.  The C library needs every object of a context
        destroyed first; while some are alive (the garbage collector may
        finalise a context before the objects of the same reference cycle),
        the destruction waits for the last of them."""
        if not self.handle:
            return
        if self._live > 0:
            self._close_pending = True
            return
        load().felog_ctx_destroy(self.handle)
        self.handle = None

    def _child_closed(self):
        self._live -= 1
        if self._live == 0 and self._close_pending:
            self._close_pending = False
            self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Handle:
    _destroy = ""

    def __init__(self, handle, owner):
        self.handle = None
        self._owner = owner          # keeps the context (and graph) alive
        self._ctx = owner if isinstance(owner, Context) else owner._ctx
        self._ctx._live += 1
        self.handle = handle

    def close(self):
        if self.handle:
            getattr(load(), self._destroy)(self.handle)
            self.handle = None
            self._ctx._child_closed()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph(_Handle):
    _destroy = "felog_graph_destroy"

    @classmethod
    def from_csr(cls, ctx: Context, indptr, indices, weights=None) -> "Graph":
        ip, ipp = _arr(indptr, np.int64)
        ix, ixp = _arr(indices, np.int32)
        wp = None
        if weights is not None:
            w, wp = _arr(weights, np.float32)
        n = ip.shape[0] - 1
        h = C.c_void_p()
        _check(load().felog_graph_load_csr(ctx.handle, n, ix.shape[0], ipp, ixp, wp, C.byref(h)))
        g = cls(h, ctx)
        g.n = n
        g.nnz = int(ix.shape[0])
        return g


class Active(_Handle):
    _destroy = "felog_active_destroy"

    @classmethod
    def from_host(cls, g: Graph, nodes) -> "Active":
        a, ap = _arr(nodes, np.int32)
        h = C.c_void_p()
        _check(load().felog_active_from_host(g.handle, ap, a.shape[0], C.byref(h)))
        return cls(h, g)

    @classmethod
    def all(cls, g: Graph) -> "Active":
        h = C.c_void_p()
        _check(load().felog_active_all(g.handle, C.byref(h)))
        return cls(h, g)

    def count(self) -> int:
        c = C.c_int64()
        _check(load().felog_active_count(self.handle, C.byref(c)))
        return c.value

    def read(self) -> np.ndarray:
        n = self.count()
        out = np.zeros(max(n, 1), np.int32)
        c = C.c_int64()
        _check(load().felog_active_read(self.handle, out.ctypes.data, out.shape[0], C.byref(c)))
        return out[:c.value]


class Walks(_Handle):
    _destroy = "felog_walks_destroy"

    @classmethod
    def generate(cls, g: Graph, *, r: int, L: int, seed: int, id_base: int = 0,
                 kind: int = WALK_UNIFORM, p: float = 1.0, q: float = 1.0,
                 starts: Active | None = None) -> "Walks":
        prm = felog_walk_params(kind, r, L, p, q, seed, id_base)
        h = C.c_void_p()
        _check(load().felog_walks_generate(g.handle, C.byref(prm),
                                           starts.handle if starts else None, C.byref(h)))
        return cls(h, g)

    def info(self):
        W, L, b = C.c_int64(), C.c_int32(), C.c_int64()
        _check(load().felog_walks_info(self.handle, C.byref(W), C.byref(L), C.byref(b)))
        return W.value, L.value, b.value

    def read(self) -> np.ndarray:
        W, L, _ = self.info()
        out = np.zeros((max(W, 1), L), np.int32)
        _check(load().felog_walks_read(self.handle, out.ctypes.data, out.size))
        return out[:W]

    def read_range(self, first: int, count: int) -> np.ndarray:
        """Walks first .. first + count - 1, walk-major [count][L]."""
        _, L, _ = self.info()
        out = np.zeros((max(count, 1), L), np.int32)
        _check(load().felog_walks_read_range(self.handle, first, count, out.ctypes.data,
                                             out.size))
        return out[:count]

    def capped(self) -> int:
        c = C.c_int64()
        _check(load().felog_walks_capped(self.handle, C.byref(c)))
        return c.value

    def fabc_profile(self, k_max: int = FABC_MAX_SYMBOLS):
        """(k, ranked symbols, their counts, total positions): the codec's profile."""
        k, m, tot = C.c_int32(), C.c_int32(), C.c_uint64()
        sym = np.zeros(FABC_MAX_SYMBOLS, np.int32)
        cnt = np.zeros(FABC_MAX_SYMBOLS, np.uint64)
        _check(load().felog_fabc_profile(self.handle, k_max, C.byref(k), sym.ctypes.data,
                                         cnt.ctypes.data, C.byref(m), C.byref(tot)))
        return k.value, sym[:m.value].copy(), cnt[:m.value].copy(), tot.value

    def pack(self, symbols) -> "Packed":
        s, sp = _arr(np.asarray(symbols, np.int32).reshape(-1), np.int32)
        h = C.c_void_p()
        ms = np.zeros(2, np.float64)
        _check(load().felog_walks_pack(self.handle, s.shape[0], sp if s.shape[0] else None,
                                       C.byref(h), ms.ctypes.data))
        pk = Packed(h, self._owner)
        pk.ms = (float(ms[0]), float(ms[1]))
        return pk


class Packed(_Handle):
    """A walk corpus in the codec's byte format, in device memory."""
    _destroy = "felog_packed_destroy"

    @classmethod
    def from_host(cls, g: Graph, data: bytes) -> "Packed":
        b = np.frombuffer(data, np.uint8)
        h = C.c_void_p()
        _check(load().felog_packed_from_host(g.handle, b.ctypes.data, b.shape[0], C.byref(h)))
        return cls(h, g)

    def info(self):
        """(bytes, k, walks, length, residual positions)."""
        by, k, W, L, R = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int32(), C.c_int64()
        _check(load().felog_packed_info(self.handle, C.byref(by), C.byref(k), C.byref(W),
                                        C.byref(L), C.byref(R)))
        return by.value, k.value, W.value, L.value, R.value

    def read(self) -> bytes:
        n = self.info()[0]
        out = np.zeros(max(n, 1), np.uint8)
        _check(load().felog_packed_read(self.handle, out.ctypes.data, out.shape[0]))
        return out[:n].tobytes()

    def unpack(self) -> Walks:
        h = C.c_void_p()
        ms = np.zeros(1, np.float64)
        _check(load().felog_packed_unpack(self.handle, C.byref(h), ms.ctypes.data))
        w = Walks(h, self._owner)
        w.unpack_ms = float(ms[0])
        return w


def train_params(*, window, negatives, lr_start=0.025, lr_end=1e-4, minibatch_pairs,
                 chunk_walks=0, seed=0, shared_negatives=0) -> felog_train_params:
    return felog_train_params(window, negatives, lr_start, lr_end, minibatch_pairs,
                              chunk_walks, seed, shared_negatives)


class Model(_Handle):
    _destroy = "felog_model_destroy"

    @classmethod
    def create(cls, g: Graph, *, dim: int, neg_dist: int = NEG_DEGREE, seed: int = 0,
               precision: int = PREC_FP32) -> "Model":
        prm = felog_model_params(dim, neg_dist, seed, precision)
        h = C.c_void_p()
        _check(load().felog_model_create(g.handle, C.byref(prm), C.byref(h)))
        m = cls(h, g)
        m.n = g.n
        m.dim = dim
        return m

    def save(self, path: str, *, active: Active | None = None, round: int = 0,
             walk_id_base: int = 0):
        """Tables, noise table, active list and round metadata to `path`."""
        meta = felog_checkpoint_meta(round, walk_id_base)
        _check(load().felog_model_save(self.handle, active.handle if active else None,
                                       C.byref(meta), os.fsencode(path)))

    @classmethod
    def load(cls, g: Graph, path: str):
        """(model, active list or None, round, walk_id_base) from a checkpoint."""
        h, a = C.c_void_p(), C.c_void_p()
        meta = felog_checkpoint_meta()
        _check(load().felog_model_load(g.handle, os.fsencode(path), C.byref(h), C.byref(a),
                                       C.byref(meta)))
        m = cls(h, g)
        n, d, neg, prec = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().felog_model_info(m.handle, C.byref(n), C.byref(d), C.byref(neg),
                                       C.byref(prec)))
        m.n, m.dim, m.neg_dist, m.precision = n.value, d.value, neg.value, prec.value
        act = Active(a, g) if a.value else None
        return m, act, meta.round, meta.walk_id_base

    def set_unigram(self, corpus: Walks):
        _check(load().felog_model_set_unigram(self.handle, corpus.handle))

    def reset(self, seed: int):
        _check(load().felog_model_reset(self.handle, seed))

    def read_cdf(self) -> np.ndarray:
        out = np.zeros(self.n + 1, np.uint64)
        _check(load().felog_model_read_cdf(self.handle, out.ctypes.data, out.shape[0]))
        return out

    def read(self, which: int = TABLE_IN) -> np.ndarray:
        out = np.zeros((self.n, self.dim), np.float32)
        _check(load().felog_embeddings_read(self.handle, which, out.ctypes.data, out.size))
        return out

    def read_bf16(self, which: int = TABLE_IN) -> np.ndarray:
        out = np.zeros((self.n, self.dim), np.uint16)
        _check(load().felog_embeddings_read_bf16(self.handle, which, out.ctypes.data, out.size))
        return out

    def read_dev(self, which: int, ptr: int, cap: int):
        _check(load().felog_embeddings_read_dev(self.handle, which, ptr, cap))

    def write(self, which: int, values):
        v, vp = _arr(values, np.float32)
        _check(load().felog_embeddings_write(self.handle, which, vp, v.size))

    def train_epoch(self, corpus: Walks, prm: felog_train_params) -> felog_train_stats:
        st = felog_train_stats()
        _check(load().felog_train_epoch(self.handle, corpus.handle, C.byref(prm), C.byref(st)))
        return st

    def train_steps(self, corpus: Walks, prm: felog_train_params, first_mb: int,
                    n_mb: int) -> felog_train_stats:
        st = felog_train_stats()
        _check(load().felog_train_steps(self.handle, corpus.handle, C.byref(prm), first_mb, n_mb,
                                        C.byref(st)))
        return st

    def train_delta(self, corpus: Walks, prm: felog_train_params, mb: int):
        """Deltas of one minibatch, not applied: (rows_in, d_in, rows_out, d_out, loss)."""
        P = prm.minibatch_pairs
        K = prm.negatives
        ri = np.zeros(P, np.int32)
        di = np.zeros((P, self.dim), np.float32)
        ro = np.zeros(P * (K + 1), np.int32)
        do = np.zeros((P * (K + 1), self.dim), np.float32)
        ni, no, loss = C.c_int64(), C.c_int64(), C.c_double()
        _check(load().felog_train_delta(self.handle, corpus.handle, C.byref(prm), mb,
                                        ri.ctypes.data, di.ctypes.data, P, C.byref(ni),
                                        ro.ctypes.data, do.ctypes.data, P * (K + 1), C.byref(no),
                                        C.byref(loss)))
        a, b = ni.value, no.value
        return ri[:a], di[:a], ro[:b], do[:b], loss.value

    def feedback(self, *, mu: float, k_s: int, seed: int, round: int,
                 mode: int = FEEDBACK_MONOTONE, active: Active | None = None,
                 want_psi: bool = False):
        prm = felog_feedback_params(mu, k_s, mode, seed, round)
        h = C.c_void_p()
        n_scored = self.n if (active is None or mode == FEEDBACK_RECOMPUTE_ALL) else active.count()
        psi = np.zeros(max(1, n_scored), np.float64) if want_psi else None
        _check(load().felog_feedback(self.handle, C.byref(prm),
                                     active.handle if active else None, C.byref(h),
                                     psi.ctypes.data if want_psi else None,
                                     psi.shape[0] if want_psi else 0))
        nxt = Active(h, self._owner)
        return (nxt, psi[:n_scored]) if want_psi else nxt

    def feedback_noalloc(self, *, mu: float, k_s: int, seed: int, round: int,
                         in_nodes_dev: int | None, count: int, out_nodes_dev: int, out_cap: int,
                         psi_dev: int, psi_cap: int, mode: int = FEEDBACK_MONOTONE) -> int:
        """felog_feedback_noalloc on caller-owned device buffers (raw device
        addresses); returns the number of kept nodes."""
        prm = felog_feedback_params(mu, k_s, mode, seed, round)
        n = C.c_int64()
        _check(load().felog_feedback_noalloc(self.handle, C.byref(prm), in_nodes_dev, count,
                                             out_nodes_dev, out_cap, psi_dev, psi_cap,
                                             C.byref(n)))
        return n.value

    def run(self, prm: felog_run_params) -> felog_run_stats:
        st = felog_run_stats()
        _check(load().felog_run(self.handle, C.byref(prm), C.byref(st)))
        return st


class Server:
    """Continuous-admission serving loop (felog_server)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, *, slots: int = 4,
                 minibatch_pairs: int = 65536, negatives: int = 5, lr_start: float = 0.025,
                 lr_end: float = 1e-4, update_mode: int = 0):
        prm = felog_server_params(slots, minibatch_pairs, negatives, lr_start, lr_end,
                                  update_mode)
        h = C.c_void_p()
        _check(load().felog_server_create(device, hbm_budget, C.byref(prm), C.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, indptr, indices, *, dim, r, L, window, seed, arrival_time=0.0) -> int:
        ip, ipp = _arr(indptr, np.int64)
        ix, ixp = _arr(indices, np.int32)
        d = felog_job_desc(ip.shape[0] - 1, ix.shape[0], ipp, ixp, dim, r, L, window, seed,
                           arrival_time)
        jid = C.c_uint64()
        _check(load().felog_server_submit(self.handle, C.byref(d), C.byref(jid)))
        self._keep[jid.value] = (ip.shape[0] - 1, dim)
        return jid.value

    def poll(self, jid: int) -> felog_job_state:
        st = felog_job_state()
        _check(load().felog_server_poll(self.handle, jid, C.byref(st)))
        return st

    def wait(self, jid: int, timeout: float = -1.0) -> felog_job_state:
        st = felog_job_state()
        _check(load().felog_server_wait(self.handle, jid, timeout, C.byref(st)))
        return st

    def fetch(self, jid: int) -> np.ndarray:
        n, dim = self._keep[jid]
        out = np.zeros((n, dim), np.float32)
        _check(load().felog_server_fetch(self.handle, jid, out.ctypes.data, out.size))
        return out

    def release(self, jid: int):
        _check(load().felog_server_release(self.handle, jid))
        self._keep.pop(jid, None)

    def stats(self):
        c, pk, q = C.c_double(), C.c_uint64(), C.c_int64()
        _check(load().felog_server_stats(self.handle, C.byref(c), C.byref(pk), C.byref(q)))
        return c.value, pk.value, q.value

    def close(self):
        """Finish the running jobs and stop the server's threads."""
        if getattr(self, "handle", None):
            load().felog_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
