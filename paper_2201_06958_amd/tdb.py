"""ctypes binding of the C ABI in include/tdb.h (argument marshalling only).

Every numerical step runs inside libtdb.so on the GPU; this module only converts
Python arguments to the C structs, passes torch device pointers and streams, and
raises TDBError on a non-zero status. If the library is missing it raises at
load time instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdb.so")

MAX_ORDER = 8
SIGMA_K = 16

OK, EINVAL, ENOMEM, EHIP, ESTATE, ENUMERIC, EUNSUPPORTED = range(7)
F64, F32 = 0, 1
PREC_F64, PREC_F32, PREC_BF16SPLIT = 0, 1, 2
PATH_AUTO, PATH_PLAIN, PATH_FUSED = 0, 1, 2
INT_HEUN, INT_EULER = 0, 1
COPY, BORROW = 0, 1
EVENTS = {0: "", 1: "reinit", 2: "add", 3: "remove", 4: "numeric"}

_STATUS = {1: "TDB_EINVAL", 2: "TDB_ENOMEM", 3: "TDB_EHIP", 4: "TDB_ESTATE", 5: "TDB_ENUMERIC",
           6: "TDB_EUNSUPPORTED"}


class TDBError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class TdbConfig(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("dims", ctypes.c_int64 * MAX_ORDER),
        ("rank_init", ctypes.c_int32 * MAX_ORDER),
        ("rank_max", ctypes.c_int32 * MAX_ORDER),
        ("weights", ctypes.POINTER(ctypes.c_double) * MAX_ORDER),
        ("dt", ctypes.c_double),
        ("data_dtype", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("adaptive", ctypes.c_int32),
        ("snapshot_mode", ctypes.c_int32),
        ("eps_th", ctypes.c_double),
        ("gamma_th", ctypes.c_double),
        ("slope_window", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
        ("fd_order", ctypes.c_int32),
    ]


class TdbStats(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("t", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("nu", ctypes.c_double),
        ("eps_after", ctypes.c_double),
        ("ranks", ctypes.c_int32 * MAX_ORDER),
        ("event", ctypes.c_int32),
        ("sigma", (ctypes.c_double * SIGMA_K) * 4),
        ("cr", ctypes.c_double),
        ("crbar", ctypes.c_double),
        ("n_reinit", ctypes.c_int32),
        ("n_add", ctypes.c_int32),
        ("n_remove", ctypes.c_int32),
        ("n_numeric", ctypes.c_int32),
        ("gated", ctypes.c_int32),
        ("would_skip", ctypes.c_int32),
        ("eps_pred", ctypes.c_double),
        ("precision_used", ctypes.c_int32),
        ("path_used", ctypes.c_int32),
        ("fused_steps", ctypes.c_int64),
        ("plain_steps", ctypes.c_int64),
        ("n_nonfinite", ctypes.c_int64),
        ("graph_steps", ctypes.c_int64),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtdb.so and declare the C signatures. Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    H = ctypes.c_void_p
    P = ctypes.c_void_p
    lib.tdb_init.argtypes = [ctypes.POINTER(TdbConfig), P, P, ctypes.POINTER(H)]
    lib.tdb_init_from_factors.argtypes = [ctypes.POINTER(TdbConfig), P, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.POINTER(ctypes.c_double)), P,
                                          ctypes.POINTER(H)]
    lib.tdb_ingest_snapshot.argtypes = [H, P, P]
    lib.tdb_ingest_with_derivative.argtypes = [H, P, P, P]
    lib.tdb_flush.argtypes = [H]
    lib.tdb_get_core_and_bases.argtypes = [H, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.POINTER(ctypes.c_double))]
    lib.tdb_reconstruct.argtypes = [H, P, P]
    lib.tdb_set_threshold.argtypes = [H, ctypes.c_double, ctypes.c_double]
    lib.tdb_get_stats.argtypes = [H, ctypes.POINTER(TdbStats)]
    lib.tdb_destroy.argtypes = [H]
    lib.tdb_destroy.restype = None
    lib.tdb_last_error.argtypes = [H]
    lib.tdb_last_error.restype = ctypes.c_char_p
    lib.tdb_profile_enable.argtypes = [H, ctypes.c_int32]
    lib.tdb_profile_enable.restype = ctypes.c_int32
    lib.tdb_profile_read.argtypes = [H, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.tdb_profile_read.restype = ctypes.c_int32
    lib.tdb_reconstruct_noalloc.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int32), P, ctypes.POINTER(P), ctypes.c_int32, P,
                                            P]
    lib.tdb_reconstruct_noalloc.restype = ctypes.c_int32
    lib.tdb_struct_sizes.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.tdb_struct_sizes.restype = None
    lib.tdb_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(TdbConfig), ctypes.POINTER(P), P,
                                     ctypes.POINTER(H)]
    lib.tdb_batch_ingest.argtypes = [H, ctypes.POINTER(P), P]
    lib.tdb_batch_flush.argtypes = [H]
    lib.tdb_batch_plan.argtypes = [H, ctypes.POINTER(TdbBatchPlan)]
    lib.tdb_batch_stream.argtypes = [H, ctypes.c_int32, ctypes.POINTER(H)]
    lib.tdb_batch_profile_enable.argtypes = [H, ctypes.c_int32]
    lib.tdb_batch_profile_read.argtypes = [H, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.tdb_batch_gate_attach.argtypes = [H, H, ctypes.POINTER(ctypes.c_float), ctypes.c_int32]
    lib.tdb_gate_load.argtypes = [H, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                  ctypes.c_int32]
    F = ctypes.POINTER(ctypes.c_float)
    lib.tdb_gate_create.argtypes = [ctypes.c_int32, ctypes.POINTER(H)]
    lib.tdb_gate_set_params.argtypes = [H, F]
    lib.tdb_gate_get_params.argtypes = [H, F]
    lib.tdb_gate_forward.argtypes = [H, P, ctypes.c_int32, P, P]
    lib.tdb_gate_grad.argtypes = [H, P, P, ctypes.c_int32, P, F, P]
    lib.tdb_gate_train_step.argtypes = [H, P, P, ctypes.c_int32, ctypes.c_float, F, P]
    lib.tdb_gate_destroy.argtypes = [H]
    lib.tdb_gate_destroy.restype = None
    lib.tdb_gate_last_error.argtypes = [H]
    lib.tdb_gate_last_error.restype = ctypes.c_char_p
    lib.tdb_batch_destroy.argtypes = [H]
    lib.tdb_batch_destroy.restype = None
    lib.tdb_batch_last_error.argtypes = [H]
    lib.tdb_batch_last_error.restype = ctypes.c_char_p
    for name in ("tdb_init", "tdb_init_from_factors", "tdb_ingest_snapshot", "tdb_flush", "tdb_get_core_and_bases",
                 "tdb_reconstruct", "tdb_set_threshold", "tdb_get_stats", "tdb_batch_create",
                 "tdb_batch_ingest", "tdb_batch_flush", "tdb_batch_plan", "tdb_batch_stream",
                 "tdb_batch_profile_enable",
                 "tdb_batch_profile_read", "tdb_batch_gate_attach", "tdb_gate_load", "tdb_gate_create", "tdb_gate_set_params",
                 "tdb_gate_get_params", "tdb_gate_forward", "tdb_gate_grad", "tdb_gate_train_step"):
        getattr(lib, name).restype = ctypes.c_int32
    a, b = ctypes.c_int64(), ctypes.c_int64()
    lib.tdb_struct_sizes(ctypes.byref(a), ctypes.byref(b))
    if a.value != ctypes.sizeof(TdbConfig) or b.value != ctypes.sizeof(TdbStats):
        raise RuntimeError("tdb.h struct layout does not match the binding")
    _lib = lib
    return lib


def reconstruct_noalloc(C, U, out, stream=None):
    """tdb_reconstruct_noalloc: out (a contiguous float32 or float64 device tensor of
    the full shape) <- C x_1 U[0] ... from contiguous float64 device tensors C and U[n]
    (N_n x r_n), with no device allocation inside the library."""
    lib = load_library()
    p = C.dim()
    dims = (ctypes.c_int64 * MAX_ORDER)(*([int(u.shape[0]) for u in U] + [0] * (MAX_ORDER - p)))
    ranks = (ctypes.c_int32 * MAX_ORDER)(*([int(s) for s in C.shape] + [0] * (MAX_ORDER - p)))
    uptr = (ctypes.c_void_p * MAX_ORDER)(*([_dev_ptr(u).value for u in U] + [None] * (MAX_ORDER - p)))
    import torch
    dt = F32 if out.dtype == torch.float32 else F64
    st = lib.tdb_reconstruct_noalloc(p, dims, ranks, _dev_ptr(C), uptr, dt, _dev_ptr(out), _stream_ptr(stream))
    if st != OK:
        raise TDBError(st, (lib.tdb_last_error(None) or b"").decode())
    return out


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("snapshots must be contiguous device tensors")
    return ctypes.c_void_p(t.data_ptr())


class Compressor:
    """One streaming tensor compressed with time-dependent bases (see tdb.h)."""

    def __init__(self, dims: Sequence[int], dt: float, rank_max: Sequence[int],
                 rank_init: Optional[Sequence[int]] = None,
                 weights: Optional[Sequence[np.ndarray]] = None, data_dtype: str = "f32",
                 precision: str = "f32", path: str = "auto", adaptive: bool = True,
                 snapshot_mode: str = "copy", eps_th: float = 1e-4, gamma_th: float = 0.0,
                 slope_window: int = 0, integrator: str = "heun", fd_order: int = 1):
        self.lib = load_library()
        p = len(dims)
        self.dims = tuple(int(d) for d in dims)
        self.data_dtype = data_dtype
        cfg = TdbConfig()
        cfg.order = p
        for n in range(p):
            cfg.dims[n] = int(dims[n])
            cfg.rank_max[n] = int(rank_max[n])
            cfg.rank_init[n] = int(rank_init[n]) if rank_init is not None else 0
        self._w = []
        if weights is not None:
            for n in range(p):
                arr = np.ascontiguousarray(weights[n], dtype=np.float64)
                self._w.append(arr)
                cfg.weights[n] = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cfg.dt = float(dt)
        cfg.data_dtype = F32 if data_dtype == "f32" else F64
        cfg.precision = {"f64": PREC_F64, "f32": PREC_F32, "bf16s": PREC_BF16SPLIT}[precision]
        cfg.path = {"auto": PATH_AUTO, "plain": PATH_PLAIN, "fused": PATH_FUSED}[path]
        cfg.adaptive = 1 if adaptive else 0
        cfg.snapshot_mode = BORROW if snapshot_mode == "borrow" else COPY
        cfg.eps_th = float(eps_th)
        cfg.gamma_th = float(gamma_th)
        cfg.slope_window = int(slope_window)
        cfg.integrator = {"heun": INT_HEUN, "euler": INT_EULER}[integrator]
        cfg.fd_order = int(fd_order)
        self.cfg = cfg
        self.h = ctypes.c_void_p()

    # -- status handling
    def _check(self, status: int):
        if status != OK:
            msg = self.lib.tdb_last_error(self.h if self.h else None)
            raise TDBError(status, (msg or b"").decode())

    def init(self, V0, stream=None):
        st = self.lib.tdb_init(ctypes.byref(self.cfg), _dev_ptr(V0), _stream_ptr(stream),
                               ctypes.byref(self.h))
        self._check(st)
        return self

    def init_from_factors(self, V0, C: np.ndarray, U: List[np.ndarray], stream=None):
        ranks = (ctypes.c_int32 * MAX_ORDER)(*([int(s) for s in C.shape] + [0] * (MAX_ORDER - C.ndim)))
        Cc = np.ascontiguousarray(C, dtype=np.float64)
        Us = [np.ascontiguousarray(u, dtype=np.float64) for u in U]
        uptr = (ctypes.POINTER(ctypes.c_double) * MAX_ORDER)()
        for n, u in enumerate(Us):
            uptr[n] = u.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st = self.lib.tdb_init_from_factors(ctypes.byref(self.cfg), _dev_ptr(V0), ranks,
                                            Cc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), uptr,
                                            _stream_ptr(stream), ctypes.byref(self.h))
        self._check(st)
        return self

    def ingest(self, V, stream=None):
        self._check(self.lib.tdb_ingest_snapshot(self.h, _dev_ptr(V), _stream_ptr(stream)))

    def ingest_with_derivative(self, V, D, stream=None):
        """One step with the given data derivative D (same shape and dtype as V)."""
        self._check(self.lib.tdb_ingest_with_derivative(self.h, _dev_ptr(V), _dev_ptr(D), _stream_ptr(stream)))

    def flush(self):
        """Act on the newest enqueued step's decision (borrowed snapshots pipeline the
        ingest: a step's decision is otherwise read by the next call)."""
        self._check(self.lib.tdb_flush(self.h))

    def ranks(self):
        r = (ctypes.c_int32 * MAX_ORDER)()
        self._check(self.lib.tdb_get_core_and_bases(self.h, 0, r, None, None))
        return tuple(r[: len(self.dims)])

    def get_core_and_bases(self, rotate: bool = False):
        r = self.ranks()
        C = np.zeros(r, dtype=np.float64)
        Us = [np.zeros((self.dims[n], r[n]), dtype=np.float64) for n in range(len(r))]
        uptr = (ctypes.POINTER(ctypes.c_double) * MAX_ORDER)()
        for n, u in enumerate(Us):
            uptr[n] = u.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rr = (ctypes.c_int32 * MAX_ORDER)()
        self._check(self.lib.tdb_get_core_and_bases(self.h, 1 if rotate else 0, rr,
                                                    C.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                    uptr))
        return r, C, Us

    def reconstruct(self, out=None, stream=None):
        import torch
        if out is None:
            dt = torch.float32 if self.data_dtype == "f32" else torch.float64
            out = torch.empty(self.dims, dtype=dt, device="cuda")
        self._check(self.lib.tdb_reconstruct(self.h, _dev_ptr(out), _stream_ptr(stream)))
        return out

    def set_threshold(self, eps_th: float, gamma_th: float = 0.0):
        self._check(self.lib.tdb_set_threshold(self.h, float(eps_th), float(gamma_th)))

    def stats(self) -> dict:
        s = TdbStats()
        self._check(self.lib.tdb_get_stats(self.h, ctypes.byref(s)))
        p = len(self.dims)
        return {
            "step": s.step, "t": s.t, "eps": s.eps, "nu": s.nu, "eps_after": s.eps_after,
            "ranks": tuple(s.ranks[:p]), "event": EVENTS.get(s.event, str(s.event)),
            "sigma": [list(s.sigma[n][: s.ranks[n]]) for n in range(p)], "cr": s.cr,
            "crbar": s.crbar, "n_reinit": s.n_reinit, "n_add": s.n_add, "n_remove": s.n_remove,
            "n_numeric": s.n_numeric, "gated": bool(s.gated), "would_skip": bool(s.would_skip),
            "eps_pred": s.eps_pred,
            "sigma16": [list(s.sigma[n][:SIGMA_K]) for n in range(p)],
            "precision_used": {-1: None, PREC_F64: "f64", PREC_F32: "f32",
                               PREC_BF16SPLIT: "bf16s"}.get(s.precision_used),
            "path_used": {0: None, PATH_PLAIN: "plain", PATH_FUSED: "fused"}.get(s.path_used),
            "fused_steps": s.fused_steps, "plain_steps": s.plain_steps, "n_nonfinite": s.n_nonfinite,
            "graph_steps": s.graph_steps,
        }

    def gate_load(self, params=None, mean_std=None, mode: str = "active"):
        """Copy a trained gate (TDB_GATE_PARAMS floats) and its feature statistics (768
        floats: means, then standard deviations) into this stream. mode: off | record |
        active | shadow."""
        mid = {"off": 0, "record": 1, "active": 2, "shadow": 3}[mode]
        pp = ms = None
        n = 0
        if params is not None:
            self._gp = np.ascontiguousarray(params, dtype=np.float32)
            pp = self._gp.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            n = int(self._gp.size)
        if mean_std is not None:
            self._gms = np.ascontiguousarray(mean_std, dtype=np.float32)
            ms = self._gms.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._check(self.lib.tdb_gate_load(self.h, pp, ms, n, mid))

    def profile_enable(self, on: bool = True, every: int = 1):
        """Pass timing: every launch (every=1) or the passes of every `every`-th step."""
        self._check(self.lib.tdb_profile_enable(self.h, max(1, int(every)) if on else 0))

    def profile_read(self, pass_name: str = "project") -> dict:
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        pid = {"project": 0, "error": 1}[pass_name]
        self._check(self.lib.tdb_profile_read(self.h, pid, ctypes.byref(n), ctypes.byref(ms),
                                              ctypes.byref(by)))
        return {"launches": n.value, "total_ms": ms.value, "bytes_per_launch": by.value}

    def close(self):
        if self.h and not getattr(self, "_borrowed", False):
            self.lib.tdb_destroy(self.h)
        self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TdbBatchPlan(ctypes.Structure):
    _fields_ = [("pass_kind", ctypes.c_int32), ("pass_cols", ctypes.c_int32), ("err_kind", ctypes.c_int32),
                ("source", ctypes.c_int32), ("pass_us", ctypes.c_double * 3), ("err_us", ctypes.c_double * 2)]


class Batch:
    """Many independent third-order streams advanced together (see tdb.h): one launch
    per kernel covers every stream. `configs` holds one keyword dict per stream with
    the Compressor arguments (dims, dt, rank_max, ...); all share data_dtype and
    precision."""

    def __init__(self, configs: Sequence[dict]):
        self.lib = load_library()
        self._members = [Compressor(**kw) for kw in configs]
        self.n = len(self._members)
        self._cfgs = (TdbConfig * self.n)(*[m.cfg for m in self._members])
        self.h = ctypes.c_void_p()
        self.streams: List[Compressor] = []

    def _check(self, status: int):
        if status != OK:
            msg = self.lib.tdb_batch_last_error(self.h if self.h else None)
            raise TDBError(status, (msg or b"").decode())

    def _ptrs(self, Vs):
        if len(Vs) != self.n:
            raise ValueError(f"need {self.n} snapshots, got {len(Vs)}")
        return (ctypes.c_void_p * self.n)(*[_dev_ptr(v) for v in Vs])

    def init(self, V0s, stream=None):
        self._check(self.lib.tdb_batch_create(self.n, self._cfgs, self._ptrs(V0s), _stream_ptr(stream),
                                              ctypes.byref(self.h)))
        for i, m in enumerate(self._members):
            hh = ctypes.c_void_p()
            self._check(self.lib.tdb_batch_stream(self.h, i, ctypes.byref(hh)))
            m.h = hh
            m._borrowed = True
            self.streams.append(m)
        return self

    def ingest(self, Vs, stream=None):
        self._check(self.lib.tdb_batch_ingest(self.h, self._ptrs(Vs), _stream_ptr(stream)))

    def flush(self):
        """Read the newest step if it has not been read (pipelined batches)."""
        self._check(self.lib.tdb_batch_flush(self.h))

    def plan(self) -> dict:
        """The kernel plan chosen at creation (see tdb_batch_plan)."""
        q = TdbBatchPlan()
        self._check(self.lib.tdb_batch_plan(self.h, ctypes.byref(q)))
        kinds = {0: "vector-alu-tiles", 1: "matrix-core-tiles", 2: "matrix-core-columns"}
        return {"pass": kinds[q.pass_kind], "pass_cols": q.pass_cols,
                "error_pass": "columns" if q.err_kind else "row-slabs",
                "source": {0: "rule", 1: "timed", 2: "cached"}[q.source],
                "pass_us": list(q.pass_us), "err_us": list(q.err_us)}

    def gate_attach(self, gate, mean_std=None, mode: str = "active"):
        """Use a trained Gate (kept alive by the caller) with the given feature statistics
        (768 floats: means, then standard deviations). mode: off | record | active | shadow."""
        mid = {"off": 0, "record": 1, "active": 2, "shadow": 3}[mode]
        ms = None
        if mean_std is not None:
            self._ms = np.ascontiguousarray(mean_std, dtype=np.float32)
            ms = self._ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._check(self.lib.tdb_batch_gate_attach(self.h, gate.h if gate is not None else None, ms, mid))

    def profile_enable(self, on: bool = True, every: int = 1):
        self._check(self.lib.tdb_batch_profile_enable(self.h, max(1, int(every)) if on else 0))

    def profile_read(self, pass_name: str = "project") -> dict:
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        pid = {"project": 0, "error": 1}[pass_name]
        self._check(self.lib.tdb_batch_profile_read(self.h, pid, ctypes.byref(n), ctypes.byref(ms),
                                                    ctypes.byref(by)))
        return {"launches": n.value, "total_ms": ms.value, "bytes_per_launch": by.value}

    def close(self):
        for m in self.streams:
            m.h = ctypes.c_void_p()
        self.streams = []
        if self.h:
            self.lib.tdb_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Gate:
    """Trainer and holder of the learned error gate's parameters (see tdb.h)."""

    N_PARAMS = 65921
    N_IN = 384

    def __init__(self, max_batch: int = 1024):
        self.lib = load_library()
        self.h = ctypes.c_void_p()
        self._check(self.lib.tdb_gate_create(int(max_batch), ctypes.byref(self.h)))
        self.max_batch = int(max_batch)

    def _check(self, status: int):
        if status != OK:
            msg = self.lib.tdb_gate_last_error(self.h if self.h else None)
            raise TDBError(status, (msg or b"").decode())

    def set_params(self, theta: np.ndarray):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        if t.size != self.N_PARAMS:
            raise ValueError("wrong parameter count")
        self._check(self.lib.tdb_gate_set_params(self.h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.N_PARAMS, dtype=np.float32)
        self._check(self.lib.tdb_gate_get_params(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def forward(self, X, stream=None):
        import torch
        X = X.contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        self._check(self.lib.tdb_gate_forward(self.h, _dev_ptr(X), X.shape[0], _dev_ptr(y), _stream_ptr(stream)))
        return y

    def grad(self, X, t, stream=None):
        import torch
        g = torch.empty(self.N_PARAMS, dtype=torch.float32, device=X.device)
        loss = ctypes.c_float()
        self._check(self.lib.tdb_gate_grad(self.h, _dev_ptr(X.contiguous()), _dev_ptr(t.contiguous()), X.shape[0],
                                           _dev_ptr(g), ctypes.byref(loss), _stream_ptr(stream)))
        return g, loss.value

    def train_step(self, X, t, lr: float, want_loss: bool = False, stream=None):
        loss = ctypes.c_float()
        self._check(self.lib.tdb_gate_train_step(self.h, _dev_ptr(X), _dev_ptr(t), X.shape[0], float(lr),
                                                 ctypes.byref(loss) if want_loss else None, _stream_ptr(stream)))
        return loss.value if want_loss else None

    def close(self):
        if self.h:
            self.lib.tdb_gate_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
