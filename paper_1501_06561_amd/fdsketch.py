"""ctypes binding of libfdsketch.so (argument marshalling only).

Every step of the sketch runs in the library's HIP kernels; this module only
converts tensors to pointers, strides and enum codes.  PyTorch supplies device
memory and the HIP stream.  If the library is missing the binding raises: it
has no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdsketch.so")

VARIANTS = {"fd": 0, "isvd": 1, "alpha": 2, "fast_alpha": 3, "ssd": 4, "cfd": 5}
PRECISIONS = {"fp64": 0, "bf16": 1, "bf16x3": 2, "fp8x3": 3}
F64, F32, BF16 = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
ERRORS = {0: "OK", -1: "EINVAL", -2: "ESTATE", -3: "ENOMEM", -4: "EDEVICE", -5: "ENONFINITE",
          -6: "EUNSUPPORTED"}

# Every symbol the header declares (checked by the CPU test-suite).
EXPORTS = ("sketch_create", "sketch_append_rows", "sketch_merge", "sketch_finalize", "sketch_error",
           "fdsk_evaluate", "sketch_stats", "sketch_destroy", "sketch_last_error", "fdsk_version",
           "fdsk_gram", "fdsk_eigh", "sketch_reset", "sketch_profile", "sketch_batch_create",
           "sketch_batch_append", "sketch_batch_finalize", "sketch_batch_stats",
           "sketch_batch_reset", "sketch_batch_profile", "sketch_batch_destroy",
           "sketch_batch_last_error", "fdsk_eigh_noalloc", "rsketch_create", "rsketch_append",
           "rsketch_finalize", "rsketch_stats", "rsketch_destroy", "rsketch_last_error",
           "fdsk_tune_set_mode", "fdsk_tune_get_mode", "fdsk_tune_lookup", "fdsk_tune_set",
           "fdsk_tune_clear", "fdsk_tune_set_path", "fdsk_tune_path", "fdsk_tune_load",
           "fdsk_tune_save", "fdsk_tune_dump", "fdsk_tune_last_error")


class FdskConfig(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int64), ("l", ctypes.c_int32), ("buffer_rows", ctypes.c_int32),
                ("variant", ctypes.c_int), ("alpha", ctypes.c_double), ("precision", ctypes.c_int),
                ("flags", ctypes.c_uint32)]


class FdskReport(ctypes.Structure):
    _fields_ = [("cov_err", ctypes.c_double), ("proj_err_k", ctypes.c_double),
                ("proj_full_over_fro2", ctypes.c_double), ("fro2_A", ctypes.c_double),
                ("fro2_B", ctypes.c_double), ("delta_sum", ctypes.c_double),
                ("shrink_total", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("lambda_min", ctypes.c_double), ("n_rows", ctypes.c_int64),
                ("n_reduce", ctypes.c_int64), ("k", ctypes.c_int32), ("rows_out", ctypes.c_int32),
                ("eig_unconverged", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("eig_sweeps", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


STAGES = ("ingest", "gram", "eig", "shrink", "rebuild", "tridiag", "dc", "backtr", "tridiag_head")
FLAG_PROFILE = 1
FLAG_EIG_JACOBI = 2
FLAG_GRAPH = 4
EIG_METHODS = {"auto": 0, "jacobi": 1}


class FdskProfile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 9), ("launches", ctypes.c_int64 * 9),
                ("work", ctypes.c_double * 9)]

    def as_dict(self):
        """{stage: (total_ms, launches, algorithmic work)}; work is bytes for
        ingest and flops for the other stages."""
        return {name: (self.ms[i], self.launches[i], self.work[i]) for i, name in enumerate(STAGES)}


class FdskRsStats(ctypes.Structure):
    _fields_ = [("fro2_A", ctypes.c_double), ("tau", ctypes.c_double), ("weight_sum", ctypes.c_double),
                ("n_rows", ctypes.c_int64), ("rows_kept", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


RS_KINDS = {"hash": 0, "osnap": 1, "priority": 2, "varopt": 3}


class FdskError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None
# Library objects still open.  They are closed at interpreter exit, before the
# HIP runtime and any profiler attached to the process shut down, instead of
# whenever the garbage collector reaches them during teardown.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def _init_device_runtime():
    """Bring up torch's HIP runtime (the library shares it) before the first
    library call, so the device is open when the library allocates."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.empty(1, device="cuda")


def lib():
    """Load libfdsketch.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1501_06561_amd.build`")
    _init_device_runtime()
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, cint = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    L.sketch_create.argtypes = [ctypes.POINTER(FdskConfig), vp, ctypes.POINTER(vp)]
    L.sketch_append_rows.argtypes = [vp, vp, i64, i64, cint, cint]
    L.sketch_finalize.argtypes = [vp, vp, i64, cint, cint, ctypes.POINTER(i32)]
    L.sketch_merge.argtypes = [vp, vp]
    L.sketch_error.argtypes = [vp, vp, i64, i64, cint, cint, i32, i32, ctypes.POINTER(FdskReport)]
    L.fdsk_evaluate.argtypes = [vp, i64, i64, cint, vp, i64, i64, cint, i64, cint, i32, i32, vp,
                                ctypes.POINTER(FdskReport)]
    L.sketch_stats.argtypes = [vp, ctypes.POINTER(FdskReport)]
    L.sketch_destroy.argtypes = [vp]
    L.sketch_destroy.restype = None
    L.sketch_last_error.argtypes = [vp]
    L.sketch_last_error.restype = ctypes.c_char_p
    L.fdsk_version.restype = ctypes.c_char_p
    L.fdsk_gram.argtypes = [vp, i32, i64, i64, vp, i64, cint, vp]
    L.sketch_reset.argtypes = [vp]
    L.sketch_batch_create.argtypes = [i32, ctypes.POINTER(FdskConfig), vp, ctypes.POINTER(vp)]
    L.sketch_batch_append.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64), cint, cint, i32]
    L.sketch_batch_finalize.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i64), cint, cint,
                                        i32, ctypes.POINTER(i32)]
    L.sketch_batch_stats.argtypes = [vp, i32, ctypes.POINTER(FdskReport)]
    L.sketch_batch_reset.argtypes = [vp]
    L.sketch_batch_profile.argtypes = [vp, ctypes.POINTER(FdskProfile)]
    L.sketch_batch_destroy.argtypes = [vp]
    L.sketch_batch_destroy.restype = None
    L.sketch_batch_last_error.argtypes = [vp]
    L.sketch_batch_last_error.restype = ctypes.c_char_p
    L.sketch_profile.argtypes = [vp, ctypes.POINTER(FdskProfile)]
    L.fdsk_eigh.argtypes = [vp, i32, i64, vp, vp, i64, i32, vp]
    L.fdsk_eigh_noalloc.argtypes = [vp, i32, i64, vp, vp, i64, vp]
    L.rsketch_create.argtypes = [i32, i64, i32, i32, ctypes.c_uint64, vp, ctypes.POINTER(vp)]
    L.rsketch_append.argtypes = [vp, vp, i64, i64, cint, cint]
    L.rsketch_finalize.argtypes = [vp, vp, i64, cint, cint, vp, ctypes.POINTER(i32)]
    L.rsketch_stats.argtypes = [vp, ctypes.POINTER(FdskRsStats)]
    L.rsketch_destroy.argtypes = [vp]
    L.rsketch_destroy.restype = None
    L.rsketch_last_error.argtypes = [vp]
    L.rsketch_last_error.restype = ctypes.c_char_p
    L.fdsk_tune_set_mode.argtypes = [i32]
    L.fdsk_tune_get_mode.argtypes = []
    L.fdsk_tune_lookup.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32)]
    L.fdsk_tune_set.argtypes = [ctypes.c_char_p, i32]
    L.fdsk_tune_clear.argtypes = []
    L.fdsk_tune_set_path.argtypes = [ctypes.c_char_p]
    L.fdsk_tune_path.argtypes = []
    L.fdsk_tune_path.restype = ctypes.c_char_p
    L.fdsk_tune_load.argtypes = [ctypes.c_char_p]
    L.fdsk_tune_save.argtypes = [ctypes.c_char_p]
    L.fdsk_tune_dump.argtypes = [ctypes.c_char_p, i64]
    L.fdsk_tune_dump.restype = i32
    L.fdsk_tune_last_error.argtypes = []
    L.fdsk_tune_last_error.restype = ctypes.c_char_p
    for f in ("fdsk_tune_set_mode", "fdsk_tune_get_mode", "fdsk_tune_lookup", "fdsk_tune_set",
              "fdsk_tune_clear", "fdsk_tune_set_path", "fdsk_tune_load", "fdsk_tune_save"):
        getattr(L, f).restype = cint
    for f in ("sketch_create", "sketch_append_rows", "sketch_merge", "sketch_finalize", "sketch_error",
              "fdsk_evaluate", "sketch_stats", "fdsk_gram", "fdsk_eigh", "sketch_reset",
              "sketch_profile", "sketch_batch_create", "sketch_batch_append",
              "sketch_batch_finalize", "sketch_batch_stats", "sketch_batch_reset",
              "sketch_batch_profile", "fdsk_eigh_noalloc", "rsketch_create", "rsketch_append",
              "rsketch_finalize", "rsketch_stats"):
        getattr(L, f).restype = cint
    _lib = L
    return L


def _check(rc, handle=None):
    if rc != 0:
        msg = lib().sketch_last_error(handle)
        raise FdskError(rc, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if isinstance(t, np.ndarray):
        return {np.dtype(np.float64): F64, np.dtype(np.float32): F32}[t.dtype]
    return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[t.dtype]


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _bound_stream(stream):
    """The torch stream a library object is bound to: the given one, else the
    one current at creation (None without a GPU runtime)."""
    if stream is not None:
        return stream
    torch = _torch()
    return torch.cuda.current_stream() if torch.cuda.is_available() else None


def _order_after_current(stream, *tensors):
    """Make `stream` wait for the current stream and keep the device tensors'
    memory from reuse until `stream` has passed them (no-op when they are
    the same stream or nothing is on the device)."""
    dev = [t for t in tensors if getattr(t, "is_cuda", False)]
    if stream is None or not dev:
        return
    cur = _torch().cuda.current_stream()
    if stream != cur:
        stream.wait_stream(cur)
        for t in dev:
            t.record_stream(stream)


def _rows_arg(rows):
    """(pointer, n, stride, dtype code, mem kind, keepalive) for a 2-D matrix."""
    if isinstance(rows, np.ndarray):
        if rows.ndim != 2 or rows.strides[1] != rows.itemsize:
            rows = np.ascontiguousarray(rows)
        return (rows.ctypes.data, rows.shape[0], rows.strides[0] // rows.itemsize,
                _dtype_code(rows), MEM_HOST, rows)
    torch = _torch()
    if rows.dim() != 2:
        raise ValueError("rows must be a 2-D matrix")
    if rows.stride(1) != 1:
        rows = rows.contiguous()
    mem = MEM_DEVICE if rows.is_cuda else MEM_HOST
    return rows.data_ptr(), rows.shape[0], rows.stride(0), _dtype_code(rows), mem, rows


class FDSketch:
    """One streaming sketch (Algorithm 1 with the chosen ReduceRank rule)."""

    def __init__(self, d, l, variant="fd", alpha=0.2, buffer_rows=0, precision="fp64",
                 stream=None, profile=False, eig="auto"):
        self.d, self.l = int(d), int(l)
        flags = (FLAG_PROFILE if profile else 0) | (FLAG_EIG_JACOBI if eig == "jacobi" else 0)
        if eig not in EIG_METHODS:
            raise ValueError(f"eig must be one of {sorted(EIG_METHODS)}")
        cfg = FdskConfig(self.d, self.l, int(buffer_rows), VARIANTS[variant], float(alpha),
                         PRECISIONS[precision], flags)
        # The library keeps the stream it is created with; remember it as a
        # torch stream object so later calls can order themselves after it.
        self._stream = _bound_stream(stream)
        h = ctypes.c_void_p()
        _check(lib().sketch_create(ctypes.byref(cfg), _stream_handle(self._stream), ctypes.byref(h)))
        self._h = h
        _live.add(self)

    def _on_stream(self, t):
        """A device tensor made on the current stream and read by the library
        on the sketch's own stream: that stream waits for the current one, and
        the tensor's memory is kept from reuse until the sketch's stream is
        past it."""
        _order_after_current(self._stream, t)

    def append(self, rows):
        ptr, n, stride, dt, mem, keep = _rows_arg(rows)
        self._on_stream(keep)
        _check(lib().sketch_append_rows(self._h, ctypes.c_void_p(ptr), n, stride, dt, mem), self._h)
        return self

    def merge(self, other):
        """Absorb `other` (same configuration): afterwards this sketch covers
        both streams; `other` is unchanged."""
        _check(lib().sketch_merge(self._h, other._h), self._h)
        return self

    def finalize(self, dtype=None, device="cuda"):
        torch = _torch()
        dtype = dtype or torch.float64
        out = torch.empty((self.l, self.d), dtype=dtype, device=device)
        rows = ctypes.c_int32()
        mem = MEM_DEVICE if out.is_cuda else MEM_HOST
        _check(lib().sketch_finalize(self._h, ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                     _dtype_code(out), mem, ctypes.byref(rows)), self._h)
        self.rows_out = rows.value
        return out

    def reset(self):
        _check(lib().sketch_reset(self._h), self._h)
        return self

    def profile(self):
        """{stage: (total_ms, launches, work)} since create/reset (needs profile=True)."""
        p = FdskProfile()
        _check(lib().sketch_profile(self._h, ctypes.byref(p)), self._h)
        return p.as_dict()

    def stats(self):
        rep = FdskReport()
        _check(lib().sketch_stats(self._h, ctypes.byref(rep)), self._h)
        return rep.as_dict()

    def error(self, A, k=10, method=0):
        ptr, n, stride, dt, mem, keep = _rows_arg(A)
        self._on_stream(keep)
        rep = FdskReport()
        _check(lib().sketch_error(self._h, ctypes.c_void_p(ptr), n, stride, dt, mem, k, method,
                                  ctypes.byref(rep)), self._h)
        return rep.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sketch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def evaluate(A, B, k=10, method=0, stream=None):
    """Device evaluator of the Section 1.1 error measures for any sketch B."""
    pa, n, lda, dta, mema, ka = _rows_arg(A)
    pb, nb, ldb, dtb, memb, kb = _rows_arg(B)
    if mema != memb:
        raise ValueError("A and B must both be on the device or both on the host")
    rep = FdskReport()
    _check(lib().fdsk_evaluate(ctypes.c_void_p(pa), n, lda, dta, ctypes.c_void_p(pb), nb, ldb, dtb,
                               A.shape[1], mema, k, method, _stream_handle(stream),
                               ctypes.byref(rep)))
    return rep.as_dict()


def gram(C, precision="fp64", stream=None):
    """G = C C^T on the device; C: cuda float64 2-D tensor."""
    torch = _torch()
    if C.dtype != torch.float64 or not C.is_cuda or C.stride(1) != 1:
        raise ValueError("C must be a row-major cuda float64 matrix")
    G = torch.empty((C.shape[0], C.shape[0]), dtype=torch.float64, device=C.device)
    _check(lib().fdsk_gram(ctypes.c_void_p(C.data_ptr()), C.shape[0], C.shape[1], C.stride(0),
                           ctypes.c_void_p(G.data_ptr()), G.stride(0), PRECISIONS[precision],
                           _stream_handle(stream)))
    return G


def eigh(G, method="auto", stream=None):
    """(lam, V) with G = V diag(lam) V^T, unsorted, from the device solver
    ("auto": Householder tridiagonalization, divide and conquer and
    back-transformation at every m the library takes;
    "jacobi": the Jacobi solvers at every size)."""
    torch = _torch()
    if G.dtype != torch.float64 or not G.is_cuda or G.stride(1) != 1:
        raise ValueError("G must be a row-major cuda float64 matrix")
    m = G.shape[0]
    lam = torch.empty(m, dtype=torch.float64, device=G.device)
    V = torch.empty((m, m), dtype=torch.float64, device=G.device)
    _check(lib().fdsk_eigh(ctypes.c_void_p(G.data_ptr()), m, G.stride(0),
                           ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                           V.stride(0), EIG_METHODS[method], _stream_handle(stream)))
    return lam, V


def _check_batch(rc, handle=None):
    if rc != 0:
        msg = lib().sketch_batch_last_error(handle)
        raise FdskError(rc, msg.decode() if msg else "")


class FDSketchBatch:
    """Many independent sketches advanced together in lock-step rounds: one schedule per
    class of buffer rows, each class on its own library stream ordered after the batch's
    stream, and one launch per stage and round over the class's active sketches.  With
    graph=True (and profile=False) each append call runs through HIP graphs captured per
    size class (replayed when the next call has the same schedule, e.g. after reset())."""

    def __init__(self, configs, stream=None, profile=False, graph=False):
        """configs: list of dicts with keys d, l and optionally variant, alpha, buffer_rows,
        precision ("fp64", "bf16x3")."""
        self.S = len(configs)
        flags = (FLAG_PROFILE if profile else 0) | (FLAG_GRAPH if graph else 0)
        arr = (FdskConfig * self.S)()
        self.shapes = []
        for i, c in enumerate(configs):
            arr[i] = FdskConfig(int(c["d"]), int(c["l"]), int(c.get("buffer_rows", 0)),
                                VARIANTS[c.get("variant", "fd")], float(c.get("alpha", 0.2)),
                                PRECISIONS[c.get("precision", "fp64")], flags)
            self.shapes.append((int(c["l"]), int(c["d"])))
        self._stream = _bound_stream(stream)
        h = ctypes.c_void_p()
        _check_batch(lib().sketch_batch_create(self.S, arr, _stream_handle(self._stream), ctypes.byref(h)))
        self._h = h
        _live.add(self)

    def append(self, rows_list, grid_size=0):
        """rows_list[i]: 2-D matrix for sketch i (or None for no rows): all cuda
        tensors, or all host arrays / CPU tensors."""
        ptrs = (ctypes.c_void_p * self.S)()
        ns = (ctypes.c_int64 * self.S)()
        strides = (ctypes.c_int64 * self.S)()
        dt, mem = None, None
        keep = []
        for i, t in enumerate(rows_list):
            if t is None or t.shape[0] == 0:
                ptrs[i], ns[i], strides[i] = None, 0, self.shapes[i][1]
                continue
            ptr, n, stride, code, m, kept = _rows_arg(t)
            keep.append(kept)
            if dt is None:
                dt, mem = code, m
            elif dt != code or mem != m:
                raise ValueError("all sketches of one append call share a dtype and a memory kind")
            ptrs[i], ns[i], strides[i] = ptr, n, stride
        # Inputs made on the current stream, read on the batch's stream.
        _order_after_current(self._stream, *keep)
        _check_batch(lib().sketch_batch_append(self._h, ptrs, ns, strides, F64 if dt is None else dt,
                                               MEM_DEVICE if mem is None else mem, int(grid_size)),
                     self._h)
        return self

    def finalize(self, dtype=None, grid_size=0):
        torch = _torch()
        dtype = dtype or torch.float64
        outs = [torch.empty(shape, dtype=dtype, device="cuda") for shape in self.shapes]
        ptrs = (ctypes.c_void_p * self.S)(*[o.data_ptr() for o in outs])
        lds = (ctypes.c_int64 * self.S)(*[o.stride(0) for o in outs])
        rows = (ctypes.c_int32 * self.S)()
        _check_batch(lib().sketch_batch_finalize(self._h, ptrs, lds, _dtype_code(outs[0]), MEM_DEVICE,
                                                 int(grid_size), rows), self._h)
        self.rows_out = list(rows)
        return outs

    def reset(self):
        _check_batch(lib().sketch_batch_reset(self._h), self._h)
        return self

    def profile(self):
        """{stage: (total_ms, launches, work)} since create/reset (needs profile=True)."""
        p = FdskProfile()
        _check_batch(lib().sketch_batch_profile(self._h, ctypes.byref(p)), self._h)
        return p.as_dict()

    def stats(self, i):
        rep = FdskReport()
        _check_batch(lib().sketch_batch_stats(self._h, int(i), ctypes.byref(rep)), self._h)
        return rep.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sketch_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RSketch:
    """One hashing or sampling sketch (Hashing, OSNAP, Priority or VarOpt;
    see the rsketch_* declarations in include/fdsketch.h)."""

    def __init__(self, kind, d, l, s=4, key=0, stream=None):
        self.kind, self.d, self.l = kind, int(d), int(l)
        self._stream = _bound_stream(stream)
        h = ctypes.c_void_p()
        rc = lib().rsketch_create(RS_KINDS[kind], self.d, self.l, int(s), ctypes.c_uint64(int(key)),
                                  _stream_handle(self._stream), ctypes.byref(h))
        if rc != 0:
            msg = lib().rsketch_last_error(None)
            raise FdskError(rc, msg.decode() if msg else "")
        self._h = h
        _live.add(self)

    def _check(self, rc):
        if rc != 0:
            msg = lib().rsketch_last_error(self._h)
            raise FdskError(rc, msg.decode() if msg else "")

    def append(self, rows):
        ptr, n, stride, dt, mem, keep = _rows_arg(rows)
        _order_after_current(self._stream, keep)
        self._check(lib().rsketch_append(self._h, ctypes.c_void_p(ptr), n, stride, dt, mem))
        return self

    def finalize(self, dtype=None, device="cuda"):
        """(B, indices of the kept rows or None for the hashing kinds)."""
        torch = _torch()
        dtype = dtype or torch.float64
        out = torch.empty((self.l, self.d), dtype=dtype, device=device)
        idx = torch.full((self.l,), -1, dtype=torch.int64, device=device)
        rows = ctypes.c_int32()
        mem = MEM_DEVICE if out.is_cuda else MEM_HOST
        self._check(lib().rsketch_finalize(self._h, ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                           _dtype_code(out), mem, ctypes.c_void_p(idx.data_ptr()),
                                           ctypes.byref(rows)))
        self.rows_out = rows.value
        if self.kind in ("hash", "osnap"):
            return out, None
        return out, idx[:rows.value]

    def stats(self):
        st = FdskRsStats()
        self._check(lib().rsketch_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().rsketch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# Launch-shape tuning of the Gram and rebuild products (fdsk_tune_* in the
# header): a process-wide table of choices persisted to a cache file.
TUNE_MODES = {"off": 0, "on": 1, "refresh": 2}


def tune_mode(mode=None):
    """Set the tuning mode ("off", "on", "refresh") if given; return the
    current one."""
    L = lib()
    if mode is not None:
        rc = L.fdsk_tune_set_mode(TUNE_MODES[mode])
        if rc != 0:
            raise FdskError(rc, f"bad tuning mode {mode!r}")
    cur = L.fdsk_tune_get_mode()
    return {v: k for k, v in TUNE_MODES.items()}[cur]


def tune_lookup(key):
    """The tuned value of key, or None."""
    v = ctypes.c_int32()
    rc = lib().fdsk_tune_lookup(key.encode(), ctypes.byref(v))
    if rc < 0:
        raise FdskError(rc, "tune_lookup")
    return v.value if rc == 0 else None


def tune_set(key, value):
    rc = lib().fdsk_tune_set(key.encode(), int(value))
    if rc != 0:
        raise FdskError(rc, f"bad tuning key {key!r}")


def tune_clear():
    lib().fdsk_tune_clear()


def tune_path(path=None):
    """Set the cache file if given ("" for none); return the current one."""
    L = lib()
    if path is not None:
        L.fdsk_tune_set_path(path.encode())
    return L.fdsk_tune_path().decode()


def tune_load(path=None):
    rc = lib().fdsk_tune_load(path.encode() if path is not None else None)
    if rc != 0:
        raise FdskError(rc, lib().fdsk_tune_last_error().decode())


def tune_save(path=None):
    rc = lib().fdsk_tune_save(path.encode() if path is not None else None)
    if rc != 0:
        raise FdskError(rc, lib().fdsk_tune_last_error().decode())


def tune_table():
    """The table as {key: (value, note)}."""
    L = lib()
    n = L.fdsk_tune_dump(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    L.fdsk_tune_dump(buf, n + 1)
    out = {}
    for line in buf.value.decode().splitlines():
        parts = line.split("\t")
        if len(parts) >= 2:
            out[parts[0]] = (int(parts[1]), parts[2] if len(parts) > 2 else "")
    return out
