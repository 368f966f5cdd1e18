"""Python binding of the gfx950 two-table Figaro library (``libfigaro.so``).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/figaro.h``.  PyTorch supplies
device memory and the current HIP stream.  Importing this package does not
load the library; the first call does, and raises if it is not built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfigaro.so")

FIGARO_OK = 0
FIGARO_EINVAL = -1
FIGARO_EUNSORTED = -2
FIGARO_EWORKSPACE = -3
FIGARO_EHIP = -4
FIGARO_ETIMEOUT = -5

FIGARO_F32 = 0
FIGARO_F64 = 1

PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_refine": 2}
FIGARO_TWO_SIDED = 0x100
FIGARO_GIVENS = 0x200


def precision_code(precision, two_sided=False, givens=False):
    return PRECISIONS[precision] | (FIGARO_TWO_SIDED if two_sided else 0) | (FIGARO_GIVENS if givens else 0)


class FigaroError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"figaro error {code}: {msg}")
        self.code = code


class Table(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("dtype", ctypes.c_int32), ("keys", ctypes.c_void_p)]


class View(ctypes.Structure):
    _fields_ = [("counts", ctypes.c_void_p), ("g_key", ctypes.c_void_p), ("g_offA", ctypes.c_void_p),
                ("g_m1", ctypes.c_void_p), ("g_offB", ctypes.c_void_p), ("g_m2", ctypes.c_void_p),
                ("g_r1", ctypes.c_void_p), ("g_r2", ctypes.c_void_p), ("group_cap", ctypes.c_int64),
                ("heads", ctypes.c_void_p), ("m1", ctypes.c_void_p), ("m2", ctypes.c_void_p),
                ("heads_a", ctypes.c_void_p), ("tails_a", ctypes.c_void_p),
                ("m_dtype", ctypes.c_int32), ("status", ctypes.c_void_p)]


class Memory(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_int64), ("join_rows", ctypes.c_int64), ("compact_rows", ctypes.c_int64),
                ("input_bytes", ctypes.c_double), ("compact_bytes", ctypes.c_double),
                ("workspace_bytes", ctypes.c_double), ("join_bytes", ctypes.c_double)]


class Instance(ctypes.Structure):
    _fields_ = [("A", Table), ("B", Table)]


EXPORTS = [
    "figaro_r_workspace_size", "figaro_r", "figaro_compact", "figaro_inspect",
    "figaro_sigma_workspace_size", "figaro_sigma", "figaro_sigma_jacobi", "figaro_sigma_bidiag", "figaro_status", "figaro_last_error",
    "figaro_plan_create", "figaro_plan_workspace_size", "figaro_plan_offsets",
    "figaro_plan_execute", "figaro_plan_execute_eager", "figaro_plan_destroy", "figaro_plan_autotune",
    "figaro_sort_workspace_size", "figaro_sort_table", "figaro_memory_report", "figaro_svd_workspace_size",
    "figaro_svd", "figaro_sigma_dqds",
    "figaro_r_autotune", "figaro_tune_load", "figaro_tune_save", "figaro_tune_dump", "figaro_timing_enable", "figaro_timing_read",
    "figaro_sigma_noalloc",
]

_lib = None


def lib():
    """Load libfigaro.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python paper_2503_23385_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    TP = ctypes.POINTER(Table)
    L.figaro_r_workspace_size.argtypes = [TP, TP, I32, ctypes.POINTER(SZ)]
    L.figaro_r.argtypes = [TP, TP, I32, P, I64, P, SZ, P]
    L.figaro_compact.argtypes = [TP, TP, I32, P, SZ, P]
    L.figaro_inspect.argtypes = [TP, TP, I32, P, SZ, ctypes.POINTER(View)]
    L.figaro_sigma_workspace_size.argtypes = [I64, ctypes.POINTER(SZ)]
    L.figaro_sigma.argtypes = [P, I64, I64, P, P, SZ, P]
    L.figaro_sigma_jacobi.argtypes = [P, I64, I64, P, P, SZ, P]
    L.figaro_sigma_bidiag.argtypes = [P, I64, I64, P, P, SZ, P]
    L.figaro_sigma_dqds.argtypes = [P, I64, I64, P, P, SZ, P]
    L.figaro_sigma_noalloc.argtypes = [P, I64, I64, P, P]
    L.figaro_status.argtypes = [P, P, ctypes.POINTER(I32)]
    L.figaro_last_error.argtypes = []
    L.figaro_last_error.restype = ctypes.c_char_p
    L.figaro_plan_create.argtypes = [ctypes.POINTER(Instance), I32, I32, ctypes.POINTER(P)]
    L.figaro_plan_workspace_size.argtypes = [P, ctypes.POINTER(SZ)]
    L.figaro_plan_offsets.argtypes = [P, P, P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    L.figaro_plan_execute.argtypes = [P, P, SZ, P, P, P]
    L.figaro_plan_execute_eager.argtypes = [P, P, SZ, P, P, P]
    L.figaro_plan_autotune.argtypes = [P, P, SZ, P, P, P]
    L.figaro_r_autotune.argtypes = [TP, TP, I32, P, I64, P, SZ, P]
    L.figaro_svd_workspace_size.argtypes = [I64, ctypes.POINTER(SZ)]
    L.figaro_svd.argtypes = [P, I64, I64, P, P, I64, P, SZ, P]
    L.figaro_sort_workspace_size.argtypes = [I64, ctypes.POINTER(SZ)]
    L.figaro_sort_table.argtypes = [TP, P, I64, P, P, SZ, P]
    L.figaro_memory_report.argtypes = [TP, TP, I32, P, SZ, P, ctypes.POINTER(Memory)]
    L.figaro_tune_load.argtypes = [ctypes.c_char_p]
    L.figaro_tune_save.argtypes = [ctypes.c_char_p]
    L.figaro_tune_dump.argtypes = [P, SZ, ctypes.POINTER(SZ)]
    L.figaro_plan_destroy.argtypes = [P]
    L.figaro_plan_destroy.restype = None
    L.figaro_timing_enable.argtypes = [I32]
    L.figaro_timing_read.argtypes = [P, P, P, I32, ctypes.POINTER(I32)]
    for name in EXPORTS:
        if name not in ("figaro_last_error", "figaro_plan_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != FIGARO_OK:
        raise FigaroError(rc, lib().figaro_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return FIGARO_F64
    if t.dtype == torch.float32:
        return FIGARO_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def require_device(name, t, device=None):
    """Raise unless t is a GPU tensor (on `device` when given): the kernels dereference
    its address, and a host address there faults the GPU."""
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor, got one on {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


def make_table(X, keys=None) -> Table:
    """Describe a device tensor (rows x cols, unit column stride) and optional int32 keys."""
    torch = _torch()
    require_device("table", X)
    require_device("keys", keys, X.device)
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("table must be 2-D with unit column stride")
    if keys is not None:
        if keys.dtype != torch.int32 or not keys.is_contiguous():
            raise TypeError("keys must be a contiguous int32 tensor")
        if keys.numel() != X.shape[0]:
            raise ValueError("one key per row")
    ld = X.stride(0) if X.shape[0] > 1 else X.shape[1]
    return Table(X.data_ptr() if X.numel() else None, X.shape[0], X.shape[1], max(ld, X.shape[1]),
                 _dtype_code(X), keys.data_ptr() if keys is not None else None)


def r_workspace_size(A, B, keys_A=None, keys_B=None, precision="fp64", two_sided=False, givens=False) -> int:
    ta, tb = make_table(A, keys_A), make_table(B, keys_B)
    n = ctypes.c_size_t(0)
    _check(lib().figaro_r_workspace_size(ctypes.byref(ta), ctypes.byref(tb),
                                         precision_code(precision, two_sided, givens), ctypes.byref(n)))
    return n.value


def alloc_workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def r(A, B, keys_A=None, keys_B=None, precision="fp64", ws=None, out=None, stream=None,
      two_sided=False, givens=False):
    """R (N x N, FP64, diag >= 0) of the join of A and B on the device.  Returns (R, ws).
    givens: reduce the compact matrix by Givens rotations (FP64) instead of Householder."""
    torch = _torch()
    ta, tb = make_table(A, keys_A), make_table(B, keys_B)
    require_device("B", B, A.device)
    N = A.shape[1] + B.shape[1]
    if ws is None:
        ws = alloc_workspace(r_workspace_size(A, B, keys_A, keys_B, precision, two_sided, givens), A.device)
    if out is None:
        out = torch.empty((N, N), dtype=torch.float64, device=A.device)
    require_device("ws", ws, A.device)
    require_device("out", out, A.device)
    if out.dtype != torch.float64 or out.dim() != 2 or out.shape[0] < N or out.shape[1] < N or out.stride(1) != 1:
        raise ValueError("out must be an FP64 N x N (or larger) matrix with unit column stride")
    _check(lib().figaro_r(ctypes.byref(ta), ctypes.byref(tb), precision_code(precision, two_sided, givens),
                          ctypes.c_void_p(out.data_ptr()), out.stride(0),
                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    return out, ws


def sigma_workspace_size(n) -> int:
    nb = ctypes.c_size_t(0)
    _check(lib().figaro_sigma_workspace_size(n, ctypes.byref(nb)))
    return nb.value


def sigma(R, out=None, ws=None, stream=None, method="default"):
    """Singular values (descending, FP64) of a square device matrix R.

    method: "default" (bidiagonal route for n <= 128, Jacobi above), "jacobi" (one-sided
    Jacobi, any n <= 512), "bidiag" (bidiagonalisation + multisection, n <= 128) or "dqds"
    (bidiagonalisation + dqds, n <= 128)."""
    torch = _torch()
    require_device("R", R)
    if R.dtype != torch.float64 or R.dim() != 2 or R.shape[0] != R.shape[1] or R.stride(1) != 1:
        raise ValueError("R must be a square FP64 matrix with unit column stride")
    n = R.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=R.device)
    if ws is None:
        ws = alloc_workspace(sigma_workspace_size(n), R.device)
    require_device("out", out, R.device)
    require_device("ws", ws, R.device)
    if out.dtype != torch.float64 or out.numel() < n:
        raise ValueError("out must hold n FP64 values")
    fns = {"default": lib().figaro_sigma, "jacobi": lib().figaro_sigma_jacobi, "bidiag": lib().figaro_sigma_bidiag,
           "dqds": lib().figaro_sigma_dqds}
    if method not in fns:
        raise ValueError(f"unknown sigma method {method!r}")
    fn = fns[method]
    _check(fn(ctypes.c_void_p(R.data_ptr()), n, R.stride(0),
                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), _stream_ptr(stream)))
    return out


def sigma_noalloc(R, out=None, stream=None):
    """Singular values of R by the route of sigma(method="default"), with no workspace: the
    library's static per-GPU scratch serves instead (n <= 512; calls on one GPU must not
    overlap).  Allocates nothing itself when `out` is given."""
    torch = _torch()
    require_device("R", R)
    if R.dtype != torch.float64 or R.dim() != 2 or R.shape[0] != R.shape[1] or R.stride(1) != 1:
        raise ValueError("R must be a square FP64 matrix with unit column stride")
    n = R.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=R.device)
    require_device("out", out, R.device)
    if out.dtype != torch.float64 or out.numel() < n:
        raise ValueError("out must hold n FP64 values")
    _check(lib().figaro_sigma_noalloc(ctypes.c_void_p(R.data_ptr()), n, R.stride(0),
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def status(ws, stream=None) -> int:
    code = ctypes.c_int32(0)
    _check(lib().figaro_status(ctypes.c_void_p(ws.data_ptr()), _stream_ptr(stream), ctypes.byref(code)))
    return code.value


def compact(A, B, keys_A=None, keys_B=None, precision="fp64", ws=None, stream=None, two_sided=False):
    """Run grouping, head/tail scans and assembly; return host copies of the intermediates."""
    ta, tb = make_table(A, keys_A), make_table(B, keys_B)
    code = precision_code(precision, two_sided)
    if ws is None:
        ws = alloc_workspace(r_workspace_size(A, B, keys_A, keys_B, precision, two_sided), A.device)
    require_device("ws", ws, A.device)
    _check(lib().figaro_compact(ctypes.byref(ta), ctypes.byref(tb), code,
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    return inspect(A, B, keys_A, keys_B, precision, ws, stream, two_sided)


def inspect(A, B, keys_A, keys_B, precision, ws, stream=None, two_sided=False):
    """Copy the group table, counts, heads and compact-matrix regions out of a workspace."""
    torch = _torch()
    ta, tb = make_table(A, keys_A), make_table(B, keys_B)
    v = View()
    _check(lib().figaro_inspect(ctypes.byref(ta), ctypes.byref(tb), precision_code(precision, two_sided),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(v)))
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    base = ws.data_ptr()

    def view(ptr, count, dtype):
        off = ptr - base
        esz = torch.empty((), dtype=dtype).element_size()
        return ws[off:off + count * esz].view(dtype).cpu().numpy()

    counts = view(v.counts, 4, torch.int64)
    G, R1, R2 = int(counts[0]), int(counts[1]), int(counts[2])
    groups = {name: view(getattr(v, "g_" + name), G, torch.int32)
              for name in ("key", "offA", "m1", "offB", "m2", "r1", "r2")}
    n1, n2 = A.shape[1], B.shape[1]
    mdt = torch.float64 if v.m_dtype == FIGARO_F64 else torch.float32
    out = {
        "counts": counts,
        "groups": groups,
        "heads": view(v.heads, G * n2, torch.float64).reshape(G, n2),
        "M2": view(v.m2, R2 * n2, mdt).reshape(R2, n2),
        "status": int(view(v.status, 1, torch.int32)[0]),
    }
    if two_sided:
        out["heads_rows"] = view(v.m1, G * (n1 + n2), mdt).reshape(G, n1 + n2)
        out["heads_a"] = view(v.heads_a, G * n1, torch.float64).reshape(G, n1)
        out["tails_a"] = view(v.tails_a, (R1 - G) * n1, mdt).reshape(R1 - G, n1)
    else:
        out["M1"] = view(v.m1, R1 * (n1 + n2), mdt).reshape(R1, n1 + n2)
    return out


def r_autotune(A, B, keys_A=None, keys_B=None, precision="fp64", two_sided=False, ws=None, out=None, stream=None):
    """Time the tree candidates of figaro_r on this problem and keep the fastest (tuning table)."""
    torch = _torch()
    ta, tb = make_table(A, keys_A), make_table(B, keys_B)
    N = A.shape[1] + B.shape[1]
    if ws is None:
        ws = alloc_workspace(r_workspace_size(A, B, keys_A, keys_B, precision, two_sided), A.device)
    if out is None:
        out = torch.empty((N, N), dtype=torch.float64, device=A.device)
    require_device("ws", ws, A.device)
    require_device("out", out, A.device)
    _check(lib().figaro_r_autotune(ctypes.byref(ta), ctypes.byref(tb), precision_code(precision, two_sided),
                                   ctypes.c_void_p(out.data_ptr()), out.stride(0), ctypes.c_void_p(ws.data_ptr()),
                                   ws.numel(), _stream_ptr(stream)))


def svd(R, stream=None):
    """Singular values (descending) and right singular vectors V (column j for sigma[j]) of a
    square FP64 device matrix R, n <= 128.  Returns (sigma, V)."""
    torch = _torch()
    require_device("R", R)
    if R.dtype != torch.float64 or R.dim() != 2 or R.shape[0] != R.shape[1] or R.stride(1) != 1:
        raise ValueError("R must be a square FP64 matrix with unit column stride")
    n = R.shape[0]
    nb = ctypes.c_size_t(0)
    _check(lib().figaro_svd_workspace_size(n, ctypes.byref(nb)))
    ws = alloc_workspace(nb.value, R.device)
    S = torch.empty(n, dtype=torch.float64, device=R.device)
    V = torch.empty((n, n), dtype=torch.float64, device=R.device)
    _check(lib().figaro_svd(ctypes.c_void_p(R.data_ptr()), n, R.stride(0), ctypes.c_void_p(S.data_ptr()),
                            ctypes.c_void_p(V.data_ptr()), n, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                            _stream_ptr(stream)))
    return S, V


def sort_table(X, keys, stream=None):
    """Rows of X and their int32 keys in ascending key order, equal keys in input order (on the
    device).  Returns (X_sorted, keys_sorted)."""
    torch = _torch()
    require_device("X", X)
    require_device("keys", keys, X.device)
    t = make_table(X, keys)
    n = ctypes.c_size_t(0)
    _check(lib().figaro_sort_workspace_size(X.shape[0], ctypes.byref(n)))
    ws = alloc_workspace(n.value, X.device)
    out = torch.empty((X.shape[0], X.shape[1]), dtype=X.dtype, device=X.device)
    kout = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
    _check(lib().figaro_sort_table(ctypes.byref(t), ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                   ctypes.c_void_p(kout.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream_ptr(stream)))
    return out, kout


def memory_report(A, B, keys_A, keys_B, ws, precision="fp64", two_sided=False, stream=None):
    """Memory footprint (dict) of the compact path against the materialised join, from the counts
    that r() or compact() left in ws (synchronous)."""
    ta, tb = make_table(A, keys_A), make_table(B, keys_B)
    m = Memory()
    _check(lib().figaro_memory_report(ctypes.byref(ta), ctypes.byref(tb), precision_code(precision, two_sided),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream),
                                      ctypes.byref(m)))
    return {k: getattr(m, k) for k, _ in Memory._fields_}


def tune_load(path):
    _check(lib().figaro_tune_load(os.fsencode(path)))


def tune_save(path):
    _check(lib().figaro_tune_save(os.fsencode(path)))


def tune_table():
    """The tuning table as a list of dicts."""
    import json
    n = ctypes.c_size_t(0)
    _check(lib().figaro_tune_dump(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib().figaro_tune_dump(buf, n.value + 1, ctypes.byref(n)))
    return [json.loads(line) for line in buf.value.decode().splitlines() if line.strip()]


def timing_enable(on=True):
    _check(lib().figaro_timing_enable(1 if on else 0))


def timing_read():
    """Per-stage device time {stage: (ms, launches)} since the last read (synchronous)."""
    cap = 64
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int32 * cap)()
    n = ctypes.c_int32(0)
    _check(lib().figaro_timing_read(ctypes.cast(names, ctypes.c_void_p), ctypes.cast(ms, ctypes.c_void_p),
                                    ctypes.cast(cnt, ctypes.c_void_p), cap, ctypes.byref(n)))
    return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(n.value, cap))}


class Plan:
    """Batched plan over many independent two-table instances."""

    def __init__(self, instances, precision="fp64", two_sided=False):
        """instances: list of (A, B, keys_A, keys_B) device tensors."""
        self._keep = instances
        arr = (Instance * len(instances))()
        for i, (A, B, kA, kB) in enumerate(instances):
            arr[i].A = make_table(A, kA)
            arr[i].B = make_table(B, kB)
        self._arr = arr
        h = ctypes.c_void_p()
        _check(lib().figaro_plan_create(arr, len(instances), precision_code(precision, two_sided),
                                        ctypes.byref(h)))
        self.handle = h
        nb = ctypes.c_size_t(0)
        _check(lib().figaro_plan_workspace_size(h, ctypes.byref(nb)))
        self.ws_bytes = nb.value
        import numpy as np
        self.r_off = np.zeros(len(instances), dtype=np.int64)
        self.s_off = np.zeros(len(instances), dtype=np.int64)
        rt, st = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().figaro_plan_offsets(h, self.r_off.ctypes.data_as(ctypes.c_void_p),
                                         self.s_off.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(rt), ctypes.byref(st)))
        self.r_total, self.s_total = rt.value, st.value

    def execute(self, ws, R, S, stream=None):
        _check(lib().figaro_plan_execute(self.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                         _stream_ptr(stream)))

    def execute_eager(self, ws, R, S, stream=None):
        """The same launches without the graph (one by one on the stream; stage timing sees them)."""
        _check(lib().figaro_plan_execute_eager(self.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                               ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                               _stream_ptr(stream)))

    def autotune(self, ws, R, S, stream=None):
        """Time the tree candidates on this plan and keep the fastest per width class."""
        _check(lib().figaro_plan_autotune(self.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                          ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                                          _stream_ptr(stream)))

    def __del__(self):
        try:
            if self.handle:
                lib().figaro_plan_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
