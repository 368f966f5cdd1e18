"""Python access to the plain FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  It
shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

G_COLS = 7  # key, offA, m1_g, offB, m2_g, r1_g, r2_g


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i64, i32p, dp, i64p = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
        L.oracle_groups.argtypes = [ctypes.c_void_p, i64, ctypes.c_void_p, i64, i64, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_groups.restype = ctypes.c_int
        L.oracle_compact.argtypes = [dp, i64, i64, i64, dp, i64, i64, i64, dp, i64, i64, dp, i64, dp]
        L.oracle_compact.restype = ctypes.c_int
        L.oracle_householder.argtypes = [dp, i64, i64, i64]
        L.oracle_householder.restype = ctypes.c_int
        L.oracle_sign_normalise.argtypes = [dp, i64, i64]
        L.oracle_sign_normalise.restype = None
        L.oracle_extract_r.argtypes = [dp, i64, i64, i64, dp, i64]
        L.oracle_extract_r.restype = None
        L.oracle_r.argtypes = [dp, i64, i64, i64, dp, dp, i64, i64, i64, dp, dp, i64, dp]
        L.oracle_r.restype = ctypes.c_int
        L.oracle_sigma.argtypes = [dp, i64, i64, dp, ctypes.c_int]
        L.oracle_sigma.restype = ctypes.c_int
        L.oracle_svd_v.argtypes = [dp, i64, i64, dp, dp, i64, ctypes.c_int]
        L.oracle_svd_v.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(X):
    return np.ascontiguousarray(np.asarray(X, dtype=np.float64))  # FP32 upcast is exact


def _keys(k):
    return None if k is None else np.ascontiguousarray(np.asarray(k, dtype=np.int32))


def groups(keys_A, keys_B, m1=None, m2=None):
    """Group table (G x 7 int64) and counts (G, R1, R2, join_rows)."""
    kA, kB = _keys(keys_A), _keys(keys_B)
    if m1 is None:
        m1 = len(kA)
    if m2 is None:
        m2 = len(kB)
    cap = max(1, min(m1, m2))
    tab = np.zeros((cap, G_COLS), dtype=np.int64)
    counts = np.zeros(4, dtype=np.int64)
    rc = lib().oracle_groups(_p(kA), m1, _p(kB), m2, cap, _p(tab), _p(counts))
    if rc != 0:
        raise OracleError(f"oracle_groups failed: {rc}")
    G = int(counts[0])
    return tab[:G].copy(), counts


def compact(inst):
    """Compact matrix M ((R1+R2) x N, FP64) of Claim 1, heads (G x n2), table, counts."""
    A, B = _f64(inst.A), _f64(inst.B)
    m1, n1 = A.shape
    m2, n2 = B.shape
    tab, counts = groups(inst.keys_A, inst.keys_B, m1, m2)
    G, R1, R2 = int(counts[0]), int(counts[1]), int(counts[2])
    N = n1 + n2
    M = np.zeros((R1 + R2, N), dtype=np.float64)
    heads = np.zeros((G, n2), dtype=np.float64)
    tabc = np.ascontiguousarray(tab)
    rc = lib().oracle_compact(_p(A), m1, n1, n1, _p(B), m2, n2, n2, _p(tabc), G, R1,
                              _p(M), N, _p(heads))
    if rc != 0:
        raise OracleError(f"oracle_compact failed: {rc}")
    return M, heads, tab, counts


def householder_r(X, normalise=True):
    """R (N x N) of the Householder QR of X (rows x N); rows normalised to diag >= 0."""
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    rows, N = X.shape
    rc = lib().oracle_householder(_p(X), rows, N, N)
    if rc != 0:
        raise OracleError(f"oracle_householder failed: {rc}")
    R = np.zeros((N, N), dtype=np.float64)
    lib().oracle_extract_r(_p(X), rows, N, N, _p(R), N)
    if normalise:
        lib().oracle_sign_normalise(_p(R), N, N)
    return R


def sign_normalise(R):
    R = np.array(R, dtype=np.float64, order="C", copy=True)
    N = R.shape[0]
    lib().oracle_sign_normalise(_p(R), N, N)
    return R


def r(inst):
    """R (N x N FP64, diag >= 0) of the join matrix, through the compact matrix."""
    A, B = _f64(inst.A), _f64(inst.B)
    m1, n1 = A.shape
    m2, n2 = B.shape
    kA, kB = _keys(inst.keys_A), _keys(inst.keys_B)
    N = n1 + n2
    R = np.zeros((N, N), dtype=np.float64)
    counts = np.zeros(4, dtype=np.int64)
    rc = lib().oracle_r(_p(A), m1, n1, n1, _p(kA), _p(B), m2, n2, n2, _p(kB), _p(R), N, _p(counts))
    if rc != 0:
        raise OracleError(f"oracle_r failed: {rc}")
    return R


def sigma(R, max_sweeps=60, return_sweeps=False):
    """Singular values (descending) of a square R by one-sided Jacobi."""
    R = np.ascontiguousarray(np.asarray(R, dtype=np.float64))
    N = R.shape[0]
    out = np.zeros(N, dtype=np.float64)
    sw = lib().oracle_sigma(_p(R), N, N, _p(out), max_sweeps)
    if sw < 0:
        raise OracleError(f"oracle_sigma failed: {sw}")
    return (out, sw) if return_sweeps else out


def svd_v(R, max_sweeps=60):
    """Singular values (descending) and right singular vectors of a square R by one-sided
    Jacobi with the rotations accumulated: V[:, j] belongs to sigma[j]."""
    R = np.ascontiguousarray(np.asarray(R, dtype=np.float64))
    N = R.shape[0]
    s = np.zeros(N, dtype=np.float64)
    V = np.zeros((N, N), dtype=np.float64)
    sw = lib().oracle_svd_v(_p(R), N, N, _p(s), _p(V), N, max_sweeps)
    if sw < 0:
        raise OracleError(f"oracle_svd_v failed: {sw}")
    return s, V


def sort_table(X, keys):
    """The rows of X and their keys in ascending (signed int32) key order, rows with equal keys
    in their input order: the plain definition of a stable sort (the method's precondition on
    its relations, Experiments section), with numpy's stable argsort as the sorting step."""
    keys = np.asarray(keys, dtype=np.int32)
    order = np.argsort(keys, kind="stable")
    return np.ascontiguousarray(np.asarray(X)[order]), np.ascontiguousarray(keys[order])


def num_threads() -> int:
    return int(lib().oracle_num_threads())
