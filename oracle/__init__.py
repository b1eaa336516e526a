"""CPU oracle for BP + LSD (test infrastructure only).

This package is the reference the HIP decoder is checked against.  It is plain
float64 C (``qlsd_oracle.c``) behind ctypes; it shares no code with the HIP
library.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it.  The decoder product path never does.

Functions follow the paper's Sec. 2-4, Alg. 1/2 and Appendix D; the readings
taken where the paper is silent are listed in the C file's header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qlsd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

ST_BP_CONVERGED, ST_LSD_RUN, ST_UNSAT, ST_BAD_LLR = 1, 2, 4, 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I = ctypes.c_int
            D = ctypes.c_double
            L.oracle_code_new.restype = P
            L.oracle_code_new.argtypes = [I, I, P, P]
            L.oracle_code_free.argtypes = [P]
            L.oracle_lambda.argtypes = [P, I, P]
            L.oracle_omega.argtypes = [P, I, P]
            L.oracle_bp.argtypes = [P, P, P, I, D, I, P, P, P]
            L.oracle_bp_traj.argtypes = [P, P, P, I, D, I, P, P, P, P]
            L.oracle_lsd.argtypes = [P, P, P, I, P, I, P, P]
            L.oracle_lsd_cs.argtypes = [P, P, P, I, I, P, P, P]
            L.oracle_osd0.argtypes = [P, P, P, P]
            L.oracle_osd_cs.argtypes = [P, P, P, I, P, P]
            L.oracle_error_clusters.argtypes = [P, P, P]
            L.oracle_decode_batch.argtypes = [P, P, P, I, I, D, I, P, P, P, P, P, I]
            L.oracle_max_threads.restype = I
            _lib = L
        return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Code:
    """Oracle-side handle on a check matrix given as CSR (row_ptr, col_idx)."""

    def __init__(self, m: int, n: int, row_ptr: np.ndarray, col_idx: np.ndarray):
        self.m, self.n = int(m), int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self._h = lib().oracle_code_new(self.m, self.n, _p(self.row_ptr), _p(self.col_idx))

    @classmethod
    def from_dense(cls, H: np.ndarray) -> "Code":
        H = np.asarray(H, dtype=np.uint8)
        m, n = H.shape
        row_ptr = np.zeros(m + 1, dtype=np.int32)
        cols = []
        for i in range(m):
            nz = np.nonzero(H[i])[0]
            cols.extend(nz.tolist())
            row_ptr[i + 1] = len(cols)
        return cls(m, n, row_ptr, np.array(cols, dtype=np.int32))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.oracle_code_free(self._h)
            self._h = None


def llr_from_priors(priors: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(priors, dtype=np.float64)
    lam = np.empty_like(p)
    if lib().oracle_lambda(_p(p), p.shape[0], _p(lam)) != 0:
        raise ValueError("priors must lie strictly inside (0, 1)")
    return lam


def omega_from_llr(lam: np.ndarray) -> np.ndarray:
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    om = np.empty(lam.shape[0], dtype=np.int64)
    lib().oracle_omega(_p(lam), lam.shape[0], _p(om))
    return om


def bp(code: Code, lam: np.ndarray, s: np.ndarray, max_iter: int, alpha: float = 0.625,
       early_exit: bool = True):
    """One shot of min-sum BP -> (converged, iters, L float64[n], hard uint8[n])."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.uint8)
    L = np.empty(code.n, dtype=np.float64)
    hard = np.empty(code.n, dtype=np.uint8)
    it = np.zeros(1, dtype=np.int32)
    conv = lib().oracle_bp(code._h, _p(lam), _p(s), int(max_iter), float(alpha), int(early_exit),
                           _p(L), _p(hard), _p(it))
    return bool(conv), int(it[0]), L, hard


def bp_min_magnitude(code: Code, lam: np.ndarray, s: np.ndarray, iters: int, alpha: float = 0.625) -> float:
    """Smallest |q_{j->i}| or |L_j| over the first `iters` BP iterations (all run, no early exit).
    A shot whose float64 trajectory comes this close to zero can take a different sign in float32."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.uint8)
    mm = np.zeros(1, dtype=np.float64)
    lib().oracle_bp_traj(code._h, _p(lam), _p(s), int(iters), float(alpha), 0, None, None, None, _p(mm))
    return float(mm[0])


def lsd(code: Code, s: np.ndarray, llr: np.ndarray, mu: int = 0, omega: np.ndarray | None = None,
        force_merge: bool = False):
    """One shot of LSD-mu on soft information llr -> (corr uint8[n], status, stats[7]):
    stats = clusters, largest cluster's columns, rounds, clustered columns, clustered checks,
    largest cluster's checks, sum of squared cluster column counts."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    corr = np.empty(code.n, dtype=np.uint8)
    stats = np.zeros(7, dtype=np.int32)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.int64)
    st = lib().oracle_lsd(code._h, _p(s), _p(llr), int(mu), None if om is None else _p(om),
                          int(force_merge), _p(corr), _p(stats))
    return corr, int(st), stats


def lsd_cs(code: Code, s: np.ndarray, llr: np.ndarray, mu: int, cs_order: int, omega: np.ndarray):
    """One shot of LSD-mu (mu extra growth rounds) with local OSD-CS of order cs_order
    -> (corr uint8[n], status, stats[7]) as lsd()."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    corr = np.empty(code.n, dtype=np.uint8)
    stats = np.zeros(7, dtype=np.int32)
    om = np.ascontiguousarray(omega, dtype=np.int64)
    st = lib().oracle_lsd_cs(code._h, _p(s), _p(llr), int(mu), int(cs_order), _p(om), _p(corr), _p(stats))
    return corr, int(st), stats


def error_clusters(code: Code, e: np.ndarray):
    """Optimal factorization of one error (Appendix A): (nu, kappa, total faults, sum of squared
    cluster sizes) of the connected components of its faults in the fault graph."""
    e = np.ascontiguousarray(e, dtype=np.uint8)
    out = np.zeros(4, dtype=np.int64)
    lib().oracle_error_clusters(code._h, _p(e), _p(out))
    return tuple(int(x) for x in out)


def cluster_summary(nu, kappa, total, sumsq):
    """Per-shot nu, kappa and kappa_alpha = sum |C|^2 / sum |C| (the expected size of the
    cluster a random member fault belongs to, Appendix A) as float arrays; shots with no
    cluster get kappa_alpha 0."""
    total = np.asarray(total, dtype=np.float64)
    return (np.asarray(nu, np.float64), np.asarray(kappa, np.float64),
            np.where(total > 0, np.asarray(sumsq, np.float64) / np.maximum(total, 1), 0.0))


def osd0(code: Code, s: np.ndarray, llr: np.ndarray):
    s = np.ascontiguousarray(s, dtype=np.uint8)
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    corr = np.empty(code.n, dtype=np.uint8)
    st = lib().oracle_osd0(code._h, _p(s), _p(llr), _p(corr))
    return corr, int(st)


def osd_cs(code: Code, s: np.ndarray, llr: np.ndarray, cs_order: int, omega: np.ndarray):
    """Global OSD-CS of order cs_order on soft information llr -> (corr uint8[n], status): the
    combination sweep over all non-pivot columns of OSD-0's reliability-ordered elimination."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    corr = np.empty(code.n, dtype=np.uint8)
    om = np.ascontiguousarray(omega, dtype=np.int64)
    st = lib().oracle_osd_cs(code._h, _p(s), _p(llr), int(cs_order), _p(om), _p(corr))
    return corr, int(st)


def decode_batch(code: Code, lam: np.ndarray, S: np.ndarray, max_iter: int, alpha: float = 0.625,
                 mu: int = 0, omega: np.ndarray | None = None, nthreads: int = 0,
                 want_llr: bool = False):
    """BP then (if BP fails) LSD-mu, per shot -> (corr [B,n], status [B], iters [B], llr|None)."""
    S = np.ascontiguousarray(S, dtype=np.uint8)
    B = S.shape[0]
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    corr = np.empty((B, code.n), dtype=np.uint8)
    status = np.empty(B, dtype=np.uint8)
    iters = np.empty(B, dtype=np.int32)
    llr = np.empty((B, code.n), dtype=np.float64) if want_llr else None
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.int64)
    lib().oracle_decode_batch(code._h, _p(lam), _p(S), B, int(max_iter), float(alpha), int(mu),
                              None if om is None else _p(om), _p(corr), _p(status), _p(iters),
                              None if llr is None else _p(llr), int(nthreads))
    return corr, status, iters, llr


def max_threads() -> int:
    return int(lib().oracle_max_threads())
