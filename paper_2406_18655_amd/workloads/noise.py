"""Seeded code-capacity noise and syndromes (input generation only).

Errors are i.i.d. Bernoulli(p_j) per fault (the paper's code-capacity setting,
Appendix D) and the syndrome is s = H e over GF(2) (Sec. 2.1).  Shots are drawn
in fixed blocks, each from its own Philox key (seed, block), so any shot range
can be regenerated on its own.
"""
from __future__ import annotations

import numpy as np

from .codes import CheckMatrix

BLOCK = 4096


def _block_rng(seed: int, block: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=np.array([seed & (2**64 - 1), block], dtype=np.uint64)))


def sample_errors(priors: np.ndarray, shots: int, seed: int, start: int = 0) -> np.ndarray:
    """uint8 [shots, n] with e_sj ~ Bernoulli(priors[j]); shot i depends only on (seed, start+i)."""
    n = priors.shape[0]
    out = np.empty((shots, n), dtype=np.uint8)
    thr = priors.astype(np.float64)
    i = 0
    while i < shots:
        g = start + i
        b, off = divmod(g, BLOCK)
        take = min(shots - i, BLOCK - off)
        u = _block_rng(seed, b).random((BLOCK, n))[off:off + take]
        out[i:i + take] = (u < thr[None, :]).astype(np.uint8)
        i += take
    return out


def syndromes(code: CheckMatrix, errors: np.ndarray) -> np.ndarray:
    """uint8 [shots, m]: s = H e mod 2 (sparse product, works for the large DEM too)."""
    import scipy.sparse as sp
    Hs = sp.csr_matrix(code.H.astype(np.int32))
    s = (Hs @ errors.T.astype(np.int32)).T
    return np.ascontiguousarray(np.asarray(s) & 1, dtype=np.uint8)


def sample(code: CheckMatrix, shots: int, seed: int, start: int = 0):
    """(errors uint8 [shots,n], syndromes uint8 [shots,m])."""
    e = sample_errors(code.priors, shots, seed, start)
    return e, syndromes(code, e)  # both C-contiguous


def logical_failures(code: CheckMatrix, errors: np.ndarray, corrections: np.ndarray) -> np.ndarray:
    """bool [shots]: residual r = e + e_hat is a logical error (or, without logicals, r != 0)."""
    r = (errors ^ corrections).astype(np.int32)
    if code.logicals is None:
        return r.any(axis=1)
    return ((r @ code.logicals.T.astype(np.int32)) & 1).any(axis=1)
