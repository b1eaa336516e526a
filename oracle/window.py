"""Overlapping-window decoding of a multi-round detector error model (test infrastructure only).

The (w, c) window scheme the paper uses for its multi-round simulations (Sec. 4.3, numerical
decoding simulations; w = 3, c = 1): windows of w syndrome rounds slide forward by c rounds;
each window is decoded with BP + LSD on the detectors of its rounds and the faults whose
earliest detector lies in them, and only the faults of its first c rounds are committed (the
last window commits everything).  Committed faults update the syndrome the later windows see.
Written out plainly on top of the float64 oracle (oracle.decode_batch); shares nothing with the
library's window driver.
"""
from __future__ import annotations

import numpy as np

from . import Code, decode_batch, llr_from_priors, omega_from_llr


def fault_rounds(H: np.ndarray, det_round: np.ndarray) -> np.ndarray:
    """Round of each fault: the earliest round among its detectors."""
    H = np.asarray(H, dtype=np.uint8)
    big = np.iinfo(np.int32).max
    r = np.where(H.astype(bool), np.asarray(det_round)[:, None], big).min(axis=0)
    return r.astype(np.int64)


def windows(det_round: np.ndarray, w: int, c: int):
    """[(first round, last round + 1, commit rounds end), ...]: windows of w rounds every c
    rounds while a further window fits; the last one runs to the final round and commits all."""
    n_rounds = int(np.max(det_round)) + 1
    out, k = [], 0
    while k + w < n_rounds:
        out.append((k, k + w, k + c))
        k += c
    out.append((k, n_rounds, n_rounds))
    return out


def window_decode(H, priors, det_round, S, w: int, c: int, max_iter: int, mu: int = 0, alpha: float = 0.625):
    """Corrections uint8 [B, n] of the (w, c) window decoder for syndromes S [B, m]."""
    H = np.asarray(H, dtype=np.uint8)
    S = np.asarray(S, dtype=np.uint8)
    det_round = np.asarray(det_round)
    fr = fault_rounds(H, det_round)
    B, n = S.shape[0], H.shape[1]
    corr = np.zeros((B, n), dtype=np.uint8)
    for lo, hi, commit in windows(det_round, w, c):
        rows = np.nonzero((det_round >= lo) & (det_round < hi))[0]
        cols = np.nonzero((fr >= lo) & (fr < hi))[0]
        Hw = H[np.ix_(rows, cols)]
        # syndrome left after the faults committed so far
        s_res = (S[:, rows].astype(np.int64) + corr.astype(np.int64) @ H[rows].T.astype(np.int64)) & 1
        code = Code.from_dense(Hw)
        lam = llr_from_priors(priors[cols])
        om = omega_from_llr(lam) if mu > 0 else None
        ew, _, _, _ = decode_batch(code, lam, s_res.astype(np.uint8), max_iter, alpha=alpha, mu=mu, omega=om)
        keep = fr[cols] < commit
        corr[:, cols[keep]] = ew[:, keep]
    return corr


def per_cycle(p_total: float, cycles: int) -> float:
    """Per-cycle logical error rate: 1 - (1 - P_L)^(1 / N_c)."""
    return 1.0 - (1.0 - p_total) ** (1.0 / cycles)
