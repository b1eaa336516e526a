"""Seeded builders for the check matrices the decoder is exercised on.

These are input generators only: they construct sparse GF(2) matrices (and, for
CSS codes, the conjugate check matrix used to score logical failures).  They
hold none of the decoder's arithmetic and are shared by the oracle side and the
GPU side of the tests and the benchmark.

Families (the decoding problem and the Tanner graph are defined in the paper's
Sec. 2.1; the code families are the ones its numerical results use):

* ``surface_hgp(d)``   -- unrotated distance-d surface code built as the
  hypergraph product of the open length-d repetition code (code capacity,
  X errors decoded with H_X).
* ``bivariate_bicycle(l, m, a_terms, b_terms)`` -- H_X = [A|B], H_Z = [B^T|A^T]
  with A, B sums of monomials in the commuting cyclic shifts x = S_l (x) I_m and
  y = I_l (x) S_m.
* ``random_34_hgp(n_cl, seed)`` -- hypergraph product of a seeded random
  (3,4)-regular classical LDPC code with no 4-cycles (girth >= 6) and full
  row rank.
* ``synthetic_dem(...)`` -- a band-diagonal sparse detector matrix shaped like a
  12-round circuit-level detector error model, with log-uniform fault priors.
* ``round_dem(code, rounds, p_data, p_meas)`` -- the detector error model of a memory
  experiment with noisy syndrome rounds (phenomenological noise: data flips before every
  round, flipped measurements) followed by one perfect round, with detectors per round and
  the code's logicals carried over to the data faults; the multi-round workload of the
  overlapping-window decoder.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np


@dataclasses.dataclass
class CheckMatrix:
    """A sparse GF(2) matrix H (rows = detectors/checks, cols = faults)."""

    name: str
    H: np.ndarray                     # uint8 dense m x n (small enough for all workloads here)
    priors: np.ndarray                # float64 [n], 0 < p_j < 1
    Hz: Optional[np.ndarray] = None   # conjugate checks (CSS), used only to score failures
    logicals: Optional[np.ndarray] = None  # uint8 [k, n]: residual r fails iff logicals @ r != 0
    det_round: Optional[np.ndarray] = None  # int32 [m]: syndrome round of each detector (multi-round DEMs)

    @property
    def m(self) -> int:
        return int(self.H.shape[0])

    @property
    def n(self) -> int:
        return int(self.H.shape[1])

    def csr(self):
        """(row_ptr int32[m+1], col_idx int32[nnz]) with sorted unique columns per row."""
        rows, cols = np.nonzero(self.H)
        order = np.lexsort((cols, rows))
        rows, cols = rows[order], cols[order]
        row_ptr = np.zeros(self.m + 1, dtype=np.int32)
        np.add.at(row_ptr, rows + 1, 1)
        row_ptr = np.cumsum(row_ptr).astype(np.int32)
        return row_ptr, cols.astype(np.int32)

    @property
    def nnz(self) -> int:
        return int(self.H.sum())


# ---------------------------------------------------------------------------
# small GF(2) helpers used only for code construction (rank checks, logicals)
# ---------------------------------------------------------------------------

def _gf2_row_reduce(A: np.ndarray):
    """Row-reduce a copy of A over GF(2); return (reduced, pivot_cols)."""
    M = (A.copy() & 1).astype(np.uint8)
    rows, cols = M.shape
    pivots = []
    r = 0
    for c in range(cols):
        if r >= rows:
            break
        nz = np.nonzero(M[r:, c])[0]
        if nz.size == 0:
            continue
        p = r + nz[0]
        if p != r:
            M[[r, p]] = M[[p, r]]
        others = np.nonzero(M[:, c])[0]
        others = others[others != r]
        M[others] ^= M[r]
        pivots.append(c)
        r += 1
    return M, pivots


def gf2_rank(A: np.ndarray) -> int:
    return len(_gf2_row_reduce(A)[1])


def gf2_nullspace(A: np.ndarray) -> np.ndarray:
    """Basis (rows) of {x : A x = 0} over GF(2)."""
    R, piv = _gf2_row_reduce(A)
    n = A.shape[1]
    free = [c for c in range(n) if c not in set(piv)]
    basis = []
    for f in free:
        x = np.zeros(n, dtype=np.uint8)
        x[f] = 1
        for i, pc in enumerate(piv):
            x[pc] = R[i, f]
        basis.append(x)
    return np.array(basis, dtype=np.uint8).reshape(len(basis), n)


def css_logicals(Hx: np.ndarray, Hz: np.ndarray) -> np.ndarray:
    """Representatives of ker(Hz) / rowspace(Hx).

    A residual r = e + e_hat with Hx r = 0 is a stabilizer (Hz-rowspace) iff it is
    orthogonal to all of ker(Hz); since rowspace(Hx) is orthogonal to r anyway, it
    suffices to test the k coset representatives returned here.  Rows are inserted
    into one echelon basis (as Python-int bitsets): first Hx, then ker(Hz); the
    ker(Hz) vectors that raise the rank are the representatives.
    """
    def as_int(v):
        return int("".join("1" if b else "0" for b in v[::-1]) or "0", 2)

    basis = {}  # leading bit -> row

    def insert(x):
        while x:
            top = x.bit_length() - 1
            if top in basis:
                x ^= basis[top]
            else:
                basis[top] = x
                return True
        return False

    for row in Hx:
        insert(as_int(row))
    reps = [v for v in gf2_nullspace(Hz) if insert(as_int(v))]
    return np.array(reps, dtype=np.uint8).reshape(len(reps), Hx.shape[1])


def _uniform_priors(n: int, p: float) -> np.ndarray:
    return np.full(n, float(p), dtype=np.float64)


# ---------------------------------------------------------------------------
# families
# ---------------------------------------------------------------------------

def repetition_code(d: int) -> np.ndarray:
    """Open repetition code: (d-1) x d, row i has ones at columns i, i+1."""
    H = np.zeros((d - 1, d), dtype=np.uint8)
    for i in range(d - 1):
        H[i, i] = H[i, i + 1] = 1
    return H


def hypergraph_product(H1: np.ndarray, H2: np.ndarray):
    """HGP(H1, H2): Hx = [H1 (x) I_n2 | I_r1 (x) H2^T], Hz = [I_n1 (x) H2 | H1^T (x) I_r2]."""
    r1, n1 = H1.shape
    r2, n2 = H2.shape
    Hx = np.hstack([np.kron(H1, np.eye(n2, dtype=np.uint8)),
                    np.kron(np.eye(r1, dtype=np.uint8), H2.T)]) & 1
    Hz = np.hstack([np.kron(np.eye(n1, dtype=np.uint8), H2),
                    np.kron(H1.T, np.eye(r2, dtype=np.uint8))]) & 1
    return Hx.astype(np.uint8), Hz.astype(np.uint8)


def surface_hgp(d: int = 5, p: float = 0.05) -> CheckMatrix:
    Hrep = repetition_code(d)
    Hx, Hz = hypergraph_product(Hrep, Hrep)
    return CheckMatrix(name=f"surface_d{d}_hgp", H=Hx, priors=_uniform_priors(Hx.shape[1], p),
                       Hz=Hz, logicals=css_logicals(Hx, Hz))


def _shift(l: int) -> np.ndarray:
    S = np.zeros((l, l), dtype=np.uint8)
    for i in range(l):
        S[i, (i + 1) % l] = 1
    return S


def bivariate_bicycle(l: int = 12, m: int = 6,
                      a_terms: Sequence = (("x", 3), ("y", 1), ("y", 2)),
                      b_terms: Sequence = (("y", 3), ("x", 1), ("x", 2)),
                      p: float = 0.05) -> CheckMatrix:
    """BB code; defaults give [[144,12,12]] (A = x^3+y+y^2, B = y^3+x+x^2)."""
    x = np.kron(_shift(l), np.eye(m, dtype=np.uint8))
    y = np.kron(np.eye(l, dtype=np.uint8), _shift(m))

    def poly(terms):
        acc = np.zeros((l * m, l * m), dtype=np.int64)
        for var, e in terms:
            base = x if var == "x" else y
            acc += np.linalg.matrix_power(base.astype(np.int64), e)
        return (acc & 1).astype(np.uint8)

    A, B = poly(a_terms), poly(b_terms)
    Hx = np.hstack([A, B])
    Hz = np.hstack([B.T, A.T])
    return CheckMatrix(name=f"bb_{l}x{m}", H=Hx, priors=_uniform_priors(Hx.shape[1], p),
                       Hz=Hz, logicals=css_logicals(Hx, Hz))


def _random_34_regular(n_cl: int, rng: np.random.Generator, max_tries: int = 20000) -> np.ndarray:
    """Random (3,4)-regular classical code (3n/4 x n), girth >= 6, full row rank.

    Columns are filled one at a time: each picks 3 distinct checks with free sockets,
    weighted by the remaining socket count, avoiding any check pair already used by an
    earlier column (a 4-cycle).  Dead ends and rank-deficient draws restart.
    """
    assert n_cl % 4 == 0
    r = 3 * n_cl // 4
    for _ in range(max_tries):
        H = np.zeros((r, n_cl), dtype=np.uint8)
        free = np.full(r, 4, dtype=np.int64)
        pair_used = np.zeros((r, r), dtype=bool)
        ok = True
        for j in range(n_cl):
            chosen = []
            for _k in range(3):
                cand = [i for i in range(r) if free[i] > 0 and i not in chosen
                        and not any(pair_used[i, c] for c in chosen)]
                if not cand:
                    ok = False
                    break
                w = free[cand].astype(np.float64)
                chosen.append(int(rng.choice(cand, p=w / w.sum())))
            if not ok:
                break
            for a in chosen:
                free[a] -= 1
                for b in chosen:
                    if a != b:
                        pair_used[a, b] = True
            H[chosen, j] = 1
        if not ok or gf2_rank(H) != r:
            continue
        return H
    raise RuntimeError("no (3,4)-regular code found")


def random_34_hgp(n_cl: int = 16, seed: int = 1, p: float = 0.03) -> CheckMatrix:
    rng = np.random.Generator(np.random.Philox(seed))
    H1 = _random_34_regular(n_cl, rng)
    Hx, Hz = hypergraph_product(H1, H1)
    return CheckMatrix(name=f"hgp34_n{n_cl}_s{seed}", H=Hx, priors=_uniform_priors(Hx.shape[1], p),
                       Hz=Hz, logicals=css_logicals(Hx, Hz))


def synthetic_dem(n_det: int = 936, n_fault: int = 8800, rounds: int = 12, max_row: int = 30,
                  seed: int = 7, p_lo: float = 1e-4, p_hi: float = 1e-2,
                  weight_probs=(0.45, 0.40, 0.08, 0.04, 0.03)) -> CheckMatrix:
    """Band-diagonal detector matrix shaped like a multi-round circuit-level DEM.

    Detectors are split into `rounds` bands; fault j lives in band b = floor((rounds-1)*j/n)
    and touches w in {2..6} detectors (probabilities `weight_probs`) drawn from detector
    bands b and b+1 among detectors whose load is still below `max_row`.  Duplicate columns
    are redrawn; every detector ends with weight >= 2.  Priors are log-uniform.
    """
    rng = np.random.Generator(np.random.Philox(seed))
    band = n_det // rounds
    H = np.zeros((n_det, n_fault), dtype=np.uint8)
    load = np.zeros(n_det, dtype=np.int64)
    seen = set()
    weights = np.arange(2, 2 + len(weight_probs))
    for j in range(n_fault):
        b = ((rounds - 1) * j) // n_fault          # fault bands 0..rounds-2 span detector bands b, b+1
        lo, hi = b * band, min(n_det, (b + 2) * band)
        cand = np.arange(lo, hi)
        cand = cand[load[cand] < max_row]
        for _ in range(1000):
            w = min(int(rng.choice(weights, p=np.asarray(weight_probs))), cand.size)
            sup = tuple(sorted(rng.choice(cand, size=w, replace=False).tolist()))
            if sup not in seen:
                break
        seen.add(sup)
        H[list(sup), j] = 1
        load[list(sup)] += 1
    # every detector needs weight >= 2 for min-sum: attach light detectors to extra faults
    for i in np.nonzero(load < 2)[0]:
        b = min(i // band, rounds - 2)
        js = np.arange((b * n_fault) // (rounds - 1), ((b + 1) * n_fault) // (rounds - 1))
        while load[i] < 2:
            j = int(rng.choice(js))
            if H[i, j] == 0:
                H[i, j] = 1
                load[i] += 1
    priors = np.exp(rng.uniform(np.log(p_lo), np.log(p_hi), size=n_fault))
    return CheckMatrix(name=f"dem_{n_det}x{n_fault}_s{seed}", H=H, priors=priors)


def round_dem(code: CheckMatrix, rounds: int = 12, p_data: float = 0.01, p_meas: float = 0.01) -> CheckMatrix:
    """Memory experiment over `rounds` noisy syndrome rounds plus one perfect final round.

    Detector (r, i) = s_i(r) xor s_i(r-1), r = 0..rounds (s(-1) = 0).  A data flip on fault j
    before round r flips s_i(r'), r' >= r, for every check i of j, i.e. detectors (r, i) only;
    a flipped measurement of check i in round r < rounds flips detectors (r, i) and (r+1, i).
    Columns: data faults (r, j) at column r*n + j, then measurement faults (r, i) at
    (rounds+1)*n + r*m + i.  The logical class of a residual is that of its summed data part,
    so each data fault carries its code column of the logicals; measurement faults carry none.
    det_round[(r, i)] = r.
    """
    H0 = code.H.astype(np.uint8)
    m, n = H0.shape
    R = rounds
    nd, nm = (R + 1) * n, R * m
    H = np.zeros(((R + 1) * m, nd + nm), dtype=np.uint8)
    for r in range(R + 1):
        H[r * m:(r + 1) * m, r * n:(r + 1) * n] = H0
    for r in range(R):
        for i in range(m):
            H[r * m + i, nd + r * m + i] = 1
            H[(r + 1) * m + i, nd + r * m + i] = 1
    priors = np.concatenate([np.full(nd, p_data), np.full(nm, p_meas)])
    logicals = None
    if code.logicals is not None:
        logicals = np.concatenate([np.tile(code.logicals, (1, R + 1)),
                                   np.zeros((code.logicals.shape[0], nm), dtype=np.uint8)], axis=1)
    det_round = np.repeat(np.arange(R + 1, dtype=np.int32), m)
    return CheckMatrix(name=f"rounds{R}_{code.name}", H=H, priors=priors, logicals=logicals, det_round=det_round)
