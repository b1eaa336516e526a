"""Exact quality bounds that pin the oracle's logical error rate on the surface code.

For X errors decoded with H_X, two errors are equivalent iff they differ by an element of
S = rowspace(H_Z); the 2^(m+k) cosets of S are labelled by (syndrome H_X e, logical class L e).
Coset probabilities under i.i.d. noise follow from Poisson summation over S^perp = ker(H_Z),
whose basis is the rows of H_X plus the logicals: P(y) = 2^-(m+k) sum_c (1-2p)^|u(c)| (-1)^(c.y),
a Walsh-Hadamard transform of size 2^(m+k).  The maximum-likelihood decoder picks the likelier
class per syndrome (exact failure rate LER_ML, a lower bound for every decoder); the
minimum-weight decoder picks the class with the lighter representative, whose weight is a
breadth-first distance in the coset graph (exact LER_MW, ties split evenly).  Decoding problem:
Sec. 2.1; code-capacity surface code results: Sec. 2.3.
"""
import itertools

import numpy as np

from paper_2406_18655_amd.workloads import surface_hgp, sample, logical_failures


def _bits(v):
    return int(sum(int(b) << k for k, b in enumerate(v)))


def coset_probabilities(code, p):
    """float64 [2^(m+k)]: index bits 0..m-1 = syndrome, bits m.. = logical class."""
    basis = [_bits(r) for r in code.H] + [_bits(r) for r in code.logicals]
    U = np.zeros(1, dtype=np.int64)
    for b in basis:
        U = np.concatenate([U, U ^ b])
    a = (1.0 - 2.0 * p) ** np.bitwise_count(U).astype(np.float64)
    h = 1
    while h < a.size:  # in-place fast Walsh-Hadamard transform
        a = a.reshape(-1, 2, h)
        x, y = a[:, 0, :].copy(), a[:, 1, :].copy()
        a[:, 0, :], a[:, 1, :] = x + y, x - y
        a = a.reshape(-1)
        h *= 2
    return a / a.size


def coset_min_weights(code):
    """int32 [2^(m+k)]: weight of the lightest error in each coset (BFS from the zero error)."""
    m, k = code.m, code.logicals.shape[0]
    gens = np.array([_bits(code.H[:, j]) | (_bits(code.logicals[:, j]) << m) for j in range(code.n)],
                    dtype=np.int64)
    dist = np.full(1 << (m + k), -1, dtype=np.int32)
    dist[0] = 0
    front, d = np.array([0], dtype=np.int64), 0
    while front.size:
        d += 1
        cand = np.unique((front[:, None] ^ gens[None, :]).reshape(-1))
        cand = cand[dist[cand] < 0]
        dist[cand] = d
        front = cand
    return dist


def exact_ml_mw(code, p):
    m = code.m
    P = coset_probabilities(code, p).reshape(2, 1 << m)
    D = coset_min_weights(code).reshape(2, 1 << m)
    ler_ml = float(1.0 - P.max(axis=0).sum())
    pick0, pick1, tie = D[0] < D[1], D[1] < D[0], D[0] == D[1]
    ler_mw = float((P[1] * pick0 + P[0] * pick1 + 0.5 * (P[0] + P[1]) * tie).sum())
    return P, D, ler_ml, ler_mw


def _syndrome_ids(S):
    return (S.astype(np.int64) << np.arange(S.shape[1])).sum(axis=1)


def test_d3_coset_transform_and_bfs_match_enumeration(oracle_mod):
    """The transform and the BFS against brute force over all 2^13 errors of the d=3 code;
    then the exact BP+LSD failure rate lies between ML and a small multiple of MW, and no
    returned correction is lighter than the lightest error with its syndrome."""
    c = surface_hgp(3, p=0.05)
    n, m = c.n, c.m
    errs = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.uint8)
    S = ((errs.astype(int) @ c.H.T.astype(int)) % 2).astype(np.uint8)
    cls = ((errs.astype(int) @ c.logicals.T.astype(int)) % 2)[:, 0]
    idx = _syndrome_ids(S) | (cls << m)
    w = errs.sum(1)
    code = oracle_mod.Code.from_dense(c.H)
    corr, _, _, _ = oracle_mod.decode_batch(code, oracle_mod.llr_from_priors(c.priors), S, 30)
    fail = logical_failures(c, errs, corr)
    for p in (0.01, 0.05, 0.1):
        Pw = p ** w * (1 - p) ** (n - w)
        direct = np.zeros(1 << (m + 1))
        np.add.at(direct, idx, Pw)
        P, D, ler_ml, ler_mw = exact_ml_mw(c, p)
        np.testing.assert_allclose(P.reshape(-1), direct, rtol=0, atol=1e-14)  # rounding of 2^7-term sums
        ler = float(Pw[fail].sum())
        assert ler_ml <= ler_mw + 1e-15
        assert ler >= ler_ml - 1e-12
        assert ler <= 1.5 * ler_mw, (p, ler, ler_mw)
    mins = np.full(1 << (m + 1), 99)
    np.minimum.at(mins, idx, w)
    np.testing.assert_array_equal(coset_min_weights(c), mins)
    sid = _syndrome_ids(S)
    Dm = mins.reshape(2, -1).min(axis=0)
    assert (corr.sum(1) >= Dm[sid]).all()


def test_d5_exact_ml_and_mw_bound_the_oracle(oracle_mod, capsys):
    """Distance-5 surface code (H_X 20 x 41), p = 0.05, the 10^4 seeded shots of the parity
    tests.  Exact LER_ML (2^21 cosets) and LER_MW; the oracle's BP+LSD rate must not beat ML
    by more than 2 sigma and stays within 3 sigma of MW; every weight <= 2 error is corrected;
    no correction is lighter than the lightest error with its syndrome."""
    c = surface_hgp(5, p=0.05)
    P, D, ler_ml, ler_mw = exact_ml_mw(c, 0.05)
    assert abs(P.sum() - 1.0) < 1e-12
    assert ler_ml < ler_mw
    code = oracle_mod.Code.from_dense(c.H)
    lam = oracle_mod.llr_from_priors(c.priors)
    N = 10000
    e, S = sample(c, N, seed=2024)
    corr, _, _, _ = oracle_mod.decode_batch(code, lam, S, 30)
    assert (((corr.astype(int) @ c.H.T.astype(int)) % 2) == S).all()
    ler = float(logical_failures(c, e, corr).mean())
    sig_ml = np.sqrt(ler_ml * (1 - ler_ml) / N)
    sig_mw = np.sqrt(ler_mw * (1 - ler_mw) / N)
    with capsys.disabled():
        print(f"\n[surface d=5 p=0.05] exact LER_ML={ler_ml:.5f} LER_MW={ler_mw:.5f}; "
              f"oracle BP+LSD on {N} shots {ler:.5f} (sigma {sig_mw:.5f})")
    assert ler >= ler_ml - 2 * sig_ml
    assert ler <= ler_mw + 3 * sig_mw
    Dm = D.min(axis=0)
    assert (corr.sum(1) >= Dm[_syndrome_ids(S)]).all()
    small = [np.zeros(c.n, np.uint8)]
    for wt in (1, 2):
        for comb in itertools.combinations(range(c.n), wt):
            x = np.zeros(c.n, np.uint8)
            x[list(comb)] = 1
            small.append(x)
    E = np.array(small)
    SE = ((E.astype(int) @ c.H.T.astype(int)) % 2).astype(np.uint8)
    cs, _, _, _ = oracle_mod.decode_batch(code, lam, SE, 30)
    assert not logical_failures(c, E, cs).any()
