"""GPU parity on the synthetic circuit-level-shaped detector error model (936 x 8800,
log-uniform priors): one-workgroup-per-shot BP and LSD of order mu (Appendix D)."""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import synthetic_dem, bivariate_bicycle, sample

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


@pytest.fixture(scope="module")
def dem():
    return synthetic_dem()


def _dec(code, T, B, mu=0, flags=0):
    bc = binding.Code.from_dense(code.H)
    return bc, binding.Decoder(bc, code.priors, B, max_iter=T, lsd_order=mu, flags=flags)


@pytest.mark.parametrize("T", [3, 40, 100])
def test_dem_bp_posteriors(oracle_mod, dem, T):
    """Fixed T, no early exit; T = 100 is the configured budget, where magnitudes reach the 2^64
    clamp on both sides."""
    print(f"case dem_bp T={T}", flush=True)
    e, S = sample(dem, 12, seed=5)
    _, dec = _dec(dem, T, 12, flags=binding.FLAG_NO_EARLY_EXIT)
    llr, hard, info = dec.bp(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    L32 = llr.cpu().numpy().astype(np.float64)
    oc = oracle_mod.Code.from_dense(dem.H)
    lam = oracle_mod.llr_from_priors(dem.priors)
    floor = np.abs(lam).min()
    for b in range(12):
        conv, it, L64, h64 = oracle_mod.bp(oc, lam, S[b], T, early_exit=False)
        err = np.abs(L32[b] - L64) / np.maximum(np.abs(L64), floor)
        assert err.max() <= 1e-4, (b, float(err.max()))


@pytest.mark.parametrize("mu", [0, 10])
def test_dem_lsd_mu_bit_exact(oracle_mod, dem, mu):
    print(f"case dem_lsd mu={mu}", flush=True)
    e, S = sample(dem, 600, seed=8)
    _, dec = _dec(dem, 100, 600, mu=mu)
    llr, hard, info = dec.bp(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    inf = binding.parse_info(info)
    idx = np.nonzero((inf["status"] & 1) == 0)[0][:60]
    assert len(idx) >= 30
    L = llr.cpu().numpy()[idx]
    corr, linfo = dec.lsd(torch.from_numpy(S[idx]).cuda(), torch.from_numpy(L).cuda())
    torch.cuda.synchronize()
    corr = corr.cpu().numpy()
    li = binding.parse_info(linfo)
    oc = oracle_mod.Code.from_dense(dem.H)
    om = oracle_mod.omega_from_llr(oracle_mod.llr_from_priors(dem.priors))
    for k, b in enumerate(idx):
        want, st, stats = oracle_mod.lsd(oc, S[b], L[k].astype(np.float64), mu=mu, omega=om)
        assert not (li["status"][k] & binding.ST_OVERFLOW), k
        assert (corr[k] == want).all(), (k, mu)
        assert li["rounds"][k] == stats[2] and li["n_clusters"][k] == stats[0], k


def test_dem_decode_word_error_within_2sigma(oracle_mod, dem):
    print("case dem_decode", flush=True)
    B = 3000
    e, S = sample(dem, B, seed=77)
    _, dec = _dec(dem, 100, B, mu=10)
    corr, info = dec.decode(torch.from_numpy(S).cuda(), want_info=True)
    torch.cuda.synchronize()
    corr = corr.cpu().numpy()
    assert (((corr.astype(np.int64) @ dem.H.T.astype(np.int64)) % 2) == S).all()
    oc = oracle_mod.Code.from_dense(dem.H)
    lam = oracle_mod.llr_from_priors(dem.priors)
    om = oracle_mod.omega_from_llr(lam)
    ocorr, ost, oit, _ = oracle_mod.decode_batch(oc, lam, S, 100, mu=10, omega=om)
    f_gpu = (corr != e).any(1)
    f_ref = (ocorr != e).any(1)
    p = max(f_ref.mean(), 1.0 / B)
    two_sigma = 2 * np.sqrt(p * (1 - p) / B)
    print(f"word error gpu={f_gpu.mean():.4f} oracle={f_ref.mean():.4f} 2sigma={two_sigma:.4f}")
    assert abs(f_gpu.mean() - f_ref.mean()) <= two_sigma


def test_bb_lsd_mu_bit_exact(oracle_mod):
    code = bivariate_bicycle(p=0.06)
    e, S = sample(code, 400, seed=19)
    _, dec = _dec(code, 30, 400, mu=4)
    llr, hard, info = dec.bp(torch.from_numpy(S).cuda())
    L = llr.cpu().numpy()
    corr, li = dec.lsd(torch.from_numpy(S).cuda(), llr)
    torch.cuda.synchronize()
    corr = corr.cpu().numpy()
    oc = oracle_mod.Code.from_dense(code.H)
    om = oracle_mod.omega_from_llr(oracle_mod.llr_from_priors(code.priors))
    for b in range(400):
        want, st, stats = oracle_mod.lsd(oc, S[b], L[b].astype(np.float64), mu=4, omega=om)
        assert (corr[b] == want).all(), b


def test_dem_overflowing_shot_decoded_in_batch(oracle_mod, dem):
    """A syndrome with more flipped detectors than the LSD kernel's capacity (256 local rows with
    LSD order 10) goes on to the overflow kernels: it comes back decoded (H e_hat = s, equal to the
    oracle on the same posteriors, no OVERFLOW flag), and its neighbours in the batch are
    unaffected."""
    code = dem
    bc = binding.Code.from_dense(code.H)
    rng = np.random.default_rng(5)
    e, S = sample(code, 64, seed=8)
    S = S.copy()
    S[7] = (rng.random(code.m) < 0.5).astype(np.uint8)  # ~470 flipped detectors
    dec = binding.Decoder(bc, code.priors, 64, max_iter=20, lsd_order=10)
    s = torch.from_numpy(S).cuda()
    corr, info = dec.decode(s, want_info=True)
    llr, _, _ = dec.bp(s)
    corr, inf = corr.cpu().numpy(), binding.parse_info(info)
    assert not (inf["status"][7] & binding.ST_OVERFLOW)
    assert (((corr[7].astype(np.int64) @ code.H.T.astype(np.int64)) & 1) == S[7]).all()
    oc = oracle_mod.Code.from_dense(code.H)
    om = oracle_mod.omega_from_llr(oracle_mod.llr_from_priors(code.priors))
    want, st, stats = oracle_mod.lsd(oc, S[7], llr.cpu().numpy()[7].astype(np.float64), mu=10, omega=om)
    assert stats[4] > 256
    np.testing.assert_array_equal(corr[7], want)
    ok = np.ones(64, dtype=bool)
    ok[7] = False
    ref = dec.decode(torch.from_numpy(np.ascontiguousarray(S[ok])).cuda()).cpu().numpy()
    np.testing.assert_array_equal(corr[ok], ref)


def test_dem_batch_size_invariance(dem):
    """Shots decode the same alone, in small ragged batches and in a full batch (one workgroup per
    shot, no cross-shot state)."""
    code = dem
    bc = binding.Code.from_dense(code.H)
    e, S = sample(code, 300, seed=9)
    dec = binding.Decoder(bc, code.priors, 300, max_iter=100, lsd_order=10)
    full = dec.decode(torch.from_numpy(S).cuda()).cpu().numpy()
    for lo, hi in ((0, 1), (1, 4), (4, 37), (37, 300)):
        part = dec.decode(torch.from_numpy(np.ascontiguousarray(S[lo:hi])).cuda()).cpu().numpy()
        np.testing.assert_array_equal(part, full[lo:hi])


def test_dem_lsd10_bit_exact_on_every_failed_shot(oracle_mod, dem):
    """LSD-10 on all BP-100 failures of an 8,192-shot batch (more than a thousand shots, clusters
    of up to ~130 detectors) against the oracle on the same float32 posteriors, through the full
    decode: corrections, status, cluster counts and rounds."""
    B = 8192
    print("case dem_lsd10_all_failed", flush=True)
    e, S = sample(dem, B, seed=88)
    _, dec = _dec(dem, 100, B, mu=10)
    s = torch.from_numpy(S).cuda()
    corr, info = dec.decode(s, want_info=True)
    llr, hard, binfo = dec.bp(s)
    torch.cuda.synchronize()
    corr, L = corr.cpu().numpy(), llr.cpu().numpy()
    inf, bi = binding.parse_info(info), binding.parse_info(binfo)
    idx = np.nonzero((bi["status"] & 1) == 0)[0]
    assert len(idx) >= 1000, len(idx)
    oc = oracle_mod.Code.from_dense(dem.H)
    om = oracle_mod.omega_from_llr(oracle_mod.llr_from_priors(dem.priors))
    biggest = 0
    for b in idx:
        want, st, stats = oracle_mod.lsd(oc, S[b], L[b].astype(np.float64), mu=10, omega=om)
        assert not (inf["status"][b] & binding.ST_OVERFLOW), b
        assert (corr[b] == want).all(), b
        assert (inf["status"][b] & 0x0C) == (st & 0x0C), b
        assert inf["rounds"][b] == stats[2] and inf["n_clusters"][b] == stats[0], b
        assert inf["max_cluster_cols"][b] == stats[1], b
        biggest = max(biggest, int(stats[5]))
    print(f"{len(idx)} LSD-10 shots bit-exact; largest cluster {biggest} detectors")


def test_large_graph_bp_mixed_weights(oracle_mod):
    """The one-workgroup-per-shot BP on a graph built to reach its paths the DEM does not: columns
    of weight 1 to 7 (every degree-specialised body of the fault update, and the wave-uniform
    general one), rows of weight 2 to 32 in one weight-ordered sweep (wavefronts of one row weight
    and mixed ones), more faults than the slot BP holds.  Posteriors after 20 iterations without
    early exit against the float64 oracle."""
    rng = np.random.default_rng(77)
    m, n = 800, 6000
    H = np.zeros((m, n), dtype=np.uint8)
    rw = np.zeros(m, dtype=np.int64)
    w = rng.choice(np.arange(1, 8), size=n, p=[0.1, 0.3, 0.3, 0.15, 0.08, 0.05, 0.02])
    for j in range(n):
        ok = np.nonzero(rw < 32)[0]
        rows = rng.choice(ok, size=int(w[j]), replace=False)
        H[rows, j] = 1
        rw[rows] += 1
    for i in np.nonzero(rw < 2)[0]:
        j = rng.choice(np.nonzero(H.sum(0) < 7)[0], size=2 - int(rw[i]), replace=False)
        H[i, j] = 1
    assert H.sum(1).max() <= 32 and H.sum(1).min() >= 2 and set(H.sum(0)) >= {1, 2, 3, 4, 5, 6, 7}
    priors = rng.uniform(0.001, 0.05, size=n)
    e = (rng.random((6, n)) < priors).astype(np.uint8)
    S = ((e.astype(np.int64) @ H.T.astype(np.int64)) & 1).astype(np.uint8)
    bc = binding.Code.from_dense(H)
    dec = binding.Decoder(bc, priors, 6, max_iter=20, flags=binding.FLAG_NO_EARLY_EXIT)
    llr, hard, info = dec.bp(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    L32 = llr.cpu().numpy().astype(np.float64)
    oc = oracle_mod.Code.from_dense(H)
    lam = oracle_mod.llr_from_priors(priors)
    floor = np.abs(lam).min()
    for b in range(6):
        conv, it, L64, h64 = oracle_mod.bp(oc, lam, S[b], 20, early_exit=False)
        err = np.abs(L32[b] - L64) / np.maximum(np.abs(L64), floor)
        assert err.max() <= 1e-4, (b, float(err.max()))
