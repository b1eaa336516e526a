"""Shots whose clusters outgrow the LSD kernel's register basis (more than 64 W local rows, or,
with LSD-mu, more than 64 W dependent columns) are decoded again by the overflow kernels (512
local rows with the basis in LDS, then 1024 with the basis in device memory): they must come back
bit-exact against the oracle like every other shot (Sec. 4.1 / Alg. 1 with Appendix B's rounds;
Appendix D for LSD-mu), never as a zero correction."""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import synthetic_dem, random_34_hgp, sample

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def _heavy_batch(code, T, base_shots, fracs, seed):
    """BP-failed shots of the code plus random syndromes with the given flipped fractions
    (every syndrome of a full-row-rank H is in its image), with float32 BP posteriors."""
    rng = np.random.default_rng(seed)
    e, S = sample(code, base_shots, seed=seed)
    heavy = (rng.random((len(fracs), code.m)) < np.array(fracs)[:, None]).astype(np.uint8)
    S = np.ascontiguousarray(np.concatenate([S, heavy]))
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, S.shape[0], max_iter=T)
    llr, hard, info = dec.bp(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    inf = binding.parse_info(info)
    keep = np.nonzero((inf["status"] & 1) == 0)[0]
    return bc, np.ascontiguousarray(S[keep]), np.ascontiguousarray(llr.cpu().numpy()[keep])


@pytest.mark.parametrize("mu", [0, 10])
def test_dem_overflowing_shots_bit_exact(oracle_mod, mu):
    """Detector error model (936 detectors): ordinary BP failures and syndromes with 10-50 % of
    the detectors flipped, whose clusters reach 300-800 local rows (LSD kernel capacity 256)."""
    code = synthetic_dem()
    print(f"case wide_dem mu={mu}", flush=True)
    bc, S, L = _heavy_batch(code, 20, 200, [0.1, 0.2, 0.3, 0.4, 0.5, 0.6], seed=41)
    dec = binding.Decoder(bc, code.priors, S.shape[0], max_iter=20, lsd_order=mu)
    corr, info = dec.lsd(torch.from_numpy(S).cuda(), torch.from_numpy(L).cuda())
    torch.cuda.synchronize()
    corr, inf = corr.cpu().numpy(), binding.parse_info(info)
    oc = oracle_mod.Code.from_dense(code.H)
    om = oracle_mod.omega_from_llr(oracle_mod.llr_from_priors(code.priors))
    wide = 0
    for b in range(S.shape[0]):
        want, st, stats = oracle_mod.lsd(oc, S[b], L[b].astype(np.float64), mu=mu, omega=om)
        assert not (inf["status"][b] & binding.ST_OVERFLOW), b
        assert (corr[b] == want).all(), (b, int(stats[4]))
        assert (inf["status"][b] & 0x0C) == (st & 0x0C), b
        assert (inf["n_clusters"][b], inf["rounds"][b], inf["max_cluster_cols"][b]) == (stats[0], stats[2], stats[1]), b
        wide += int(stats[4] > 256)
    assert (((corr.astype(np.int64) @ code.H.T.astype(np.int64)) & 1) == S).all()
    print(f"{S.shape[0]} shots bit-exact, {wide} beyond 256 local rows")
    assert wide >= 4


def test_dem_decode_reaches_wide_path(oracle_mod):
    """The same heavy syndromes through the full decode (BP 20 + LSD-10): corrections equal the
    LSD-only entry point on BP's posteriors, and satisfy every syndrome."""
    code = synthetic_dem()
    bc, S, L = _heavy_batch(code, 20, 64, [0.15, 0.4], seed=43)
    dec = binding.Decoder(bc, code.priors, S.shape[0], max_iter=20, lsd_order=10)
    s = torch.from_numpy(S).cuda()
    full, info = dec.decode(s, want_info=True)
    ref, _ = dec.lsd(s, torch.from_numpy(L).cuda())
    torch.cuda.synchronize()
    full, ref, inf = full.cpu().numpy(), ref.cpu().numpy(), binding.parse_info(info)
    assert not (inf["status"] & binding.ST_OVERFLOW).any()
    np.testing.assert_array_equal(full, ref)
    assert (((full.astype(np.int64) @ code.H.T.astype(np.int64)) & 1) == S).all()


def test_hgp32_high_noise_bit_exact(oracle_mod):
    """HGP n = 1600 (768 checks) at p = 0.1, BP 30 + LSD-0 through the full decode: clusters
    beyond 256 local rows are common; every LSD shot bit-exact against the oracle on the same
    float32 posteriors."""
    code = random_34_hgp(32, p=0.1)
    print("case wide_hgp32", flush=True)
    B = 192
    e, S = sample(code, B, seed=45)
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, B, max_iter=30)
    s = torch.from_numpy(S).cuda()
    corr, info = dec.decode(s, want_info=True)
    llr, hard, binfo = dec.bp(s)
    torch.cuda.synchronize()
    corr, L, inf, bi = corr.cpu().numpy(), llr.cpu().numpy(), binding.parse_info(info), binding.parse_info(binfo)
    oc = oracle_mod.Code.from_dense(code.H)
    big = 0
    for b in np.nonzero((bi["status"] & 1) == 0)[0]:
        want, st, stats = oracle_mod.lsd(oc, S[b], L[b].astype(np.float64))
        assert not (inf["status"][b] & binding.ST_OVERFLOW), b
        assert (corr[b] == want).all(), (b, int(stats[4]))
        assert (inf["n_clusters"][b], inf["rounds"][b]) == (stats[0], stats[2]), b
        big += int(stats[4] > 256)
    print(f"{big} shots beyond 256 local rows")
    assert big >= 5
