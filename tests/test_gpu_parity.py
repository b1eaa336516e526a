"""GPU parity: the HIP decoder (through the C ABI) against the CPU oracle on the same
seeded inputs.

Bars (from the decoder's stated tolerances):
  * BP posteriors in float32 within 1e-4 relative of the float64 oracle, relative to
    max(|L64|, lambda_floor) with lambda_floor = min_j |lambda_j|;
  * LSD bit-exact on identical float32 LLR inputs (index tie-breaking);
  * end-to-end logical error rate within 2 sigma (binomial, from the oracle's rate).
"""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
import _r24
from paper_2406_18655_amd.workloads import (bivariate_bicycle, surface_hgp, random_34_hgp, sample,
                                            logical_failures)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    _need_gpu()
    binding.lib()
    yield
    torch.cuda.synchronize()


def make(code, T, max_batch, flags=0):
    bc = binding.Code.from_dense(code.H)
    return bc, binding.Decoder(bc, code.priors, max_batch, max_iter=T, flags=flags)


def ocode(oracle_mod, code):
    return oracle_mod.Code.from_dense(code.H)


def syn_dev(S):
    return torch.from_numpy(np.ascontiguousarray(S)).cuda()


def check_syndromes(code, corr, S, ok_mask=None):
    got = (corr.astype(np.int64) @ code.H.T.astype(np.int64)) % 2
    good = (got == S).all(axis=1)
    if ok_mask is not None:
        good = good | ~ok_mask
    return good


# ------------------------------------------------------------------------------- BP

@pytest.mark.parametrize("which,T,shots", [("c1", 30, 512), ("c2", 1, 256), ("c2", 7, 512),
                                           ("c2", 50, 512), ("hgp16", 20, 128)])
def test_bp_posteriors_fixed_iterations(oracle_mod, which, T, shots):
    code = {"c1": lambda: surface_hgp(5, 0.05), "c2": lambda: bivariate_bicycle(p=0.05),
            "hgp16": lambda: random_34_hgp(16, p=0.03)}[which]()
    print(f"case bp_fixed {which} T={T} shots={shots}", flush=True)
    e, S = sample(code, shots, seed=100 + T)
    _, dec = make(code, T, shots, flags=binding.FLAG_NO_EARLY_EXIT)
    llr, hard, info = dec.bp(syn_dev(S))
    torch.cuda.synchronize()
    L32 = llr.cpu().numpy().astype(np.float64)
    inf = binding.parse_info(info)
    assert (inf["bp_iters"] == T).all()
    oc = ocode(oracle_mod, code)
    lam = oracle_mod.llr_from_priors(code.priors)
    floor = np.abs(lam).min()
    worst = 0.0
    for b in range(shots):
        conv, it, L64, h64 = oracle_mod.bp(oc, lam, S[b], T, early_exit=False)
        err = np.abs(L32[b] - L64) / np.maximum(np.abs(L64), floor)
        worst = max(worst, float(err.max()))
        assert err.max() <= 1e-4, (b, float(err.max()))
        assert bool(inf["status"][b] & 1) == conv
    print(f"worst relative error {worst:.3e}")


@pytest.mark.parametrize("T", [1, 3, 5])
def test_bp_short_budget_full_batch(oracle_mod, T):
    """A full 65,536-shot batch with a tiny iteration budget: slots retire almost in lockstep,
    so staging chunks drain in the same iteration as the next chunk lands (the queue hand-over
    between the two staging buffers).  Every shot must come back once, with the oracle's
    posteriors on a sample."""
    code = bivariate_bicycle(p=0.05)
    B = 65536
    print(f"case bp_short_budget T={T} shots={B}", flush=True)
    e, S = sample(code, B, seed=300 + T)
    _, dec = make(code, T, B)
    llr, hard, info = dec.bp(syn_dev(S))
    torch.cuda.synchronize()
    inf = binding.parse_info(info)
    assert ((inf["bp_iters"] >= 1) & (inf["bp_iters"] <= T)).all()
    L32 = llr.cpu().numpy().astype(np.float64)
    oc = ocode(oracle_mod, code)
    lam = oracle_mod.llr_from_priors(code.priors)
    rng = np.random.default_rng(T)
    picks = np.concatenate([rng.choice(B, 200, replace=False), [0, B - 1]])
    exempt = [int(b) for b in picks
              if _r24.check_shot(oracle_mod, oc, lam, S[b], T, L32[b], inf["status"][b] & 1,
                                 inf["bp_iters"][b]) == "exempt"]
    print(f"{len(picks) - len(exempt)} shots within 1e-4, near-zero exempt: {exempt}")


def test_bp_early_exit_matches_oracle(oracle_mod):
    code = bivariate_bicycle(p=0.05)
    e, S = sample(code, 2000, seed=7)
    _, dec = make(code, 50, 2000)
    llr, hard, info = dec.bp(syn_dev(S))
    torch.cuda.synchronize()
    inf = binding.parse_info(info)
    L32 = llr.cpu().numpy().astype(np.float64)
    oc = ocode(oracle_mod, code)
    lam = oracle_mod.llr_from_priors(code.priors)
    H32 = hard.cpu().numpy()
    exempt = [b for b in range(2000)
              if _r24.check_shot(oracle_mod, oc, lam, S[b], 50, L32[b], inf["status"][b] & 1,
                                 inf["bp_iters"][b], hard32=H32[b]) == "exempt"]
    print(f"{2000 - len(exempt)} shots equal, near-zero exempt: {exempt}")
    assert len(exempt) <= 0.05 * 2000


# ------------------------------------------------------------------------------ LSD

def _lsd_parity(oracle_mod, code, S, llr32, max_batch=None):
    B = S.shape[0]
    _, dec = make(code, 30, max_batch or B)
    corr, info = dec.lsd(syn_dev(S), torch.from_numpy(llr32).cuda())
    torch.cuda.synchronize()
    corr = corr.cpu().numpy()
    inf = binding.parse_info(info)
    oc = ocode(oracle_mod, code)
    for b in range(B):
        want, st, stats = oracle_mod.lsd(oc, S[b], llr32[b].astype(np.float64))
        assert (corr[b] == want).all(), f"shot {b}"
        assert (inf["status"][b] & 0x0C) == (st & 0x0C), f"shot {b}"
        if not (st & 4):
            assert inf["n_clusters"][b] == stats[0] and inf["rounds"][b] == stats[2], f"shot {b}"
            assert inf["max_cluster_cols"][b] == stats[1], f"shot {b}"
    return corr, inf


@pytest.mark.parametrize("which", ["c1", "c2", "hgp16"])
def test_lsd_bit_exact_on_bp_llrs(oracle_mod, which):
    code = {"c1": lambda: surface_hgp(5, 0.08), "c2": lambda: bivariate_bicycle(p=0.06),
            "hgp16": lambda: random_34_hgp(16, p=0.05)}[which]()
    print(f"case lsd_bp_llr {which}", flush=True)
    e, S = sample(code, 600, seed=31)
    _, dec = make(code, 30, 600)
    llr, hard, info = dec.bp(syn_dev(S))
    torch.cuda.synchronize()
    _lsd_parity(oracle_mod, code, S, llr.cpu().numpy())


@pytest.mark.parametrize("which", ["c1", "c2", "hgp16"])
def test_lsd_bit_exact_with_ties(oracle_mod, which):
    """Integer-valued LLRs: most growth decisions are index tie-breaks."""
    code = {"c1": lambda: surface_hgp(5, 0.1), "c2": lambda: bivariate_bicycle(p=0.08),
            "hgp16": lambda: random_34_hgp(16, p=0.06)}[which]()
    print(f"case lsd_ties {which}", flush=True)
    e, S = sample(code, 400, seed=47)
    rng = np.random.default_rng(3)
    llr = rng.integers(-2, 4, size=(400, code.n)).astype(np.float32)
    llr[:, ::7] = -0.0  # signed zeros order like +0
    _lsd_parity(oracle_mod, code, S, llr)


def test_lsd_unsat_and_nan(oracle_mod):
    code = bivariate_bicycle()
    rng = np.random.default_rng(9)
    S = (rng.random((200, 72)) < 0.15).astype(np.uint8)
    llr = rng.normal(size=(200, 144)).astype(np.float32)
    llr[5] = np.nan
    corr, inf = _lsd_parity(oracle_mod, code, S, llr)
    assert inf["status"][5] & binding.ST_BAD_LLR and not corr[5].any()
    assert (inf["status"] & binding.ST_UNSAT).any()


# ----------------------------------------------------------------------- end to end

@pytest.mark.parametrize("which,T,shots", [("c1", 30, 10000), ("c2", 50, 10000)])
def test_decode_ler_within_2sigma(oracle_mod, which, T, shots):
    code = surface_hgp(5, 0.05) if which == "c1" else bivariate_bicycle(p=0.05)
    print(f"case decode_ler {which}", flush=True)
    e, S = sample(code, shots, seed=2024)
    _, dec = make(code, T, shots)
    corr, info = dec.decode(syn_dev(S), want_info=True)
    torch.cuda.synchronize()
    corr = corr.cpu().numpy()
    inf = binding.parse_info(info)
    assert check_syndromes(code, corr, S).all()
    oc = ocode(oracle_mod, code)
    lam = oracle_mod.llr_from_priors(code.priors)
    ocorr, ost, oit, _ = oracle_mod.decode_batch(oc, lam, S, T)
    f_gpu = logical_failures(code, e, corr)
    f_ref = logical_failures(code, e, ocorr)
    p = max(f_ref.mean(), 1.0 / shots)
    sigma = np.sqrt(p * (1 - p) / shots)
    disc = int((f_gpu != f_ref).sum())
    print(f"LER gpu={f_gpu.mean():.5f} oracle={f_ref.mean():.5f} 2sigma={2*sigma:.5f} discordant={disc}")
    assert abs(f_gpu.mean() - f_ref.mean()) <= 2 * sigma
    # BP convergence agrees on every shot whose trajectory stays away from zero
    lam_f = oracle_mod.llr_from_priors(code.priors)
    for b in np.nonzero((inf["status"] & 1) != (ost & 1))[0]:
        mm = oracle_mod.bp_min_magnitude(oc, lam_f, S[b], T)
        assert mm < _r24.NEAR_ZERO * _r24.floor_of(lam_f), (b, mm)


def test_decode_full_batch_sampled(oracle_mod):
    """The benchmark's launch: 65,536 shots of [[144,12,12]] at p = 0.05, max 50 iterations.
    Every correction satisfies its syndrome; sampled LSD shots are bit-exact against the
    oracle run on the same float32 posteriors; the run is deterministic."""
    code = bivariate_bicycle(p=0.05)
    B = 65536
    print("case full_batch", flush=True)
    e, S = sample(code, B, seed=99)
    _, dec = make(code, 50, B)
    s = syn_dev(S)
    corr1, info = dec.decode(s, want_info=True)
    corr2 = dec.decode(s)
    llr, hard, binfo = dec.bp(s)
    torch.cuda.synchronize()
    c1, c2 = corr1.cpu().numpy(), corr2.cpu().numpy()
    assert (c1 == c2).all()
    inf = binding.parse_info(info)
    assert check_syndromes(code, c1, S).all()
    L = llr.cpu().numpy()
    oc = ocode(oracle_mod, code)
    rng = np.random.default_rng(0)
    lsd_shots = np.nonzero(inf["status"] & binding.ST_LSD_RUN)[0]
    assert len(lsd_shots) > 0.05 * B
    for b in rng.choice(lsd_shots, size=300, replace=False):
        want, st, _ = oracle_mod.lsd(oc, S[b], L[b].astype(np.float64))
        assert (c1[b] == want).all(), b
    conv = np.nonzero(inf["status"] & binding.ST_BP_CONVERGED)[0]
    h = hard.cpu().numpy()
    assert (c1[conv] == h[conv]).all()


def test_edge_cases(oracle_mod):
    code = bivariate_bicycle(p=0.05)
    _, dec = make(code, 50, 4096)
    # B = 0 is a no-op
    z = torch.empty((0, 72), dtype=torch.uint8, device="cuda")
    assert dec.decode(z).shape == (0, 144)
    # zero syndromes converge at the first iteration with e_hat = 0
    S0 = torch.zeros((333, 72), dtype=torch.uint8, device="cuda")
    corr, info = dec.decode(S0, want_info=True)
    inf = binding.parse_info(info)
    assert not corr.any().item() and (inf["bp_iters"] == 1).all() and (inf["status"] == 1).all()
    # B = 1, ragged batch, B = max_batch
    for B in (1, 37, 4095, 4096):
        e, S = sample(code, B, seed=B)
        corr = dec.decode(syn_dev(S)).cpu().numpy()
        assert check_syndromes(code, corr, S).all(), B
    # B beyond max_batch is refused synchronously
    e, S = sample(code, 4097, seed=1)
    with pytest.raises(binding.QlsdError) as ex:
        dec.decode(syn_dev(S))
    assert ex.value.status == -5
    # priors outside (0, 1) are refused
    bc = binding.Code.from_dense(code.H)
    bad = code.priors.copy()
    bad[3] = 0.0
    with pytest.raises(binding.QlsdError) as ex:
        binding.Decoder(bc, bad, 16)
    assert ex.value.status == -2



@pytest.mark.parametrize("ncl,B", [(24, 2048), (32, 1024)])
def test_hgp_serving_codes_against_oracle(oracle_mod, ncl, B):
    """The larger serving codes (HGP of random (3,4)-regular codes, n = 900 and 1600 qubits,
    p = 0.03, BP 30) at their serving batch sizes: BP posteriors with early exit against the
    oracle on a sample (near-zero exemptions reported), every LSD shot of the batch bit-exact
    against the oracle run on the same float32 posteriors, converged shots equal to BP's hard
    decision, and the decode's corrections equal to both."""
    code = random_34_hgp(ncl, p=0.03)
    print(f"case hgp{ncl} B={B}", flush=True)
    e, S = sample(code, B, seed=700 + ncl)
    _, dec = make(code, 30, B)
    s = syn_dev(S)
    corr, info = dec.decode(s, want_info=True)
    llr, hard, binfo = dec.bp(s)
    torch.cuda.synchronize()
    corr, L32, H32 = corr.cpu().numpy(), llr.cpu().numpy(), hard.cpu().numpy()
    inf, bi = binding.parse_info(info), binding.parse_info(binfo)
    assert check_syndromes(code, corr, S).all()
    oc = ocode(oracle_mod, code)
    lam = oracle_mod.llr_from_priors(code.priors)
    rng = np.random.default_rng(ncl)
    picks = rng.choice(B, 150, replace=False)
    exempt = [int(b) for b in picks
              if _r24.check_shot(oracle_mod, oc, lam, S[b], 30, L32[b].astype(np.float64), bi["status"][b] & 1,
                                 bi["bp_iters"][b], hard32=H32[b]) == "exempt"]
    conv = (bi["status"] & 1) == 1
    assert (corr[conv] == H32[conv]).all()
    lsd_shots = np.nonzero(~conv)[0]
    assert len(lsd_shots) > 0
    assert not (inf["status"] & binding.ST_OVERFLOW).any()
    for b in lsd_shots:
        want, st, stats = oracle_mod.lsd(oc, S[b], L32[b].astype(np.float64))
        assert (corr[b] == want).all(), b
        assert inf["n_clusters"][b] == stats[0] and inf["rounds"][b] == stats[2], b
    print(f"hgp{ncl}: {len(lsd_shots)} LSD shots bit-exact; BP sample exempt {exempt}")
