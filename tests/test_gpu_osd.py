"""GPU global OSD-0 (the comparator of Sec. 2.2, inversion decoding) through the C ABI against
the oracle's OSD-0, which reduces all n columns in (llr_j, j) order and solves on the greedy pivot
set: bit-exact on BP posteriors and on tie-heavy integer LLRs, UNSAT exactly when s is not in the
image of H, and BP + OSD-0 decoding end to end."""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import (bivariate_bicycle, surface_hgp, random_34_hgp, synthetic_dem,
                                            sample, logical_failures, gf2_rank)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


CODES = {"c1": lambda: surface_hgp(5, 0.08), "c2": lambda: bivariate_bicycle(p=0.06),
         "hgp16": lambda: random_34_hgp(16, p=0.05), "hgp24": lambda: random_34_hgp(24, p=0.04)}


def _osd_parity(oracle_mod, code, S, L):
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, S.shape[0], max_iter=30)
    corr, info = dec.osd0(torch.from_numpy(S).cuda(), torch.from_numpy(L).cuda())
    torch.cuda.synchronize()
    corr, inf = corr.cpu().numpy(), binding.parse_info(info)
    oc = oracle_mod.Code.from_dense(code.H)
    for b in range(S.shape[0]):
        want, st = oracle_mod.osd0(oc, S[b], L[b].astype(np.float64))
        assert (corr[b] == want).all(), b
        assert bool(inf["status"][b] & binding.ST_UNSAT) == bool(st & 4), b
    return corr, inf


@pytest.mark.parametrize("which", ["c1", "c2", "hgp16", "hgp24"])
def test_osd0_bit_exact_on_bp_llrs(oracle_mod, which):
    code = CODES[which]()
    print(f"case osd0_bp_llr {which}", flush=True)
    e, S = sample(code, 800, seed=61)
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, 800, max_iter=30)
    llr, hard, info = dec.bp(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    inf = binding.parse_info(info)
    idx = np.nonzero((inf["status"] & 1) == 0)[0]
    assert len(idx) > 10
    S2 = np.ascontiguousarray(S[idx])
    corr, oinf = _osd_parity(oracle_mod, code, S2, np.ascontiguousarray(llr.cpu().numpy()[idx]))
    assert (((corr.astype(np.int64) @ code.H.T.astype(np.int64)) & 1) == S2).all()
    print(f"{which}: {len(idx)} shots; columns reduced per shot median {np.median(oinf['max_cluster_cols'])}")


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_osd0_bit_exact_with_ties_and_unsat(oracle_mod, which):
    """Integer LLRs (most of the order decided by the index) and, on the rank-deficient BB code,
    random syndromes of which some lie outside the image of H."""
    code = CODES[which]()
    rng = np.random.default_rng(8)
    e, S = sample(code, 300, seed=62)
    if which == "c2":
        S = np.concatenate([S, (rng.random((100, code.m)) < 0.2).astype(np.uint8)])
    L = rng.integers(-2, 4, size=(S.shape[0], code.n)).astype(np.float32)
    L[:, ::5] = -0.0
    corr, inf = _osd_parity(oracle_mod, code, np.ascontiguousarray(S), L)
    if which == "c2":
        unsat = inf["status"][300:] & binding.ST_UNSAT
        in_image = [gf2_rank(np.concatenate([code.H, s[:, None]], 1)) == gf2_rank(code.H) for s in S[300:]]
        assert (unsat.astype(bool) == ~np.array(in_image)).all()
        assert unsat.any() and not unsat.all()


@pytest.mark.parametrize("which,T", [("c1", 30), ("c2", 50)])
def test_bp_osd0_decode_against_oracle(oracle_mod, which, T):
    """qlsd_decode with QLSD_FLAG_OSD0_POST: converged shots equal BP's hard decision, the others
    equal the oracle's OSD-0 on the same float32 posteriors, and the logical error rate is within
    2 sigma of the oracle's BP + OSD-0 on the same shots."""
    code = surface_hgp(5, 0.05) if which == "c1" else bivariate_bicycle(p=0.05)
    B = 10000
    e, S = sample(code, B, seed=2024)
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, B, max_iter=T, flags=binding.FLAG_OSD0_POST)
    s = torch.from_numpy(S).cuda()
    corr, info = dec.decode(s, want_info=True)
    llr, hard, binfo = dec.bp(s)
    torch.cuda.synchronize()
    corr, L, H = corr.cpu().numpy(), llr.cpu().numpy(), hard.cpu().numpy()
    bi = binding.parse_info(binfo)
    conv = (bi["status"] & 1) == 1
    np.testing.assert_array_equal(corr[conv], H[conv])
    oc = oracle_mod.Code.from_dense(code.H)
    for b in np.nonzero(~conv)[0]:
        want, _ = oracle_mod.osd0(oc, S[b], L[b].astype(np.float64))
        assert (corr[b] == want).all(), b
    lam = oracle_mod.llr_from_priors(code.priors)
    ocorr, ost, _, ollr = oracle_mod.decode_batch(oc, lam, S, T, want_llr=True)
    for b in np.nonzero((ost & 1) == 0)[0]:
        ocorr[b], _ = oracle_mod.osd0(oc, S[b], ollr[b])
    f_gpu, f_ref = logical_failures(code, e, corr), logical_failures(code, e, ocorr)
    p = max(f_ref.mean(), 1.0 / B)
    two_sigma = 2 * np.sqrt(p * (1 - p) / B)
    print(f"{which}: BP+OSD-0 LER gpu {f_gpu.mean():.5f} oracle {f_ref.mean():.5f} (2 sigma {two_sigma:.5f})")
    assert abs(f_gpu.mean() - f_ref.mean()) <= two_sigma


def test_osd0_refuses_graphs_beyond_its_sort():
    code = synthetic_dem()
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, 4, max_iter=10)
    s = torch.zeros((4, code.m), dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.QlsdError) as ex:
        dec.osd0(s, torch.zeros((4, code.n), dtype=torch.float32, device="cuda"))
    assert ex.value.status == -6
    with pytest.raises(binding.QlsdError):
        binding.Decoder(bc, code.priors, 4, max_iter=10, flags=binding.FLAG_OSD0_POST)


# ------------------------------------------------------------------ global OSD-CS of order w

def _osd_cs_parity(oracle_mod, code, S, L, order):
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, S.shape[0], max_iter=30)
    corr, info = dec.osd_cs(torch.from_numpy(S).cuda(), torch.from_numpy(L).cuda(), order)
    torch.cuda.synchronize()
    corr, inf = corr.cpu().numpy(), binding.parse_info(info)
    oc = oracle_mod.Code.from_dense(code.H)
    om = oracle_mod.omega_from_llr(oracle_mod.llr_from_priors(code.priors))
    changed = 0
    for b in range(S.shape[0]):
        want, st = oracle_mod.osd_cs(oc, S[b], L[b].astype(np.float64), order, om)
        assert (corr[b] == want).all(), (order, b)
        assert bool(inf["status"][b] & binding.ST_UNSAT) == bool(st & oracle_mod.ST_UNSAT), b
        if not st:
            x0, _ = oracle_mod.osd0(oc, S[b], L[b].astype(np.float64))
            changed += int((x0 != want).any())
    return corr, inf, changed


@pytest.mark.parametrize("which", ["c1", "c2", "hgp16"])
def test_osd_cs_bit_exact_on_bp_llrs(oracle_mod, which):
    """qlsd_osd_cs against the oracle's global OSD-CS on BP's float32 posteriors of the shots BP
    leaves unsolved, orders 1, 4, 7 and 12 (the sweep changes OSD-0's answer on many shots)."""
    code = CODES[which]()
    print(f"case osd_cs_bp_llr {which}", flush=True)
    e, S = sample(code, 800, seed=63)
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, 800, max_iter=30)
    llr, hard, info = dec.bp(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    inf = binding.parse_info(info)
    idx = np.nonzero((inf["status"] & 1) == 0)[0][:200]
    assert len(idx) > 10
    S2 = np.ascontiguousarray(S[idx])
    L2 = np.ascontiguousarray(llr.cpu().numpy()[idx])
    for order in (1, 4, 7, 12):
        corr, oinf, changed = _osd_cs_parity(oracle_mod, code, S2, L2, order)
        assert (((corr.astype(np.int64) @ code.H.T.astype(np.int64)) & 1) == S2).all()
        assert (oinf["max_cluster_cols"] == code.n).all()
        print(f"{which} order {order}: {len(idx)} shots, {changed} differ from OSD-0")
        if order >= 4:
            assert changed > 0


def test_osd_cs_ties_zero_and_unsat(oracle_mod):
    """Integer LLRs (order mostly decided by the index), zero syndromes and, on the rank-deficient
    BB code, syndromes outside the image of H."""
    code = CODES["c2"]()
    rng = np.random.default_rng(9)
    e, S = sample(code, 150, seed=64)
    S = np.concatenate([S, np.zeros((10, code.m), np.uint8), (rng.random((60, code.m)) < 0.2).astype(np.uint8)])
    L = rng.integers(-2, 4, size=(S.shape[0], code.n)).astype(np.float32)
    L[:, ::5] = -0.0
    corr, inf, _ = _osd_cs_parity(oracle_mod, code, np.ascontiguousarray(S), L, 7)
    assert not corr[150:160].any()
    unsat = inf["status"][160:] & binding.ST_UNSAT
    assert unsat.any() and not unsat.all()


def test_bp_osd_cs_decode_against_oracle(oracle_mod):
    """qlsd_decode with QLSD_FLAG_OSD0_POST and osd_method 1: BP, then global OSD-CS-7 on the shots
    BP leaves unsolved -- converged shots equal BP's hard decision, the others the oracle's OSD-CS
    on the same float32 posteriors; fewer logical failures than BP + OSD-0 on the same shots."""
    code = bivariate_bicycle(p=0.05)
    B = 4000
    e, S = sample(code, B, seed=2025)
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, B, max_iter=50, flags=binding.FLAG_OSD0_POST,
                          osd_method=binding.OSD_CS, osd_order=7)
    dec0 = binding.Decoder(bc, code.priors, B, max_iter=50, flags=binding.FLAG_OSD0_POST)
    s = torch.from_numpy(S).cuda()
    corr, info = dec.decode(s, want_info=True)
    corr0 = dec0.decode(s)
    llr, hard, binfo = dec.bp(s)
    torch.cuda.synchronize()
    corr, corr0, L, H = corr.cpu().numpy(), corr0.cpu().numpy(), llr.cpu().numpy(), hard.cpu().numpy()
    conv = (binding.parse_info(binfo)["status"] & 1) == 1
    np.testing.assert_array_equal(corr[conv], H[conv])
    oc = oracle_mod.Code.from_dense(code.H)
    om = oracle_mod.omega_from_llr(oracle_mod.llr_from_priors(code.priors))
    for b in np.nonzero(~conv)[0]:
        want, _ = oracle_mod.osd_cs(oc, S[b], L[b].astype(np.float64), 7, om)
        assert (corr[b] == want).all(), b
    f_cs, f_0 = logical_failures(code, e, corr).sum(), logical_failures(code, e, corr0).sum()
    print(f"BP50 + OSD-CS-7 failures {f_cs}, BP50 + OSD-0 {f_0} of {B}")
    assert f_cs < f_0


def test_osd_cs_refusals():
    code = synthetic_dem()
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, 4, max_iter=10)
    s = torch.zeros((4, code.m), dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.QlsdError) as ex:
        dec.osd_cs(s, torch.zeros((4, code.n), dtype=torch.float32, device="cuda"), 7)
    assert ex.value.status == -6
    with pytest.raises(binding.QlsdError):
        binding.Decoder(bc, code.priors, 4, max_iter=10, flags=binding.FLAG_OSD0_POST, osd_method=binding.OSD_CS,
                        osd_order=7)
    c2 = bivariate_bicycle()
    d2 = binding.Decoder(binding.Code.from_dense(c2.H), c2.priors, 4, max_iter=10)
    s2 = torch.zeros((4, c2.m), dtype=torch.uint8, device="cuda")
    for bad in (0, 13):
        with pytest.raises(binding.QlsdError) as ex:
            d2.osd_cs(s2, torch.zeros((4, c2.n), dtype=torch.float32, device="cuda"), bad)
        assert ex.value.status == -1  # QLSD_E_INVALID
