"""Bivariate bicycle codes other than [[144,12,12]] through the regular-code BP instantiation (every
row of weight 6, every column of weight 3: packed per-fault records, one active slot per thread):
[[72,12,6]] (36 checks: one 64-row LSD slice, BP and LSD in one kernel) and [[288,12,18]] (144
checks: four slices, BP and LSD as separate kernels).  BP posteriors against the float64 oracle;
a full decode whose converged shots equal BP's hard decision and whose LSD shots are bit-exact
against the oracle's LSD on the same float32 posteriors."""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import bivariate_bicycle, sample

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CODES = {
    # A = x^3 + y + y^2, B = y^3 + x + x^2 on l = m = 6
    "bb72": lambda p: bivariate_bicycle(6, 6, p=p),
    # A = x^3 + y^2 + y^7, B = y^3 + x + x^2 on l = m = 12
    "bb288": lambda p: bivariate_bicycle(12, 12, a_terms=(("x", 3), ("y", 2), ("y", 7)),
                                         b_terms=(("y", 3), ("x", 1), ("x", 2)), p=p),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()
    yield
    torch.cuda.synchronize()


def _dec(code, T, B, flags=0):
    bc = binding.Code.from_dense(code.H)
    return binding.Decoder(bc, code.priors, B, max_iter=T, flags=flags)


@pytest.mark.parametrize("which", ["bb72", "bb288"])
def test_regular_code_shape(which):
    code = CODES[which](0.05)
    assert (code.H.sum(axis=1) == 6).all() and (code.H.sum(axis=0) == 3).all()


@pytest.mark.parametrize("which", ["bb72", "bb288"])
def test_bp_posteriors_fixed_iterations(oracle_mod, which):
    code = CODES[which](0.05)
    T, shots = 20, 256
    print(f"case bb_family_bp {which}", flush=True)
    e, S = sample(code, shots, seed=210)
    dec = _dec(code, T, shots, flags=binding.FLAG_NO_EARLY_EXIT)
    llr, hard, info = dec.bp(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    L32 = llr.cpu().numpy().astype(np.float64)
    inf = binding.parse_info(info)
    assert (inf["bp_iters"] == T).all()
    oc = oracle_mod.Code.from_dense(code.H)
    lam = oracle_mod.llr_from_priors(code.priors)
    floor = np.abs(lam).min()
    for b in range(shots):
        conv, it, L64, h64 = oracle_mod.bp(oc, lam, S[b], T, early_exit=False)
        err = np.abs(L32[b] - L64) / np.maximum(np.abs(L64), floor)
        assert err.max() <= 1e-4, (b, float(err.max()))
        assert bool(inf["status"][b] & 1) == conv


@pytest.mark.parametrize("which,B", [("bb72", 20000), ("bb288", 8192)])
def test_decode_matches_bp_and_oracle_lsd(oracle_mod, which, B):
    code = CODES[which](0.07)
    T = 30
    print(f"case bb_family_decode {which} B={B}", flush=True)
    e, S = sample(code, B, seed=211)
    dec = _dec(code, T, B)
    s = torch.from_numpy(S).cuda()
    corr, info = dec.decode(s, want_info=True)
    llr, hard, _ = dec.bp(s)
    torch.cuda.synchronize()
    c = corr.cpu().numpy()
    inf = binding.parse_info(info)
    bad = (inf["status"] & (binding.ST_UNSAT | binding.ST_OVERFLOW)) != 0
    good = (((c.astype(np.int64) @ code.H.T.astype(np.int64)) % 2) == S).all(axis=1)
    assert (good | bad).all()
    conv = np.nonzero(inf["status"] & binding.ST_BP_CONVERGED)[0]
    assert (c[conv] == hard.cpu().numpy()[conv]).all()
    lsd_shots = np.nonzero(inf["status"] & binding.ST_LSD_RUN)[0]
    assert len(lsd_shots) >= 50, len(lsd_shots)
    L = llr.cpu().numpy()
    oc = oracle_mod.Code.from_dense(code.H)
    rng = np.random.default_rng(5)
    for b in rng.choice(lsd_shots, size=min(120, len(lsd_shots)), replace=False):
        want, st, stats = oracle_mod.lsd(oc, S[b], L[b].astype(np.float64))
        assert (c[b] == want).all(), b
        assert inf["rounds"][b] == stats[2] and inf["n_clusters"][b] == stats[0], b
