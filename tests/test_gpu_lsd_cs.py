"""LSD-mu with local OSD-CS (combination sweep) on the GPU against the oracle (Appendix D: growth
steps and local OSD order chosen separately, the growth steps as a fraction of the faults):
corrections, status, cluster counts and rounds bit-exact on identical float32 posteriors."""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import bivariate_bicycle, random_34_hgp, synthetic_dem, sample

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


@pytest.mark.parametrize("which,frac,w,T,shots", [("bb144", 0.02, 4, 30, 600), ("bb144", 0.08, 4, 30, 400),
                                                   ("hgp16", 0.01, 3, 30, 400), ("dem", 0.001, 4, 40, 3000)])
def test_lsd_cs_bit_exact(oracle_mod, which, frac, w, T, shots):
    code = {"bb144": lambda: bivariate_bicycle(p=0.06), "hgp16": lambda: random_34_hgp(16, p=0.05),
            "dem": synthetic_dem}[which]()
    mu = binding.mu_from_fraction(code.n, frac)
    print(f"case lsd_cs {which} mu={mu} w={w}", flush=True)
    e, S = sample(code, shots, seed=91)
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, shots, max_iter=T, lsd_order=mu, osd_method=binding.OSD_CS,
                          osd_order=w)
    s = torch.from_numpy(S).cuda()
    llr, hard, info = dec.bp(s)
    torch.cuda.synchronize()
    idx = np.nonzero((binding.parse_info(info)["status"] & 1) == 0)[0]
    assert len(idx) >= 20
    S2, L = np.ascontiguousarray(S[idx]), np.ascontiguousarray(llr.cpu().numpy()[idx])
    corr, linfo = dec.lsd(torch.from_numpy(S2).cuda(), torch.from_numpy(L).cuda())
    full = dec.decode(s).cpu().numpy()
    torch.cuda.synchronize()
    corr, li = corr.cpu().numpy(), binding.parse_info(linfo)
    np.testing.assert_array_equal(full[idx], corr)
    oc = oracle_mod.Code.from_dense(code.H)
    om = oracle_mod.omega_from_llr(oracle_mod.llr_from_priors(code.priors))
    changed = 0
    for k in range(len(idx)):
        want, st, stats = oracle_mod.lsd_cs(oc, S2[k], L[k].astype(np.float64), mu=mu, cs_order=w, omega=om)
        assert (corr[k] == want).all(), k
        assert (li["status"][k] & 0x1C) == (st & 0x1C), k
        assert (li["n_clusters"][k], li["rounds"][k]) == (stats[0], stats[2]), k
        w0, _, _ = oracle_mod.lsd(oc, S2[k], L[k].astype(np.float64))
        changed += int((w0 != want).any())
    assert (((corr.astype(np.int64) @ code.H.T.astype(np.int64)) & 1) == S2).all()
    print(f"{len(idx)} shots bit-exact; {changed} differ from LSD-0")
