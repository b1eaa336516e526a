"""Autotuner: qlsd_decoder_tune times candidate launch shapes on a sample batch and keeps the
fastest; decoding results must not depend on the shapes it picks."""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import bivariate_bicycle, random_34_hgp, sample

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


@pytest.mark.parametrize("which", ["bb144", "hgp16"])
def test_tuned_decoder_matches_untuned(which):
    code = bivariate_bicycle(p=0.05) if which == "bb144" else random_34_hgp(16, p=0.04)
    B = 16384
    bc = binding.Code.from_dense(code.H)
    e, S = sample(code, B, seed=81)
    s = torch.from_numpy(S).cuda()
    ref = binding.Decoder(bc, code.priors, B, max_iter=50)
    tuned = binding.Decoder(bc, code.priors, B, max_iter=50)
    report = tuned.tune(s, reps=2)
    print(report)
    assert "bp chosen" in report and "lsd chosen" in report
    c0, i0 = torch.empty((B, code.n), dtype=torch.uint8, device="cuda"), torch.empty((B, 12), dtype=torch.uint8, device="cuda")
    c1, i1 = torch.empty_like(c0), torch.empty_like(i0)
    ref.decode_into(s, c0, i0)
    tuned.decode_into(s, c1, i1)
    torch.cuda.synchronize()
    assert torch.equal(c0, c1) and torch.equal(i0, i1)
