"""qlsd_decode_static: the decode of qlsd_decode with its per-call scratch carved from the
library's static device array instead of the decoder's workspace.  Through the C ABI, against
qlsd_decode on the same decoder and shots, two calls in a row, the second with a smaller batch;
the one-kernel BP + LSD path, the separate-kernel path with LSD-mu and both overflow tiers (the
512-row LDS kernel and the 1024-row device-memory kernel, whose lists and bases also come from the
static array)."""
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


def _cases(which):
    if which == "bb144":
        code = bivariate_bicycle(p=0.05)
        return code, dict(max_iter=50), (65536, 1000), None
    if which == "dem":
        code = synthetic_dem()
        return code, dict(max_iter=100, lsd_order=10), (1024, 100), (0.12, 0.4)
    code = random_34_hgp(32, p=0.1)
    return code, dict(max_iter=30), (256, 37), None


@pytest.mark.parametrize("which", ["bb144", "dem", "hgp32"])
def test_static_scratch_decode_equals_decode(which):
    code, kw, sizes, heavy = _cases(which)
    print(f"case no_alloc {which} sizes={sizes}", flush=True)
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, sizes[0], **kw)
    rng = np.random.default_rng(17)
    for k, B in enumerate(sizes):
        e, S = sample(code, B, seed=6100 + k)
        if heavy is not None and k == 0:  # syndromes whose clusters reach the overflow kernels
            S = S.copy()
            for i, f in enumerate(heavy):
                S[3 + i] = (rng.random(code.m) < f).astype(np.uint8)
        s = torch.from_numpy(np.ascontiguousarray(S)).cuda()
        want, winfo = dec.decode(s, want_info=True)
        got, ginfo = dec.decode_static(s, want_info=True)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (which, B)
        assert torch.equal(ginfo, winfo), (which, B)
        inf = binding.parse_info(ginfo)
        assert not (inf["status"] & binding.ST_OVERFLOW).any()
        c = got.cpu().numpy()
        assert (((c.astype(np.int64) @ code.H.T.astype(np.int64)) & 1) == S).all()


def test_static_scratch_refuses_batches_beyond_it():
    code = synthetic_dem()
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, 4096, max_iter=10, lsd_order=10)
    e, S = sample(code, 4096, seed=3)
    with pytest.raises(binding.QlsdError) as ex:
        dec.decode_static(torch.from_numpy(S).cuda())
    assert ex.value.status == -5
    out = dec.decode_static(torch.from_numpy(np.ascontiguousarray(S[:64])).cuda())
    torch.cuda.synchronize()
    assert torch.equal(out, dec.decode(torch.from_numpy(np.ascontiguousarray(S[:64])).cuda()))
