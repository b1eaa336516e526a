"""BP and LSD in one kernel (qlsd_decode's default for slot BP with LSD of up to 128 local rows)
against the two-kernel path (QLSD_FLAG_SEPARATE_LSD): identical corrections and info records on
the same seeded shots.  Both paths compute every shot's LSD from the same syndrome and the same
BP posterior, so any difference is a lost, duplicated or stale hand-over between workgroups.
Oracle parity of qlsd_decode itself is in test_gpu_parity.py (which now runs the one-kernel path).
"""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import bivariate_bicycle, surface_hgp, sample

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()
    yield
    torch.cuda.synchronize()


def _pair(code, T, max_batch, flags=0):
    bc = binding.Code.from_dense(code.H)
    one = binding.Decoder(bc, code.priors, max_batch, max_iter=T, flags=flags)
    two = binding.Decoder(bc, code.priors, max_batch, max_iter=T, flags=flags | binding.FLAG_SEPARATE_LSD)
    return bc, one, two


def _run(dec, s, n):
    B = s.shape[0]
    corr = torch.full((B, n), 7, dtype=torch.uint8, device="cuda")
    info = torch.full((B, 12), 0xAB, dtype=torch.uint8, device="cuda")
    dec.decode_into(s, corr, info)
    dec.sync()
    return corr.cpu().numpy(), info.cpu().numpy()


def _same(code, one, two, S):
    s = torch.from_numpy(np.ascontiguousarray(S)).cuda()
    c1, i1 = _run(one, s, code.n)
    c2, i2 = _run(two, s, code.n)
    assert np.array_equal(c1, c2), f"{int((c1 != c2).any(axis=1).sum())} shots differ"
    assert np.array_equal(i1, i2), f"{int((i1 != i2).any(axis=1).sum())} info records differ"
    # every correction reproduces its syndrome unless the shot was flagged
    st = binding.parse_info(torch.from_numpy(i1))["status"]
    good = ((c1.astype(np.int64) @ code.H.T.astype(np.int64)) % 2 == S).all(axis=1)
    assert (good | ((st & (binding.ST_UNSAT | binding.ST_OVERFLOW)) != 0)).all()
    return st


def test_full_batch_bb144():
    """[[144,12,12]] at p = 0.05, 65,536 shots, BP 50: about one shot in seven goes to LSD."""
    code = bivariate_bicycle(p=0.05)
    _, one, two = _pair(code, 50, 65536)
    _, S = sample(code, 65536, seed=4242)
    st = _same(code, one, two, S)
    assert ((st & binding.ST_LSD_RUN) != 0).sum() > 1000


def test_repeated_calls_and_ragged_sizes():
    """Consecutive calls on one decoder (the published list is reset per call) with batch sizes
    from one shot to a ragged full batch."""
    code = bivariate_bicycle(p=0.06)
    _, one, two = _pair(code, 30, 20000)
    for k, B in enumerate((20000, 1, 65, 777, 20000, 19999)):
        _, S = sample(code, B, seed=900 + k)
        _same(code, one, two, S)


def test_every_shot_through_lsd():
    """No early exit and 3 BP iterations: nearly every shot is published to LSD."""
    code = bivariate_bicycle(p=0.05)
    _, one, two = _pair(code, 3, 65536, flags=binding.FLAG_NO_EARLY_EXIT)
    _, S = sample(code, 65536, seed=77)
    st = _same(code, one, two, S)
    assert ((st & binding.ST_LSD_RUN) != 0).mean() > 0.5


def test_irregular_small_code():
    """Surface code as a hypergraph product (irregular row and column weights, one-word LSD rows)."""
    code = surface_hgp(d=7, p=0.08)
    _, one, two = _pair(code, 20, 5000)
    _, S = sample(code, 5000, seed=11)
    _same(code, one, two, S)


def test_two_decoders_concurrently():
    """Two one-kernel decodes in flight at once on two streams: together their grids exceed
    what the GPU holds resident, so some BP workgroups start only after others have left --
    the case the bounded waits exist for.  Each result equals the same decoder's result alone."""
    code = bivariate_bicycle(p=0.05)
    bc = binding.Code.from_dense(code.H)
    decs = [binding.Decoder(bc, code.priors, 65536, max_iter=50) for _ in range(2)]
    batches = [sample(code, 65536, seed=500 + k)[1] for k in range(2)]
    alone = []
    for d, S in zip(decs, batches):
        s = torch.from_numpy(np.ascontiguousarray(S)).cuda()
        alone.append(_run(d, s, code.n))
    streams = [torch.cuda.Stream() for _ in range(2)]
    syn = [torch.from_numpy(np.ascontiguousarray(S)).cuda() for S in batches]
    outs = [(torch.full((65536, code.n), 7, dtype=torch.uint8, device="cuda"),
             torch.full((65536, 12), 0xAB, dtype=torch.uint8, device="cuda")) for _ in range(2)]
    torch.cuda.synchronize()
    for rep in range(3):
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                decs[k].decode_into(syn[k], outs[k][0], outs[k][1])
        torch.cuda.synchronize()
        for k in range(2):
            decs[k].sync()
            assert np.array_equal(outs[k][0].cpu().numpy(), alone[k][0]), (rep, k)
            assert np.array_equal(outs[k][1].cpu().numpy(), alone[k][1]), (rep, k)
