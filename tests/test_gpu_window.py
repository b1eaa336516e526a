"""(3, 1) overlapping-window BP + LSD on the GPU (include/qlsd_window.h) over a 12-round memory
experiment on [[144,12,12]] (phenomenological noise, 936 detectors x 2736 faults): every
correction satisfies the full syndrome, the logical error rate matches the oracle's window decoder
on the same shots within 2 sigma, and a single window over all rounds is plain BP + LSD."""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import round_dem, bivariate_bicycle, surface_hgp, sample, logical_failures

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def test_window_decode_against_oracle_windows(oracle_mod):
    from oracle import window as ow
    p = 0.025
    dem = round_dem(bivariate_bicycle(p=p), 12, p, p)
    B = 4096
    print("case window_bb144_r12", flush=True)
    e, S = sample(dem, B, seed=12)
    bc = binding.Code.from_dense(dem.H)
    wd = binding.WindowDecoder(bc, dem.priors, dem.det_round, 3, 1, B, max_iter=30)
    assert wd.windows == 11
    corr = wd.decode(torch.from_numpy(S).cuda()).cpu().numpy()
    assert (((corr.astype(np.int64) @ dem.H.T.astype(np.int64)) & 1) == S).all()
    ref = ow.window_decode(dem.H, dem.priors, dem.det_round, S, w=3, c=1, max_iter=30)
    f_gpu, f_ref = logical_failures(dem, e, corr), logical_failures(dem, e, ref)
    q = max(f_ref.mean(), 1.0 / B)
    two_sigma = 2 * np.sqrt(q * (1 - q) / B)
    print(f"window (3,1) LER gpu {f_gpu.mean():.4f} oracle {f_ref.mean():.4f} (2 sigma {two_sigma:.4f}); "
          f"per cycle {ow.per_cycle(f_gpu.mean(), 12):.5f}; equal shots {(corr == ref).all(1).mean():.4f}")
    assert abs(f_gpu.mean() - f_ref.mean()) <= two_sigma


def test_single_window_is_plain_decode():
    """With w covering every round there is one window, whose sub-matrix is the whole DEM in its
    own column order: the result is the ordinary decoder's, byte for byte."""
    dem = round_dem(surface_hgp(5, p=0.03), 6, 0.03, 0.03)
    B = 2048
    e, S = sample(dem, B, seed=13)
    bc = binding.Code.from_dense(dem.H)
    wd = binding.WindowDecoder(bc, dem.priors, dem.det_round, 8, 1, B, max_iter=30)
    assert wd.windows == 1
    s = torch.from_numpy(S).cuda()
    got = wd.decode(s)
    want = binding.Decoder(bc, dem.priors, B, max_iter=30).decode(s)
    torch.cuda.synchronize()
    assert torch.equal(got, want)


def test_window_batches_are_independent():
    dem = round_dem(bivariate_bicycle(p=0.02), 12, 0.02, 0.02)
    e, S = sample(dem, 700, seed=14)
    bc = binding.Code.from_dense(dem.H)
    wd = binding.WindowDecoder(bc, dem.priors, dem.det_round, 3, 1, 700, max_iter=30)
    full = wd.decode(torch.from_numpy(S).cuda()).cpu().numpy()
    for lo, hi in ((0, 1), (1, 50), (50, 700)):
        part = wd.decode(torch.from_numpy(np.ascontiguousarray(S[lo:hi])).cuda()).cpu().numpy()
        np.testing.assert_array_equal(part, full[lo:hi])
