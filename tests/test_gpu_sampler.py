"""The library's Philox4x64-10 sampler (include/qlsd_sample.h) against the host sampler
(workloads.sample: numpy's Philox with key [seed, block]) bit for bit, for arbitrary shot ranges,
ragged rows (n not a multiple of 4) and the 8,800-fault detector error model; syndromes and
logical-failure flags against their host definitions."""
import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import (bivariate_bicycle, surface_hgp, synthetic_dem, sample, syndromes,
                                            logical_failures)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


@pytest.mark.parametrize("which", ["surface", "bb144", "dem"])
def test_device_shots_equal_host_shots(which):
    code = {"surface": lambda: surface_hgp(5, 0.1), "bb144": lambda: bivariate_bicycle(p=0.05),
            "dem": synthetic_dem}[which]()
    print(f"case sampler {which}", flush=True)
    ds = binding.DeviceSampler(code)
    ranges = [(7, 0, 5000), (7, 4090, 20), (2 ** 63 + 12345, 10001, 3), (99, 123, 1)]
    if which == "dem":
        ranges = [(7, 0, 600), (7, 4000, 200), (5_000_001, 70000, 5)]
    for seed, start, B in ranges:
        e_h, s_h = sample(code, B, seed=seed, start=start)
        e_d, s_d = ds.sample(B, seed, start=start)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(e_d.cpu().numpy(), e_h, err_msg=f"{which} {seed} {start} {B}")
        np.testing.assert_array_equal(s_d.cpu().numpy(), s_h)
    e0, s0 = ds.sample(0, 1)
    assert e0.shape == (0, code.n)


@pytest.mark.parametrize("which", ["bb144", "dem"])
def test_failures_and_syndromes_match_host(which):
    code = bivariate_bicycle(p=0.05) if which == "bb144" else synthetic_dem()
    ds = binding.DeviceSampler(code)
    e, s = ds.sample(3000, 11)
    rng = np.random.default_rng(0)
    c = e.cpu().numpy().copy()
    flip = rng.random(c.shape) < 0.01  # some residuals logical, some not, some zero
    flip[: len(c) // 3] = False
    c ^= flip.astype(np.uint8)
    cd = torch.from_numpy(c).cuda()
    f = ds.failures(e, cd).cpu().numpy()
    np.testing.assert_array_equal(f, logical_failures(code, e.cpu().numpy(), c))
    assert f.any() and not f.all()
    np.testing.assert_array_equal(ds.syndromes(cd).cpu().numpy(), syndromes(code, c))
