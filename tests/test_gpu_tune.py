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


def _with_heavy_shots(code, B, heavy, p_heavy, seed):
    """B sampled shots plus `heavy` shots of dense errors (density p_heavy), whose clusters
    outgrow the small LSD capacity tiers; every syndrome is H e, so in the image of H."""
    e, S = sample(code, B, seed=seed)
    rng = np.random.default_rng(seed + 1)
    E = (rng.random((heavy, code.n)) < p_heavy).astype(np.int64)
    Sh = ((E @ code.H.T.astype(np.int64)) & 1).astype(np.uint8)
    return np.ascontiguousarray(np.concatenate([S, Sh]))


@pytest.mark.parametrize("which", ["bb144", "hgp16", "dem"])
@pytest.mark.parametrize("separate", [False, True])
def test_capacity_tiers_decode_alike(which, separate):
    """Every LSD capacity tier (64, 128, 256 local rows per wavefront) returns the default tier's
    corrections and shot info: shots beyond a small tier go whole to the overflow kernels, on the
    fused BP+LSD path as on the separate one."""
    from paper_2406_18655_amd.workloads import synthetic_dem
    code = {"bb144": lambda: bivariate_bicycle(p=0.05), "hgp16": lambda: random_34_hgp(16, p=0.04),
            "dem": synthetic_dem}[which]()
    S = _with_heavy_shots(code, 4000, 96, 0.01 if which == "dem" else 0.12, seed=85)
    B = S.shape[0]
    s = torch.from_numpy(S).cuda()
    bc = binding.Code.from_dense(code.H)
    flags = binding.FLAG_SEPARATE_LSD if separate else 0
    T = 30
    ref = binding.Decoder(bc, code.priors, B, max_iter=T, flags=flags)
    c0 = torch.empty((B, code.n), dtype=torch.uint8, device="cuda")
    i0 = torch.empty((B, 12), dtype=torch.uint8, device="cuda")
    ref.decode_into(s, c0, i0)
    torch.cuda.synchronize()
    inf = binding.parse_info(i0.cpu().numpy())
    big = int((inf["max_cluster_cols"] > 64).sum())
    print(f"case {which} separate={separate}: {B} shots, {big} with a cluster beyond 64 columns", flush=True)
    assert not (inf["status"] & binding.ST_OVERFLOW).any()
    for rows in (64, 128, 256):
        d = binding.Decoder(bc, code.priors, B, max_iter=T, flags=flags)
        d.set_lsd_capacity(rows)
        c1, i1 = torch.empty_like(c0), torch.empty_like(i0)
        for _ in range(2):  # a second call reuses the overflow list and the wide workspace
            c1.fill_(7)
            d.decode_into(s, c1, i1)
            torch.cuda.synchronize()
            assert torch.equal(c0, c1), rows
            assert torch.equal(i0, i1), rows
        del d
    with pytest.raises(binding.QlsdError):
        ref.set_lsd_capacity(96)
    mu = binding.Decoder(bc, code.priors, 64, max_iter=T, lsd_order=4)
    with pytest.raises(binding.QlsdError):
        mu.set_lsd_capacity(128)
    mu.set_lsd_capacity(256)


@pytest.mark.parametrize("which,mu", [("dem", 0), ("dem", 10), ("hgp24", 0), ("hgp16", 4)])
def test_cluster_batched_schedule_decodes_alike(which, mu):
    """The cluster-batched LSD schedule (one column per cluster per batch, reduced together)
    returns the per-column schedule's corrections and shot info, with and without LSD-mu."""
    from paper_2406_18655_amd.workloads import synthetic_dem
    code = {"dem": synthetic_dem, "hgp24": lambda: random_34_hgp(24, p=0.04),
            "hgp16": lambda: random_34_hgp(16, p=0.05)}[which]()
    S = _with_heavy_shots(code, 3000, 64, 0.004 if which == "dem" else 0.06, seed=87)
    B = S.shape[0]
    s = torch.from_numpy(S).cuda()
    bc = binding.Code.from_dense(code.H)
    T = 30
    out = []
    for sched in (binding.LSD_PER_COLUMN, binding.LSD_CLUSTER_BATCHED):
        d = binding.Decoder(bc, code.priors, B, max_iter=T, lsd_order=mu)
        d.set_lsd_schedule(sched)
        c = torch.empty((B, code.n), dtype=torch.uint8, device="cuda")
        i = torch.empty((B, 12), dtype=torch.uint8, device="cuda")
        d.decode_into(s, c, i)
        torch.cuda.synchronize()
        out.append((c, i))
    inf = binding.parse_info(out[0][1].cpu().numpy())
    many = int((inf["n_clusters"] >= 4).sum())
    print(f"case {which} mu={mu}: {B} shots, {many} ending with 4 or more clusters", flush=True)
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


def test_cluster_batched_schedule_bit_exact_against_oracle(oracle_mod):
    """LSD alone on identical float32 posteriors: the cluster-batched schedule against the oracle,
    shot by shot, on DEM shots BP leaves unsolved plus denser syndromes with many clusters."""
    from paper_2406_18655_amd.workloads import synthetic_dem
    code = synthetic_dem()
    S = _with_heavy_shots(code, 1500, 40, 0.003, seed=89)
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, S.shape[0], max_iter=20)
    llr, hard, info = dec.bp(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    keep = np.nonzero((binding.parse_info(info)["status"] & 1) == 0)[0][:150]
    S, L = np.ascontiguousarray(S[keep]), np.ascontiguousarray(llr.cpu().numpy()[keep])
    d = binding.Decoder(bc, code.priors, S.shape[0], max_iter=20)
    d.set_lsd_schedule(binding.LSD_CLUSTER_BATCHED)
    corr, info = d.lsd(torch.from_numpy(S).cuda(), torch.from_numpy(L).cuda())
    torch.cuda.synchronize()
    corr, inf = corr.cpu().numpy(), binding.parse_info(info)
    oc = oracle_mod.Code.from_dense(code.H)
    for b in range(S.shape[0]):
        want, st, stats = oracle_mod.lsd(oc, S[b], L[b].astype(np.float64))
        assert (corr[b] == want).all(), b
        assert (inf["n_clusters"][b], inf["rounds"][b], inf["max_cluster_cols"][b]) == (stats[0], stats[2], stats[1]), b
    print(f"{S.shape[0]} shots bit-exact, max clusters {int(inf['n_clusters'].max())}")


def test_cluster_batched_schedule_needs_the_256_row_kernel():
    code = bivariate_bicycle(p=0.05)
    d = binding.Decoder(binding.Code.from_dense(code.H), code.priors, 64, max_iter=10)
    with pytest.raises(binding.QlsdError):
        d.set_lsd_schedule(binding.LSD_CLUSTER_BATCHED)
    with pytest.raises(binding.QlsdError):
        d.set_lsd_schedule(7)
    d.set_lsd_schedule(binding.LSD_PER_COLUMN)


def test_stage_timing_switch():
    """qlsd_decoder_set_stage_timing: with the events off a decode leaves the last timed call's
    stage times in place and its outputs unchanged; on again, the next call is timed; a decoder
    created without QLSD_FLAG_STAGE_TIMING refuses the switch."""
    code = bivariate_bicycle(p=0.05)
    B = 16384
    bc = binding.Code.from_dense(code.H)
    _, S0 = sample(code, B, seed=91)
    _, S1 = sample(code, B, seed=92)
    s0, s1 = torch.from_numpy(S0).cuda(), torch.from_numpy(S1).cuda()
    d = binding.Decoder(bc, code.priors, B, max_iter=50, flags=binding.FLAG_STAGE_TIMING)
    plain = binding.Decoder(bc, code.priors, B, max_iter=50)
    c_on = torch.empty((B, code.n), dtype=torch.uint8, device="cuda")
    c_off, c_ref = torch.empty_like(c_on), torch.empty_like(c_on)
    d.decode_into(s0, c_on, None)
    first = d.stage_ms()
    assert first[0] > 0.0
    d.set_stage_timing(False)
    d.decode_into(s1, c_off, None)
    plain.decode_into(s1, c_ref, None)
    torch.cuda.synchronize()
    assert d.stage_ms() == first, "a call with the events off must not re-record them"
    assert torch.equal(c_off, c_ref)
    d.set_stage_timing(True)
    d.decode_into(s1, c_on, None)
    second = d.stage_ms()
    assert second[0] > 0.0 and torch.equal(c_on, c_ref)
    with pytest.raises(binding.QlsdError):
        plain.set_stage_timing(True)
