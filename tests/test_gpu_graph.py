"""The decode calls launch kernels only (no allocation, no memset, no host synchronisation), so
a whole decode -- BP, compaction, optional refinement, LSD -- can be captured in a HIP graph and
replayed.  Every replay is checked against an eager decode of the same syndromes, with eager
work and synchronisations between the replays."""
import os

import numpy as np
import pytest

from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import bivariate_bicycle, random_34_hgp, sample, synthetic_dem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


@pytest.mark.parametrize("learned", [False, True])
def test_decode_graph_replays_match_eager(learned):
    code = bivariate_bicycle(p=0.05)
    B = 8192
    bc = binding.Code.from_dense(code.H)
    T = 10 if learned else 50
    graphed = binding.Decoder(bc, code.priors, B, max_iter=T)
    eager = binding.Decoder(bc, code.priors, B, max_iter=T)
    if learned:
        w = os.path.join(os.path.dirname(binding.__file__), "weights", "bb144_p0.05_T10.npy")
        net = binding.Net(bc, code.priors, np.load(w))
        binding.attach_net(graphed, net)
        binding.attach_net(eager, net)
    s_static = torch.zeros((B, code.m), dtype=torch.uint8, device="cuda")
    c_static = torch.zeros((B, code.n), dtype=torch.uint8, device="cuda")
    i_static = torch.zeros((B, 12), dtype=torch.uint8, device="cuda")
    _, S0 = sample(code, B, seed=60)
    s_static.copy_(torch.from_numpy(S0).cuda())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up launch outside the capture
        graphed.decode_into(s_static, c_static, i_static)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graphed.decode_into(s_static, c_static, i_static)
    torch.cuda.synchronize()
    for rep in range(4):
        _, S = sample(code, B, seed=61 + rep)
        s = torch.from_numpy(S).cuda()
        s_static.copy_(s)
        g.replay()
        torch.cuda.synchronize()
        got_c, got_i = c_static.clone(), i_static.clone()
        want_c = torch.empty_like(c_static)
        want_i = torch.empty_like(i_static)
        eager.decode_into(s, want_c, want_i)
        torch.cuda.synchronize()
        assert torch.equal(got_c, want_c), rep
        assert torch.equal(got_i, want_i), rep


def _dense(code, S, k, p, seed):
    """k syndromes of dense errors (H e for e of density p) in place of the first k shots: their
    clusters outgrow the 256-row LSD kernel and reach the overflow kernels."""
    rng = np.random.default_rng(seed)
    E = (rng.random((k, code.n)) < p).astype(np.int64)
    S = S.copy()
    S[:k] = ((E @ code.H.T.astype(np.int64)) & 1).astype(np.uint8)
    return np.ascontiguousarray(S)


@pytest.mark.parametrize("which", ["hgp24", "dem_batched"])
def test_overflow_and_schedule_graph_replays_match_eager(which):
    """The same with the overflow kernels in the graph (dense shots in every replay) and, on the
    DEM with LSD-10, the cluster-batched schedule."""
    if which == "hgp24":
        code, B, kw, dense_p = random_34_hgp(24, p=0.04), 2048, dict(max_iter=30), 0.15
    else:
        code, B, kw, dense_p = synthetic_dem(), 512, dict(max_iter=30, lsd_order=10), 0.02
    bc = binding.Code.from_dense(code.H)
    graphed = binding.Decoder(bc, code.priors, B, **kw)
    eager = binding.Decoder(bc, code.priors, B, **kw)
    if which == "dem_batched":
        graphed.set_lsd_schedule(binding.LSD_CLUSTER_BATCHED)
    s_static = torch.zeros((B, code.m), dtype=torch.uint8, device="cuda")
    c_static = torch.zeros((B, code.n), dtype=torch.uint8, device="cuda")
    i_static = torch.zeros((B, 12), dtype=torch.uint8, device="cuda")
    _, S0 = sample(code, B, seed=70)
    s_static.copy_(torch.from_numpy(_dense(code, S0, 3, dense_p, 70)).cuda())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        graphed.decode_into(s_static, c_static, i_static)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graphed.decode_into(s_static, c_static, i_static)
    torch.cuda.synchronize()
    for rep in range(3):
        _, S = sample(code, B, seed=71 + rep)
        S = _dense(code, S, 3, dense_p, 71 + rep)
        s = torch.from_numpy(S).cuda()
        s_static.copy_(s)
        g.replay()
        torch.cuda.synchronize()
        got_c, got_i = c_static.clone(), i_static.clone()
        want_c = torch.empty_like(c_static)
        want_i = torch.empty_like(i_static)
        eager.decode_into(s, want_c, want_i)
        torch.cuda.synchronize()
        inf = binding.parse_info(want_i.cpu().numpy())
        print(f"case graph {which} rep={rep}: largest cluster {int(inf['max_cluster_cols'].max())} columns", flush=True)
        assert not (inf["status"] & binding.ST_OVERFLOW).any()
        assert torch.equal(got_c, want_c), rep
        assert torch.equal(got_i, want_i), rep
