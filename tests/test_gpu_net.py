"""GPU parity of the learned refinement: bf16-MFMA forward and backward against the float64
oracle (oracle/learned.py), identity at zero output weights, and training on the GPU."""
import numpy as np
import pytest

import oracle.learned as ol
from paper_2406_18655_amd import binding
from paper_2406_18655_amd.workloads import bivariate_bicycle, surface_hgp, sample

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def _bp_failures(code, shots, seed, T=30):
    bc = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bc, code.priors, shots, max_iter=T)
    e, S = sample(code, shots, seed=seed)
    s = torch.from_numpy(S).cuda()
    llr, hard, info = dec.bp(s)
    torch.cuda.synchronize()
    inf = binding.parse_info(info)
    idx = np.nonzero((inf["status"] & 1) == 0)[0]
    return bc, e[idx], S[idx], llr.cpu().numpy()[idx]


def _theta(seed):
    rng = np.random.default_rng(seed)
    th = ol.init_params(seed=seed, zero_output=False)
    return (th + rng.normal(size=th.shape) * 0.05).astype(np.float32)


# Per-value bounds.  The kernels round weights and activations to bf16 (unit roundoff 2^-8) and
# accumulate in float32; an emulation of that arithmetic in float64 on these workloads put the
# largest per-value deviation at 1.2e-2 of (|value| + the shot's RMS) for Delta and 7e-2 of
# (|value| + the block's RMS) for a gradient entry.  The bounds below leave about 3x of margin; a
# wrong neighbour, sign or layer moves a value by the order of the RMS itself.
FWD_TOL = 0.04
GRAD_TOL = 0.2


def _assert_delta_close(d_gpu, d_ref, what):
    bound = FWD_TOL * (np.abs(d_ref) + np.sqrt(np.mean(d_ref ** 2)))
    ratio = float((np.abs(d_gpu - d_ref) / np.maximum(bound, 1e-12)).max())
    assert ratio <= 1.0, (what, ratio)
    return ratio


def _assert_grad_close(g, g_ref, what):
    worst, off = 0.0, 0
    for name, shp in ol.PARAM_LAYOUT:
        k = int(np.prod(shp))
        gr, gg = g_ref[off:off + k], g[off:off + k]
        bound = GRAD_TOL * (np.abs(gr) + np.sqrt(np.mean(gr ** 2)))
        r = float((np.abs(gg - gr) / np.maximum(bound, 1e-12)).max())
        assert r <= 1.0, (what, name, r)
        worst = max(worst, r)
        off += k
    return worst


def test_forward_matches_oracle():
    code = bivariate_bicycle(p=0.06)
    bc, e, S, L = _bp_failures(code, 2000, seed=4)
    S, L = S[:64], L[:64]
    th = _theta(7)
    net = binding.Net(bc, code.priors, th)
    out = net.forward(torch.from_numpy(S).cuda(), torch.from_numpy(L).cuda())
    torch.cuda.synchronize()
    d_gpu = out.cpu().numpy().astype(np.float64) - L.astype(np.float64)
    lam = np.log((1 - code.priors) / code.priors).astype(np.float32).astype(np.float64)
    worst = 0.0
    for b in range(len(S)):
        d_ref = ol.forward(th.astype(np.float64), code.H, L[b].astype(np.float64), lam, S[b])
        rel = np.linalg.norm(d_gpu[b] - d_ref) / max(np.linalg.norm(d_ref), 1e-6)
        assert rel <= 2e-2, (b, rel)
        worst = max(worst, _assert_delta_close(d_gpu[b], d_ref, b))
    print(f"worst per-value deviation of Delta: {worst:.2f} of the bound")


def test_gradient_matches_oracle():
    code = bivariate_bicycle(p=0.06)
    bc, e, S, L = _bp_failures(code, 2000, seed=5)
    S, L, e = S[:32], L[:32], e[:32]
    th = _theta(8)
    net = binding.Net(bc, code.priors, th)
    g, loss = net.gradient(torch.from_numpy(S).cuda(), torch.from_numpy(L).cuda(), torch.from_numpy(e).cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    lam = np.log((1 - code.priors) / code.priors).astype(np.float32).astype(np.float64)
    l_ref, g_ref = ol.batch_loss_and_grad(th.astype(np.float64), code.H, [x.astype(np.float64) for x in L], lam, S, e)
    assert abs(float(loss.item()) - l_ref) <= 1e-3 * max(1.0, abs(l_ref))
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    cos = float(g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref)))
    print(f"gradient relative L2 error {rel:.2e}, cosine {cos:.6f}")
    assert rel <= 5e-2 and cos >= 0.998
    # every entry of every parameter block, not only the dominant ones
    worst = _assert_grad_close(g, g_ref, "bb144")
    print(f"worst per-value gradient deviation: {worst:.2f} of the bound")


def test_zero_output_net_decodes_like_plain():
    code = bivariate_bicycle(p=0.05)
    bc = binding.Code.from_dense(code.H)
    e, S = sample(code, 20000, seed=6)
    s = torch.from_numpy(S).cuda()
    plain = binding.Decoder(bc, code.priors, 20000, max_iter=50)
    c0 = plain.decode(s).cpu().numpy()
    learned = binding.Decoder(bc, code.priors, 20000, max_iter=50)
    net = binding.Net(bc, code.priors, ol.init_params(seed=2, zero_output=True).astype(np.float32))
    binding.attach_net(learned, net)
    c1 = learned.decode(s).cpu().numpy()
    assert (c0 == c1).all()


def test_training_reduces_loss():
    code = bivariate_bicycle(p=0.05)
    bc, e, S, L = _bp_failures(code, 40000, seed=9)
    th = ol.init_params(seed=0, zero_output=True).astype(np.float32)
    net = binding.Net(bc, code.priors, th)
    Sd, Ld, Ed = (torch.from_numpy(x).cuda() for x in (S, L, e))
    _, l0 = net.gradient(Sd[:2048], Ld[:2048], Ed[:2048])
    B = 512
    for step in range(150):
        k = (step * B) % (len(S) - B)
        net.train_step(Sd[k:k + B], Ld[k:k + B], Ed[k:k + B], 2e-3)
    _, l1 = net.gradient(Sd[:2048], Ld[:2048], Ed[:2048])
    torch.cuda.synchronize()
    print(f"loss {l0.item():.4f} -> {l1.item():.4f}")
    assert l1.item() < l0.item()


def test_forward_matches_oracle_irregular_code():
    """The distance-5 surface code (row weights 2..4, column weights 1..2): the kernel instance
    that walks neighbour lists of the code's own maximum weights, padded with a zero row."""
    code = surface_hgp(5, 0.1)
    bc, e, S, L = _bp_failures(code, 4000, seed=12)
    S, L = S[:64], L[:64]
    th = _theta(9)
    net = binding.Net(bc, code.priors, th)
    out = net.forward(torch.from_numpy(S).cuda(), torch.from_numpy(L).cuda())
    torch.cuda.synchronize()
    d_gpu = out.cpu().numpy().astype(np.float64) - L.astype(np.float64)
    lam = np.log((1 - code.priors) / code.priors).astype(np.float32).astype(np.float64)
    for b in range(len(S)):
        d_ref = ol.forward(th.astype(np.float64), code.H, L[b].astype(np.float64), lam, S[b])
        rel = np.linalg.norm(d_gpu[b] - d_ref) / max(np.linalg.norm(d_ref), 1e-6)
        assert rel <= 2e-2, (b, rel)
        _assert_delta_close(d_gpu[b], d_ref, b)


def test_set_priors_equals_fresh_net():
    code_a, code_b = bivariate_bicycle(p=0.03), bivariate_bicycle(p=0.06)
    bc, e, S, L = _bp_failures(code_b, 2000, seed=13)
    th = _theta(10)
    s, l = torch.from_numpy(S[:256]).cuda(), torch.from_numpy(L[:256]).cuda()
    moved = binding.Net(bc, code_a.priors, th)
    moved.set_priors(code_b.priors)
    fresh = binding.Net(bc, code_b.priors, th)
    assert torch.equal(moved.forward(s, l), fresh.forward(s, l))


def test_trained_net_gain():
    """What the trained refinement buys on held-out shots of [[144,12,12]] at p = 0.05 (weights
    trained by paper_2406_18655_amd.train_ordering on other seeds): BP with 10 iterations, the
    net and LSD against plain BP+LSD with 50 and with 10 iterations, paired on the same shots
    (McNemar: shots one decoder gets right and the other wrong)."""
    import os
    from paper_2406_18655_amd.workloads import logical_failures
    w = os.path.join(os.path.dirname(binding.__file__), "weights", "bb144_p0.05_T10.npy")
    code = bivariate_bicycle(p=0.05)
    bc = binding.Code.from_dense(code.H)
    net = binding.Net(bc, code.priors, np.load(w))
    B = 65536
    decs = {"plain50": binding.Decoder(bc, code.priors, B, max_iter=50),
            "plain10": binding.Decoder(bc, code.priors, B, max_iter=10),
            "learned10": binding.Decoder(bc, code.priors, B, max_iter=10)}
    binding.attach_net(decs["learned10"], net)
    fails = {k: [] for k in decs}
    for rep in range(2):
        e, S = sample(code, B, seed=900_000 + rep)
        s = torch.from_numpy(S).cuda()
        for k, d in decs.items():
            c = d.decode(s).cpu().numpy()
            assert (((c.astype(np.int64) @ code.H.T.astype(np.int64)) & 1) == S).all(), k
            fails[k].append(logical_failures(code, e, c))
    f = {k: np.concatenate(v) for k, v in fails.items()}
    ler = {k: float(v.mean()) for k, v in f.items()}
    print("LER", ler)
    for base in ("plain50", "plain10"):
        b = int(np.sum(f[base] & ~f["learned10"]))  # learned fixes
        c = int(np.sum(~f[base] & f["learned10"]))  # learned breaks
        z = (b - c) / np.sqrt(max(b + c, 1))
        print(f"vs {base}: fixes {b}, breaks {c}, z = {z:.1f}")
        assert z > 3.0, (base, b, c)


@pytest.mark.parametrize("which", ["hgp16", "dem"])
def test_large_graph_forward_and_gradient_match_oracle(which):
    """Graphs whose activations do not fit in LDS (HGP n=400 and the 936 x 8800 detector error
    model): the same kernels with activations in a device workspace, forward and gradient
    against the float64 oracle."""
    from paper_2406_18655_amd.workloads import random_34_hgp, synthetic_dem
    code = random_34_hgp(16, p=0.05) if which == "hgp16" else synthetic_dem()
    bc, e, S, L = _bp_failures(code, 3000 if which == "dem" else 2000, seed=14, T=20)
    nf, ng = (6, 3) if which == "dem" else (32, 8)
    assert len(S) >= nf
    th = _theta(12)
    net = binding.Net(bc, code.priors, th)
    lam = np.log((1 - code.priors) / code.priors).astype(np.float32).astype(np.float64)
    out = net.forward(torch.from_numpy(S[:nf]).cuda(), torch.from_numpy(L[:nf]).cuda())
    torch.cuda.synchronize()
    d_gpu = out.cpu().numpy().astype(np.float64) - L[:nf].astype(np.float64)
    for b in range(nf):
        d_ref = ol.forward(th.astype(np.float64), code.H, L[b].astype(np.float64), lam, S[b])
        rel = np.linalg.norm(d_gpu[b] - d_ref) / max(np.linalg.norm(d_ref), 1e-6)
        assert rel <= 2e-2, (b, rel)
        _assert_delta_close(d_gpu[b], d_ref, (which, b))
    g, loss = net.gradient(torch.from_numpy(S[:ng]).cuda(), torch.from_numpy(L[:ng]).cuda(),
                           torch.from_numpy(e[:ng]).cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    l_ref, g_ref = ol.batch_loss_and_grad(th.astype(np.float64), code.H, [x.astype(np.float64) for x in L[:ng]],
                                          lam, S[:ng], e[:ng])
    assert abs(float(loss.item()) - l_ref) <= 1e-3 * max(1.0, abs(l_ref))
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    cos = float(g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref)))
    print(f"{which}: gradient relative L2 error {rel:.2e}, cosine {cos:.6f}")
    assert rel <= 5e-2 and cos >= 0.998
    worst = _assert_grad_close(g, g_ref, which)
    print(f"{which}: worst per-value gradient deviation {worst:.2f} of the bound")


def test_large_graph_heavy_columns_match_oracle():
    """Large-graph inference on a graph built to reach the paths the detector error model does not:
    columns of weight 7, 9 and 10 (tiles heavier than one gather pass), passes whose two tiles
    differ in weight, rows of mixed weight, and a fault count that pads its last tile (1100
    faults: more feature rows than the wave-per-shot kernel can address, so the large-graph kernel
    runs).  Forward on random syndromes and LLRs against the float64 oracle."""
    rng = np.random.default_rng(31)
    m, n = 300, 1100
    H = np.zeros((m, n), dtype=np.uint8)
    w = rng.choice([2, 3, 7, 9, 10], size=n, p=[0.5, 0.3, 0.1, 0.05, 0.05])
    for j in range(n):
        H[rng.choice(m, size=int(w[j]), replace=False), j] = 1
    for i in np.nonzero(H.sum(1) < 2)[0]:
        H[i, rng.choice(n, size=2, replace=False)] = 1
    assert H.sum(0).max() == 10 and (n + 15) // 16 * 16 + 1 > 1023
    priors = rng.uniform(0.01, 0.1, size=n)
    lam = np.log((1 - priors) / priors).astype(np.float32).astype(np.float64)
    nf = 6
    S = rng.integers(0, 2, size=(nf, m), dtype=np.uint8)
    L = (lam[None, :] + rng.normal(0.0, 3.0, size=(nf, n))).astype(np.float32)
    th = _theta(17)
    net = binding.Net(binding.Code.from_dense(H), priors, th)
    out = net.forward(torch.from_numpy(S).cuda(), torch.from_numpy(L).cuda())
    torch.cuda.synchronize()
    d_gpu = out.cpu().numpy().astype(np.float64) - L.astype(np.float64)
    worst = 0.0
    for b in range(nf):
        d_ref = ol.forward(th.astype(np.float64), H, L[b].astype(np.float64), lam, S[b])
        rel = np.linalg.norm(d_gpu[b] - d_ref) / max(np.linalg.norm(d_ref), 1e-6)
        assert rel <= 2e-2, (b, rel)
        worst = max(worst, _assert_delta_close(d_gpu[b], d_ref, ("heavy", b)))
    print(f"heavy columns: worst per-value deviation {worst:.2f} of the bound")


def test_net_rejects_other_code():
    bb, sc = bivariate_bicycle(p=0.05), surface_hgp(5, 0.05)
    net = binding.Net(binding.Code.from_dense(bb.H), bb.priors, _theta(1))
    dec = binding.Decoder(binding.Code.from_dense(sc.H), sc.priors, 16, max_iter=5)
    with pytest.raises(binding.QlsdError):
        binding.attach_net(dec, net)


def test_dem_zero_output_net_decodes_like_plain():
    """Decoding the detector error model through the large-graph refinement path (decoder-owned
    feature workspace) with a zero output layer leaves BP+LSD-10 unchanged."""
    from paper_2406_18655_amd.workloads import synthetic_dem
    code = synthetic_dem()
    bc = binding.Code.from_dense(code.H)
    e, S = sample(code, 4096, seed=15)
    s = torch.from_numpy(S).cuda()
    plain = binding.Decoder(bc, code.priors, 4096, max_iter=30, lsd_order=10)
    c0 = plain.decode(s).cpu().numpy()
    learned = binding.Decoder(bc, code.priors, 4096, max_iter=30, lsd_order=10)
    net = binding.Net(bc, code.priors, ol.init_params(seed=4, zero_output=True).astype(np.float32))
    binding.attach_net(learned, net)
    c1 = learned.decode(s).cpu().numpy()
    assert (c0 == c1).all()


def test_dem_trained_net_gain():
    """Trained refinement on the detector error model (weights from train_ordering --code dem,
    BP 30 iterations): word errors on 2^20 held-out shots drawn on the GPU, paired against plain
    BP (100 iterations) + LSD-10."""
    import os
    from paper_2406_18655_amd.workloads import synthetic_dem
    from paper_2406_18655_amd.binding import DeviceSampler
    code = synthetic_dem()
    bc = binding.Code.from_dense(code.H)
    w = os.path.join(os.path.dirname(binding.__file__), "weights", "dem_T30.npy")
    net = binding.Net(bc, code.priors, np.load(w))
    B = 65536
    plain = binding.Decoder(bc, code.priors, B, max_iter=100, lsd_order=10)
    learned = binding.Decoder(bc, code.priors, B, max_iter=30, lsd_order=10)
    binding.attach_net(learned, net)
    ds = DeviceSampler(code)
    fixes = breaks = fp = fl = 0
    for rep in range(16):
        e, s = ds.sample(B, 5_000_000 + rep)
        cp, cl = plain.decode(s), learned.decode(s)
        assert torch.equal(ds.syndromes(cl), s) and torch.equal(ds.syndromes(cp), s)
        f_p, f_l = ds.failures(e, cp), ds.failures(e, cl)
        fixes += int((f_p & ~f_l).sum().item())
        breaks += int((~f_p & f_l).sum().item())
        fp += int(f_p.sum().item())
        fl += int(f_l.sum().item())
    z = (fixes - breaks) / np.sqrt(max(fixes + breaks, 1))
    print(f"DEM word error plain {fp / (16 * B):.5f} learned {fl / (16 * B):.5f}; fixes {fixes} breaks {breaks} z {z:.1f}")
    assert z > 3.0
