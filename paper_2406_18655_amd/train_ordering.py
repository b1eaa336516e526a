"""Trains the learned LLR refinement on the GPU and scores it against plain BP+LSD.

Training data are (syndrome, true error, BP posterior) triples: syndromes and errors from the
seeded code-capacity sampler, posteriors from this library's BP (qlsd_bp) with the learned
decoder's iteration budget; only shots that BP does not solve are kept (the refinement only
ever sees those).  Every forward/backward/Adam step runs in libqlsd's HIP kernels
(include/qlsd_net.h).  Scoring decodes held-out shots with the plain decoder (BP, max_iter
iterations, then LSD) and with the learned one (BP with `learned_iter` iterations, refinement,
LSD), and reports the logical error rates and the decode throughput of both.

    python -m paper_2406_18655_amd.train_ordering --train-shots 5000000 --eval-shots 1000000

With several noise strengths (--p 0.01,0.02,0.04,0.05,0.06) the training batches cycle over
them, each decoded by BP with its own priors and fed to the net with those priors; scoring then
runs at every listed strength with the one trained net.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_DIR = os.path.join(HERE, "weights")


def _init_params(seed: int) -> np.ndarray:
    """Glorot-uniform matrices, zero vectors, zero output layer (so training starts from
    the identity refinement, i.e. plain BP+LSD)."""
    from . import binding
    rng = np.random.default_rng(seed)
    parts = []
    shapes = ([(32, 2), (32,)] + [s for _ in range(3) for s in ((32, 32), (32,), (32, 32), (32, 32), (32,))]
              + [(32,), (1,)])
    for shp in shapes:
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, size=shp).reshape(-1))
        else:
            parts.append(np.zeros(shp))
    th = np.concatenate(parts).astype(np.float32)
    assert th.shape == (binding.NET_PARAMS,)
    return th


def collect(codes, bc, shots: int, seed: int, learned_iter: int, batch: int = 65536):
    """Yields (index into codes, S, E, L) of BP failures, batch by batch, cycling over the codes
    (one matrix at several noise strengths)."""
    import torch
    from . import binding
    from .workloads import sample
    decs = [binding.Decoder(bc, c.priors, batch, max_iter=learned_iter) for c in codes]
    done = 0
    k = 0
    while done < shots:
        B = min(batch, shots - done)
        ci = k % len(codes)
        e, S = sample(codes[ci], B, seed=seed + k)
        s = torch.from_numpy(S).cuda()
        llr, hard, info = decs[ci].bp(s)
        torch.cuda.synchronize()
        inf = binding.parse_info(info)
        idx = np.nonzero((inf["status"] & binding.ST_BP_CONVERGED) == 0)[0]
        idx_t = torch.from_numpy(idx).cuda()
        yield ci, s[idx_t].contiguous(), torch.from_numpy(e[idx]).cuda(), llr[idx_t].contiguous()
        done += B
        k += 1


def train(codes, learned_iter: int, train_shots: int, seed: int = 1, lr: float = 2e-3, minibatch: int = 1024,
          log=print):
    """codes: one CheckMatrix or a list of them sharing H (different priors)."""
    import torch
    from . import binding
    codes = codes if isinstance(codes, (list, tuple)) else [codes]
    bc = binding.Code.from_dense(codes[0].H)
    net = binding.Net(bc, codes[0].priors, _init_params(seed))
    t0 = time.perf_counter()
    steps, seen, last = 0, 0, 0
    total_steps = max(1, int(train_shots * 0.2 / minibatch))
    tb = time.perf_counter()
    for ci, S, E, L in collect(codes, bc, train_shots, seed=10_000 + seed, learned_iter=learned_iter):
        t_data = time.perf_counter() - tb
        if len(codes) > 1:
            net.set_priors(codes[ci].priors)
        n = S.shape[0]
        for k in range(0, n - minibatch + 1, minibatch):
            frac = min(1.0, steps / total_steps)
            cur_lr = lr * (0.1 ** frac)  # exponential decay to lr/10
            net.train_step(S[k:k + minibatch], L[k:k + minibatch], E[k:k + minibatch], cur_lr)
            steps += 1
        torch.cuda.synchronize()
        seen += n
        if steps - last >= 100 or seen == n:
            last = steps
            _, loss = net.gradient(S[:minibatch], L[:minibatch], E[:minibatch])
            log(f"  step {steps}  examples {seen}  loss {loss.item():.4f}  data {t_data:.2f}s  "
                f"total {time.perf_counter() - t0:.1f}s")
        tb = time.perf_counter()
    torch.cuda.synchronize()
    return net, bc, {"steps": steps, "examples": seen, "seconds": round(time.perf_counter() - t0, 1)}


def evaluate(code, bc, net, plain_iter: int, learned_iter: int, eval_shots: int, seed: int = 77, batch: int = 65536,
             reps: int = 3):
    """LER of plain BP+LSD (plain_iter BP iterations), of plain BP+LSD with the learned form's
    iteration budget, and of the learned form, on the same held-out shots; decode time per batch
    of each.  Every correction is checked against its syndrome."""
    import torch
    from . import binding
    from .workloads import sample, logical_failures
    decs = {"plain": binding.Decoder(bc, code.priors, batch, max_iter=plain_iter),
            "plain_same_iter": binding.Decoder(bc, code.priors, batch, max_iter=learned_iter),
            "learned": binding.Decoder(bc, code.priors, batch, max_iter=learned_iter)}
    binding.attach_net(decs["learned"], net)
    if learned_iter == plain_iter:
        del decs["plain_same_iter"]
    fails = {k: 0 for k in decs}
    times = {k: [] for k in decs}
    Hs = code.H.astype(np.int32)
    total = 0
    corr = torch.empty((batch, code.n), dtype=torch.uint8, device="cuda")
    k = 0
    while total < eval_shots:
        B = min(batch, eval_shots - total)
        e, S = sample(code, B, seed=seed + k)
        s = torch.from_numpy(S).cuda()
        for name, dec in decs.items():
            out = corr[:B]
            for r in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                dec.decode_into(s, out)
                b.record()
                torch.cuda.synchronize()
                if k > 0 or r > 0:
                    times[name].append(a.elapsed_time(b) / B)
            c = out.cpu().numpy()
            bad = int(np.count_nonzero(((c.astype(np.int32) @ Hs.T) & 1) != S))
            if bad:
                raise RuntimeError(f"{name}: {bad} syndrome bits not matched by the corrections")
            fails[name] += int(logical_failures(code, e, c).sum())
        total += B
        k += 1
    res = {}
    for name in decs:
        p = fails[name] / total
        res[name] = {"ler": p, "sigma": float(np.sqrt(max(p, 1.0 / total) * (1 - p) / total)),
                     "shots_per_s": 1e3 / float(np.mean(times[name]))}
    res["shots"] = total
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--p", default="0.05", help="noise strength, or a comma-separated list to train over")
    ap.add_argument("--plain-iter", type=int, default=50)
    ap.add_argument("--learned-iter", type=int, default=20)
    ap.add_argument("--train-shots", type=int, default=5_000_000)
    ap.add_argument("--eval-shots", type=int, default=1_000_000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--save", default=None, help="path of the .npy to write (default weights/bb144_p{p}_T{T}.npy)")
    args = ap.parse_args()
    from .workloads import bivariate_bicycle
    ps = [float(x) for x in args.p.split(",")]
    codes = [bivariate_bicycle(p=p) for p in ps]
    print(f"training on [[144,12,12]] p={ps}, BP {args.learned_iter} iterations, {args.train_shots} shots", flush=True)
    net, bc, tinfo = train(codes, args.learned_iter, args.train_shots, seed=args.seed, lr=args.lr,
                           log=lambda s: print(s, flush=True))
    os.makedirs(WEIGHTS_DIR, exist_ok=True)
    tag = "mix" if len(ps) > 1 else f"p{ps[0]:g}"
    path = args.save or os.path.join(WEIGHTS_DIR, f"bb144_{tag}_T{args.learned_iter}.npy")
    np.save(path, net.get_params())
    print(json.dumps({"train": tinfo, "weights": os.path.relpath(path, os.path.dirname(HERE)),
                      "plain_iter": args.plain_iter, "learned_iter": args.learned_iter}), flush=True)
    for code, p in zip(codes, ps):
        res = evaluate(code, bc, net, args.plain_iter, args.learned_iter, args.eval_shots)
        print(json.dumps({"p": p, **res}), flush=True)


if __name__ == "__main__":
    main()
