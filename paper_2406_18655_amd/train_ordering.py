"""Trains the learned LLR refinement on the GPU and scores it against plain BP+LSD.

Training data are (syndrome, true error, BP posterior) triples: syndromes and errors from the
seeded noise sampler, posteriors from this library's BP (qlsd_bp) with the learned decoder's
iteration budget; only shots that BP does not solve are kept (the refinement only ever sees
those).  Every forward/backward/Adam step runs in libqlsd's HIP kernels (include/qlsd_net.h).
Scoring decodes held-out shots with the plain decoder (BP with plain_iter iterations, then LSD),
with plain BP+LSD at the learned form's iteration budget, and with the learned form (BP with
learned_iter iterations, refinement, LSD), and reports logical error rates and throughput.

    python -m paper_2406_18655_amd.train_ordering --train-shots 5000000 --eval-shots 1000000
    python -m paper_2406_18655_amd.train_ordering --code dem --learned-iter 30

[[144,12,12]] (--code bb144): shots from the host sampler; with several noise strengths
(--p 0.01,0.02,0.04,0.05,0.06) the training batches cycle over them, each decoded by BP with its
own priors and fed to the net with those priors; scoring runs at every listed strength.
Detector error model (--code dem): 936 x 8800, LSD order 10, shots drawn on the GPU
(the library's Philox sampler, binding.DeviceSampler), word error as the failure criterion.
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


class Workload:
    """One check matrix at one or more noise strengths, with its sampler and decoder settings."""

    def __init__(self, name, codes, batch, lsd_order, device_sampling):
        self.name, self.codes, self.batch, self.lsd_order = name, codes, batch, lsd_order
        self.device_sampling = device_sampling
        self._dev = {}

    def _sampler(self, ci):
        from .binding import DeviceSampler
        if ci not in self._dev:
            self._dev[ci] = DeviceSampler(self.codes[ci])
        return self._dev[ci]

    def draw(self, ci: int, shots: int, seed: int):
        """(errors, syndromes) as uint8 device tensors."""
        import torch
        if self.device_sampling:
            return self._sampler(ci).sample(shots, seed)
        from .workloads import sample
        e, S = sample(self.codes[ci], shots, seed=seed)
        return torch.from_numpy(e).cuda(), torch.from_numpy(S).cuda()

    def failures(self, ci, e, c):
        return self._sampler(ci).failures(e, c)

    def syndromes(self, ci, c):
        return self._sampler(ci).syndromes(c)


def collect(wl: Workload, bc, shots: int, seed: int, learned_iter: int):
    """Yields (index into wl.codes, S, E, L) of BP failures, batch by batch, cycling over the
    codes (one matrix at several noise strengths)."""
    import torch
    from . import binding
    decs = [binding.Decoder(bc, c.priors, wl.batch, max_iter=learned_iter, lsd_order=wl.lsd_order) for c in wl.codes]
    done = 0
    k = 0
    while done < shots:
        B = min(wl.batch, shots - done)
        ci = k % len(wl.codes)
        e, s = wl.draw(ci, B, seed + k)
        llr, hard, info = decs[ci].bp(s)
        torch.cuda.synchronize()
        inf = binding.parse_info(info)
        idx = torch.from_numpy(np.nonzero((inf["status"] & binding.ST_BP_CONVERGED) == 0)[0]).cuda()
        yield ci, s[idx].contiguous(), e[idx].contiguous(), llr[idx].contiguous()
        done += B
        k += 1


def train(wl: Workload, learned_iter: int, train_shots: int, seed: int = 1, lr: float = 2e-3, minibatch: int = 1024,
          log=print):
    import torch
    from . import binding
    bc = binding.Code.from_dense(wl.codes[0].H)
    net = binding.Net(bc, wl.codes[0].priors, _init_params(seed))
    t0 = time.perf_counter()
    steps, seen, last = 0, 0, 0
    total_steps = max(1, int(train_shots * 0.2 / minibatch))
    tb = time.perf_counter()
    for ci, S, E, L in collect(wl, bc, train_shots, seed=10_000 + seed, learned_iter=learned_iter):
        t_data = time.perf_counter() - tb
        if len(wl.codes) > 1:
            net.set_priors(wl.codes[ci].priors)
        n = S.shape[0]
        for k in range(0, n - minibatch + 1, minibatch):
            frac = min(1.0, steps / total_steps)
            cur_lr = lr * (0.1 ** frac)  # exponential decay to lr/10
            net.train_step(S[k:k + minibatch], L[k:k + minibatch], E[k:k + minibatch], cur_lr)
            steps += 1
        torch.cuda.synchronize()
        seen += n
        if steps - last >= 100 or seen == n or time.perf_counter() - tb > 20:
            last = steps
            _, loss = net.gradient(S[:minibatch], L[:minibatch], E[:minibatch])
            log(f"  step {steps}  examples {seen}  loss {loss.item():.4f}  data {t_data:.2f}s  "
                f"total {time.perf_counter() - t0:.1f}s")
        tb = time.perf_counter()
    torch.cuda.synchronize()
    if len(wl.codes) > 1:
        net.set_priors(wl.codes[0].priors)
    return net, bc, {"steps": steps, "examples": seen, "seconds": round(time.perf_counter() - t0, 1)}


def evaluate(wl: Workload, ci: int, bc, net, plain_iter: int, learned_iter: int, eval_shots: int, seed: int = 77,
             reps: int = 3, log=print):
    """LER of plain BP+LSD (plain_iter BP iterations), of plain BP+LSD with the learned form's
    iteration budget, and of the learned form, on the same held-out shots; decode time per batch
    of each.  Every correction is checked against its syndrome."""
    import torch
    from . import binding
    code, batch = wl.codes[ci], wl.batch
    mk = lambda T: binding.Decoder(bc, code.priors, batch, max_iter=T, lsd_order=wl.lsd_order)
    decs = {"plain": mk(plain_iter), "plain_same_iter": mk(learned_iter), "learned": mk(learned_iter)}
    binding.attach_net(decs["learned"], net)
    if learned_iter == plain_iter:
        del decs["plain_same_iter"]
    fails = {k: 0 for k in decs}
    times = {k: [] for k in decs}
    total = 0
    corr = torch.empty((batch, code.n), dtype=torch.uint8, device="cuda")
    k = 0
    while total < eval_shots:
        B = min(batch, eval_shots - total)
        e, s = wl.draw(ci, B, seed + k)
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
            bad = int((wl.syndromes(ci, out) != s).sum().item())
            if bad:
                raise RuntimeError(f"{name}: {bad} syndrome bits not matched by the corrections")
            fails[name] += int(wl.failures(ci, e, out).sum().item())
        total += B
        k += 1
        if k % 16 == 0:
            log(f"  scored {total} shots")
    res = {}
    for name in decs:
        p = fails[name] / total
        res[name] = {"ler": p, "sigma": float(np.sqrt(max(p, 1.0 / total) * (1 - p) / total)),
                     "shots_per_s": 1e3 / float(np.mean(times[name]))}
    res["shots"] = total
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--code", choices=["bb144", "dem"], default="bb144")
    ap.add_argument("--p", default="0.05", help="bb144: noise strength, or a comma-separated list to train over")
    ap.add_argument("--plain-iter", type=int, default=None, help="default 50 (bb144) / 100 (dem)")
    ap.add_argument("--learned-iter", type=int, default=None, help="default 10 (bb144) / 30 (dem)")
    ap.add_argument("--train-shots", type=int, default=5_000_000)
    ap.add_argument("--eval-shots", type=int, default=1_000_000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--save", default=None, help="path of the .npy to write (default under weights/)")
    args = ap.parse_args()
    from .workloads import bivariate_bicycle, synthetic_dem
    log = lambda s: print(s, flush=True)
    if args.code == "dem":
        wl = Workload("dem936x8800", [synthetic_dem()], 16384, 10, device_sampling=True)
        plain_iter, learned_iter = args.plain_iter or 100, args.learned_iter or 30
        tag, labels = f"dem_T{learned_iter}", ["dem"]
    else:
        ps = [float(x) for x in args.p.split(",")]
        wl = Workload("bb144", [bivariate_bicycle(p=p) for p in ps], 65536, 0, device_sampling=False)
        plain_iter, learned_iter = args.plain_iter or 50, args.learned_iter or 10
        tag = f"bb144_{'mix' if len(ps) > 1 else f'p{ps[0]:g}'}_T{learned_iter}"
        labels = ps
    log(f"training on {wl.name} {labels}, BP {learned_iter} iterations, {args.train_shots} shots")
    net, bc, tinfo = train(wl, learned_iter, args.train_shots, seed=args.seed, lr=args.lr, log=log)
    os.makedirs(WEIGHTS_DIR, exist_ok=True)
    path = args.save or os.path.join(WEIGHTS_DIR, f"{tag}.npy")
    np.save(path, net.get_params())
    log(json.dumps({"train": tinfo, "weights": os.path.relpath(path, os.path.dirname(HERE)),
                    "plain_iter": plain_iter, "learned_iter": learned_iter}))
    for ci, lab in enumerate(labels):
        res = evaluate(wl, ci, bc, net, plain_iter, learned_iter, args.eval_shots, log=log)
        log(json.dumps({"code": wl.name, "p": lab, **res}))


if __name__ == "__main__":
    main()
