#!/usr/bin/env python3
"""Benchmark: decoded shots/s of BP + LSD-0 on the [[144,12,12]] bivariate bicycle code.

Workload: H_X of the BB code (l=12, m=6, A = x^3+y+y^2, B = y^3+x+x^2), 72 x 144, under
code-capacity X noise at p = 0.05; 65,536 seeded shots per step; min-sum BP (alpha = 0.625,
at most 50 iterations, early exit) then LSD-0 on the shots BP does not solve.  A step is one
qlsd_decode call over a batch whose syndromes already sit in HBM.

Prints one JSON line (see --help).  Besides shots/s it reports per-launch latency
percentiles, the logical error rate of the GPU run next to the oracle's on the same shots,
the BP kernel's roofline position (algorithmic bytes per launch / its measured duration,
HIP events on the launch stream, recorded on one timed step in eight) and the CPU oracle's
throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "decoded shots/s at matched LER, [[144,12,12]] p=0.05; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=["bb144", "dem"], default="bb144",
                    help="bb144: [[144,12,12]] code capacity p=0.05, BP 50 + LSD-0, 65,536 shots (headline); "
                         "dem: synthetic 936 x 8800 detector error model, BP 100 + LSD-10, 16,384 shots")
    ap.add_argument("--shots", type=int, default=None)
    ap.add_argument("--p", type=float, default=0.05)
    ap.add_argument("--max-iter", type=int, default=None)
    ap.add_argument("--lsd-order", type=int, default=None)
    ap.add_argument("--batches", type=int, default=4, help="distinct pre-generated batches cycled")
    ap.add_argument("--seed", type=int, default=20240626)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle CPU-baseline budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-ordering leg")
    ap.add_argument("--no-grid", action="store_true",
                    help="skip the learned leg's grid of plain BP budgets and LSD orders (the comparison at "
                         "matched error rate), e.g. for short profiled runs")
    ap.add_argument("--tune", action="store_true",
                    help="run qlsd_decoder_tune on batch 0 before the timed steps (on the headline batch it "
                         "lands on the default shapes within noise)")
    ap.add_argument("--learned-iter", type=int, default=None,
                    help="BP iterations of the learned form (default 10 for bb144, 30 for dem)")
    ap.add_argument("--serve", action="store_true",
                    help="streaming mode: Poisson arrivals over a mix of codes; one JSON line per rate")
    ap.add_argument("--serve-rates", default="1e5,1e6,1e7")
    ap.add_argument("--serve-ordering", default="plain,learned",
                    help="plain: BP+LSD for every code; learned: the [[144,12,12]] lanes run BP 10 + "
                         "the trained refinement + LSD")
    ap.add_argument("--serve-requests", type=int, default=1000000, help="requests per rate (all codes together)")
    ap.add_argument("--serve-hw-queues", type=int, default=8,
                    help="HIP hardware queues for the service (GPU_MAX_HW_QUEUES, set before HIP starts; HIP's "
                         "default of 4 makes lanes beyond the fourth share a queue and wait behind each other's "
                         "batches); 0 leaves the environment as it is")
    ap.add_argument("--sweep", action="store_true",
                    help="[[144,12,12]] over p in {0.01,0.02,0.04,0.05,0.06}: 10^6 shots per point "
                         "(15 launches of 65,536 plus one of 16,960), GPU LER and shots/s, the oracle's "
                         "LER on the first 65,536 shots, and the learned form")
    ap.add_argument("--cluster-stats", action="store_true",
                    help="Appendix A's cluster statistics: nu, kappa and kappa_alpha of LSD's final clusters "
                         "(shots BP 30 does not solve) against the optimal factorization of the same errors, "
                         "[[144,12,12]] over p and the synthetic DEM, with the Bethe-lattice estimates")
    ap.add_argument("--window", action="store_true",
                    help="(3,1) overlapping-window BP + LSD over a 12-round memory experiment on [[144,12,12]] "
                         "(phenomenological noise): per-cycle logical error rate and shots/s against decoding "
                         "the whole 12-round history at once")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (three launches), the "
                         "reference for scaling HBM byte counters")
    ap.add_argument("--traffic-json", default=os.path.join(HERE, "profiles", "bp_traffic_bb144.json"),
                    help="HBM bytes per BP launch measured with rocprofv3 counters, if present")
    ap.add_argument("--counters-json", default=os.path.join(HERE, "profiles", "issue_counters_bb144.json"),
                    help="VALU / LDS instruction counts per launch of the headline kernel (rocprofv3 SQ "
                         "counters), if present and taken on the current kernel sources")
    ap.add_argument("--record-counters", nargs=2, metavar=("PASS1_CSV", "PASS2_CSV"), default=None,
                    help="write --counters-json from two rocprofv3 counter_collection.csv files of a "
                         "bench run (SQ_INSTS_VALU SQ_ACTIVE_INST_VALU ... / SQ_ACTIVE_INST_LDS ...)")
    ap.add_argument("--record-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    default=None,
                    help="write --traffic-json from rocprofv3 FETCH_SIZE / WRITE_SIZE counter_collection.csv files "
                         "of a bench run and of a --copy-calibration run")
    ap.add_argument("--latency-launches", type=int, default=200,
                    help="isolated launches timed for the per-launch latency percentiles")
    ap.add_argument("--no-stream", action="store_true", help="skip the streaming (per-request latency) leg")
    ap.add_argument("--no-osd", action="store_true", help="skip the BP + OSD-0 comparator leg")
    ap.add_argument("--no-two-streams", action="store_true",
                    help="skip the two-stream context runs (for kernel traces whose averages should not mix in "
                         "launches that overlap another decoder's)")
    ap.add_argument("--stream-requests", type=int, default=100000)
    return ap.parse_args()


def bp_algorithmic_bytes(m, n, E, iters):
    """Per shot: syndrome in and correction out as bits, plus every float32 c->v message
    and posterior written and read once per flooding iteration."""
    return float(len(iters) * ((m + 7) // 8 + (n + 7) // 8) + iters.astype(np.float64).sum() * (8 * E + 8 * n))


def lsd_algorithmic_bytes(n, n_lsd):
    """Per shot that goes on to LSD: its float32 posterior row read once (4n bytes; its syndrome
    and correction are already counted once in the BP figure)."""
    return float(n_lsd) * 4 * n


def main():
    args = parse()
    dem = args.workload == "dem"
    args.shots = args.shots or (16384 if dem else 65536)
    args.max_iter = args.max_iter or (100 if dem else 50)
    args.lsd_order = args.lsd_order if args.lsd_order is not None else (10 if dem else 0)
    args.learned_iter = args.learned_iter or (30 if dem else 10)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); shots are independent, "
              "so a multi-GPU run would be N independent copies of this launch.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2406_18655_amd import binding
    from paper_2406_18655_amd.workloads import bivariate_bicycle, synthetic_dem, sample, logical_failures, syndromes

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    code = synthetic_dem() if dem else bivariate_bicycle(p=args.p)
    B = args.shots
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)
    log(f"workload {args.workload}: sampling {args.batches} batches of {args.shots} shots")
    batches = []
    for k in range(args.batches):
        e, S = sample(code, B, seed=args.seed + k)
        batches.append((e, torch.from_numpy(S).to(dev)))
    bcode = binding.Code.from_dense(code.H)
    dec = binding.Decoder(bcode, code.priors, B, max_iter=args.max_iter, lsd_order=args.lsd_order,
                          flags=binding.FLAG_STAGE_TIMING)
    corr = torch.empty((B, code.n), dtype=torch.uint8, device=dev)
    info = torch.empty((B, 12), dtype=torch.uint8, device=dev)

    # correctness + iteration counts of each batch (untimed)
    iters_per_batch, ler_gpu, lsd_frac, lsd_count = [], [], [], []
    for e, s in batches:
        dec.decode_into(s, corr, info)
        torch.cuda.synchronize()
        inf = binding.parse_info(info)
        iters_per_batch.append(inf["bp_iters"].astype(np.int64))
        lsd_frac.append(float(((inf["status"] & binding.ST_LSD_RUN) != 0).mean()))
        lsd_count.append(int(((inf["status"] & binding.ST_LSD_RUN) != 0).sum()))
        c = corr.cpu().numpy()
        Sn = s.cpu().numpy()
        if not (syndromes(code, c) == Sn).all():
            print("correction does not satisfy its syndrome", file=sys.stderr)
            sys.exit(3)
        ler_gpu.append(logical_failures(code, e, c))

    tuning = None
    if args.tune:
        log("autotuning launch shapes on batch 0")
        tuning = dec.tune(batches[0][1], reps=3)
    log("correctness pass done; warmup and timed steps")
    for k in range(args.warmup):
        dec.decode_into(batches[k % len(batches)][1], corr, None)
    torch.cuda.synchronize()

    # timed region: exactly K steps.  The roofline's kernel durations come from the decoder's
    # stage events, recorded on one step in eight (the other steps record none: each event costs
    # a few microseconds of device time) and read once the next step is queued behind it, so the
    # sampled launch runs back to back like the others and the queue never drains
    bp_ms, lsd_ms = [], []
    pending = False
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sampled = k % 8 == 7 or k == args.steps - 1
        dec.set_stage_timing(sampled)
        dec.decode_into(batches[k % len(batches)][1], corr, None)
        if pending:
            a, b = dec.stage_ms()  # the previous step's events (this step recorded none)
            bp_ms.append(a)
            lsd_ms.append(b)
        pending = sampled
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if pending:
        a, b = dec.stage_ms()
        bp_ms.append(a)
        lsd_ms.append(b)
    dec.set_stage_timing(True)
    shots_per_s = args.steps * B / wall
    ms_per_step = wall * 1e3 / args.steps
    lat_pipe = pipelined_latencies(dec, batches, corr, args.steps)

    # per-launch latency outside the timed steps: isolated launches (each waited for), so the
    # figure is one batch's decode time, not its place in a queue of launches
    lat = isolated_latencies(dec, batches, corr, args.latency_launches)

    # Roofline of the dominant kernel: algorithmic bytes per launch over its measured average
    # duration.  [[144,12,12]]: the slot BP kernel with LSD folded in (BP's bytes plus each LSD
    # shot's posterior row); DEM: the large-graph BP kernel (LSD runs as its own kernel).
    E = code.nnz
    bp_bytes = np.mean([bp_algorithmic_bytes(code.m, code.n, E, it) for it in iters_per_batch])
    bytes_per_launch = bp_bytes if dem else bp_bytes + lsd_algorithmic_bytes(code.n, np.mean(lsd_count))
    bp_avg_ms = float(np.mean(bp_ms))
    achieved = bytes_per_launch / (bp_avg_ms * 1e-3) / 1e9
    traffic = None
    if not dem and os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            tj = json.load(f)
        if tj.get("kernel_source_hash") == _kernel_hash():
            traffic = tj.get("bytes_per_launch")
    roofline = {"bound": "hbm",
                "kernel": "bp_graph2_kernel" if dem else "bp_lds_kernel (BP + LSD-0 in one kernel)",
                "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "avg_launch_ms": round(bp_avg_ms, 4),
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "lsd_avg_launch_ms": round(float(np.mean(lsd_ms)), 4),
                "note": "algorithmic bytes count every message read and write of an HBM-resident formulation; "
                        "the messages stay in LDS, so frac compares against that formulation, not the HBM peak "
                        "(actual DRAM traffic: traffic)"}
    if not dem:
        roofline["binding"] = issue_roofline(args.counters_json, bp_avg_ms)
    if not dem:
        # context: the same BP as a kernel of its own (two-kernel path), on batch 0
        sep = binding.Decoder(bcode, code.priors, B, max_iter=args.max_iter, lsd_order=args.lsd_order,
                              flags=binding.FLAG_STAGE_TIMING | binding.FLAG_SEPARATE_LSD)
        sms = []
        for k in range(10):
            sep.decode_into(batches[0][1], corr, None)
            a, b = sep.stage_ms()
            if k >= 2:
                sms.append((a, b))
        a_ms = float(np.mean([x[0] for x in sms]))
        b0 = bp_algorithmic_bytes(code.m, code.n, E, iters_per_batch[0])
        roofline["bp_kernel_alone"] = {"avg_launch_ms": round(a_ms, 4),
                                       "frac": round(b0 / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                       "lsd_kernel_ms": round(float(np.mean([x[1] for x in sms])), 4)}
        del sep

    # logical error rate of the GPU run vs the oracle on the same shots (batch 0)
    e0, s0 = batches[0]
    if dem:
        cfg = {"workload": "dem936x8800_bp100_lsd10", "code": "synthetic detector error model, 12 rounds",
               "H": f"{code.m}x{code.n}", "nnz": int(code.nnz), "priors": "log-uniform [1e-4, 1e-2]",
               "shots_per_step": B, "max_iter": args.max_iter, "ms_scaling": 0.625, "lsd_order": args.lsd_order}
        metric = "decoded shots/s, synthetic DEM 936x8800 (BP 100 + LSD-10); p50/p99 latency"
    else:
        cfg = {"workload": "bb144_codecap_p0.05_bp50_lsd0", "code": "[[144,12,12]] BB l=12 m=6",
               "H": "72x144", "p": args.p, "shots_per_step": B, "max_iter": args.max_iter,
               "ms_scaling": 0.625, "lsd_order": 0}
        metric = METRIC
    out = {"metric": metric, "value": round(shots_per_s, 1), "unit": "shots/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": cfg,
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                          "p99": round(float(np.percentile(lat, 99)), 4),
                          "per": f"launch of {B} shots, {len(lat)} isolated launches after the timed steps; "
                                 f"pipelined: {len(lat_pipe)} back-to-back launches after them",
                          "pipelined_p50": round(float(np.percentile(lat_pipe, 50)), 4),
                          "pipelined_p99": round(float(np.percentile(lat_pipe, 99)), 4)},
           "ler": {"gpu": round(float(np.mean([f.mean() for f in ler_gpu])), 6)},
           "bp_mean_iters": round(float(np.mean([it.mean() for it in iters_per_batch])), 3),
           "lsd_fraction": round(float(np.mean(lsd_frac)), 4),
           "roofline": roofline,
           "tuning": None if tuning is None else [l for l in tuning.splitlines() if "chosen" in l]}

    log(f"timed {args.steps} steps: {shots_per_s:.4g} shots/s")
    if not args.no_two_streams:
        dec2 = binding.Decoder(bcode, code.priors, B, max_iter=args.max_iter, lsd_order=args.lsd_order)
        out["two_streams"] = {"value": round(two_stream_rate(code, [dec, dec2], batches, args.steps), 1),
                              "unit": "shots/s", "note": "consecutive batches on two streams, one launch per "
                                                         "batch each; context, not the headline"}
        del dec2
    if not dem and not args.no_stream:
        log("stream leg")
        out["stream"] = stream_leg(code, bcode, args)
    if not dem and not args.no_osd:
        log("BP + OSD-0 leg")
        out["osd0"] = osd0_leg(code, bcode, batches, args, np.concatenate(ler_gpu), shots_per_s)
        log("BP + OSD-CS legs")
        out["osd_cs"] = osd_cs_leg(code, bcode, batches, args, shots_per_s)
    if not args.no_learned:
        log("learned leg")
        out["learned"] = learned_leg(code, bcode, batches, args, out["ler"]["gpu"], shots_per_s)

    if not args.no_cpu_baseline:
        log(f"cpu baseline (about {args.cpu_seconds:.0f} s)")
        out["cpu_baseline"], ler_ref = cpu_baseline(code, e0, s0.cpu().numpy(), args)
        f_gpu = ler_gpu[0][:ler_ref.size]
        Bs = ler_ref.size
        p = max(ler_ref.mean(), 1.0 / Bs)
        out["ler"].update({"gpu_batch0": round(float(f_gpu.mean()), 6),
                           "oracle_batch0": round(float(ler_ref.mean()), 6),
                           "two_sigma": round(2 * float(np.sqrt(p * (1 - p) / Bs)), 6),
                           "matched": bool(abs(f_gpu.mean() - ler_ref.mean()) <= 2 * np.sqrt(p * (1 - p) / Bs))})
    print(json.dumps(out), flush=True)


def learned_leg(code, bcode, batches, args, ler_plain, plain_shots_per_s):
    """The learned form on the same batches: BP with fewer iterations, the trained refinement of
    the shots BP leaves unsolved, then LSD; timed like the headline (K steps, inputs in HBM).
    Plain BP + LSD also runs over a grid of BP budgets and LSD orders, every point autotuned and
    timed like the learned form, for the comparison at equal logical (or word) error rate."""
    from paper_2406_18655_amd import binding
    wdir = os.path.join(HERE, "paper_2406_18655_amd", "weights")
    if args.workload == "dem":
        wname = f"dem_T{args.learned_iter}.npy"
    else:
        wname = f"bb144_p{args.p:g}_T{args.learned_iter}.npy"
        if not os.path.exists(os.path.join(wdir, wname)):
            wname = f"bb144_mix_T{args.learned_iter}.npy"
    B = args.shots
    net = binding.Net(bcode, code.priors, np.load(os.path.join(wdir, wname)))
    dec = binding.Decoder(bcode, code.priors, B, max_iter=args.learned_iter, lsd_order=args.lsd_order)
    binding.attach_net(dec, net)
    # the learned leg and every plain grid point below get the same autotuning and timing
    tuning = [l for l in dec.tune(batches[0][1], reps=3).splitlines() if "chosen" in l]
    f, rate, ms, lat = _score_and_time(code, dec, batches, args.steps, args.warmup, "learned")
    out = {"weights": wname, "bp_max_iter": args.learned_iter, "value": round(rate, 1),
           "unit": "shots/s", "ms_per_step": round(ms, 4),
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                          "p99": round(float(np.percentile(lat, 99)), 4)},
           "ler": round(float(f.mean()), 6), "ler_plain": ler_plain,
           "speedup_vs_plain": round(rate / plain_shots_per_s, 3),
           "shots_scored": int(f.size), "tuning": tuning}
    if not args.no_two_streams:
        dec2 = binding.Decoder(bcode, code.priors, B, max_iter=args.learned_iter, lsd_order=args.lsd_order)
        binding.attach_net(dec2, net)
        out["two_streams_value"] = round(two_stream_rate(code, [dec, dec2], batches, args.steps), 1)
        del dec2
    if args.no_grid:
        return out
    # plain BP + LSD over its own knobs (BP budget, LSD order mu of Sec. 4.3), on the same
    # shots: the fastest setting whose logical error rate is not above the learned form's
    # (differences within 2 sigma count as equal) is the plain decoder at matched error rate
    q, n = float(f.mean()), f.size
    grid, best = [], None
    Ts, mus = ((10, 30, 50, 100), (0, 4, 10)) if args.workload == "dem" else ((10, 20, 50), (0, 2, 4, 8, 12))
    for T in Ts:
        for mu in mus:
            # every grid point gets the autotuner and the timing of the learned leg
            d = binding.Decoder(bcode, code.priors, B, max_iter=T, lsd_order=mu)
            chosen = [l for l in d.tune(batches[0][1], reps=3).splitlines() if "chosen" in l]
            fm, rate_m, ms_m, _ = _score_and_time(code, d, batches, args.steps, args.warmup,
                                                  f"plain BP {T} LSD-{mu}")
            qm = float(fm.mean())
            two_sigma = 2 * float(np.sqrt(max(q, 1 / n) * (1 - q) / n + max(qm, 1 / n) * (1 - qm) / n))
            grid.append([T, mu, round(qm, 6), round(rate_m / 1e6, 2)])
            if qm <= q + two_sigma and (best is None or rate_m > best["value"]):
                best = {"bp_max_iter": T, "lsd_order": mu, "ler": round(qm, 6), "value": round(rate_m, 1),
                        "ler_difference_two_sigma": round(two_sigma, 6), "tuning": chosen,
                        "mcnemar": _mcnemar(f, fm)}
    out["plain_at_matched_ler"] = {
        "best": best, "speedup_of_learned": None if best is None else round(rate / best["value"], 3),
        "timing": f"every leg autotuned, {args.steps} timed steps after {args.warmup} warm-up",
        "grid": {"columns": ["bp_max_iter", "lsd_order", "ler", "M_shots_per_s"], "rows": grid}}
    return out


def _mcnemar(f_a, f_b):
    """Paired comparison on the same shots: b = failures of b only, c = failures of a only."""
    b = int(np.sum(~f_a & f_b))
    c = int(np.sum(f_a & ~f_b))
    return {"only_learned_fails": c, "only_plain_fails": b,
            "z": round((b - c) / float(np.sqrt(max(b + c, 1))), 2)}


def pipelined_latencies(dec, batches, corr, n):
    """Device time of n decode launches issued back to back (outside the timed steps), each
    bracketed by its own events: one batch's decode time with the next already queued."""
    import torch
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    torch.cuda.synchronize()
    for k in range(n):
        starts[k].record(stream)
        dec.decode_into(batches[k % len(batches)][1], corr, None)
        ends[k].record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])


def isolated_latencies(dec, batches, corr, n):
    """Device time of n decode launches, each started on an idle GPU and waited for."""
    import torch
    out = []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    for k in range(n):
        a.record(stream)
        dec.decode_into(batches[k % len(batches)][1], corr, None)
        b.record(stream)
        b.synchronize()
        out.append(a.elapsed_time(b))
    return np.array(out)


# VALU issue peak: each of a CU's 4 SIMDs finishes one 64-lane VALU instruction every 4 clocks (16
# lanes per clock), i.e. one wave-instruction per CU per clock: 256 x 2.4 GHz (the 157.3 TFLOP/s fp32
# vector figure is this rate x 64 lanes x 2 (packed) x 2 (FMA))
VALU_PEAK_WAVE_INSTR_PER_S = 256 * 2.4e9
CLOCK_HZ = 2.4e9


def issue_roofline(path, launch_ms):
    """The resources the headline kernel is bound by (its DRAM traffic is ~1 % of the algorithmic
    bytes): VALU instructions per launch against the VALU issue peak, and LDS busy cycles against
    every CU's cycles, from rocprofv3 SQ counters of the same kernel (stored with a hash of its
    sources, null when the code has changed since) over the launch duration measured here."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    if c.get("kernel_source_hash") != _kernel_hash():
        return {"stale": True, "note": "counters were taken on other kernel sources"}
    t = launch_ms * 1e-3
    cycles = t * CLOCK_HZ
    valu = c["SQ_INSTS_VALU"] / t
    lds_busy = 4.0 * c["SQ_ACTIVE_INST_LDS"] / (256 * cycles)
    valu_busy = 4.0 * c["SQ_ACTIVE_INST_VALU"] / (1024 * cycles)
    return {"bound": "lds" if lds_busy > valu_busy else "alu",
            "valu_wave_instr_per_launch": c["SQ_INSTS_VALU"],
            "valu_achieved_per_s": round(valu, 1), "valu_peak_per_s": VALU_PEAK_WAVE_INSTR_PER_S,
            "valu_issue_frac": round(valu / VALU_PEAK_WAVE_INSTR_PER_S, 4),
            "valu_busy_frac": round(valu_busy, 4),
            "lds_instr_per_launch": c["SQ_INSTS_LDS"],
            "lds_busy_frac": round(lds_busy, 4),
            "lds_bank_conflict_frac": round(c["SQ_LDS_BANK_CONFLICT"] / (256 * cycles), 4),
            "source": os.path.relpath(path, HERE), "clock_hz": CLOCK_HZ}


def record_counters(pass1, pass2, path):
    """Median per-dispatch SQ counters of the fused BP + LSD kernel from two rocprofv3 CSVs."""
    import csv
    vals = {}
    for fn in (pass1, pass2):
        rows = list(csv.DictReader(open(fn)))
        by = {}
        for r in rows:
            if "bp_lds_kernel<6, 3, true, 2, false>" not in r.get("Kernel_Name", ""):
                continue
            by.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        for k, v in by.items():
            vals[k] = float(np.median(v))
    vals["kernel_source_hash"] = _kernel_hash()
    vals["kernel"] = "bp_lds_kernel<6, 3, true, 2, false> (BP 50 + LSD-0 in one kernel)"
    with open(path, "w") as f:
        json.dump(vals, f, indent=1)
    print(json.dumps(vals))


def osd0_leg(code, bcode, batches, args, f_plain, plain_rate):
    """The comparator of Sec. 2.2: the same BP followed by global OSD-0 instead of LSD on the shots
    BP leaves unsolved, on the same batches, timed like the headline."""
    from paper_2406_18655_amd import binding
    B = batches[0][1].shape[0]
    dec = binding.Decoder(bcode, code.priors, B, max_iter=args.max_iter, flags=binding.FLAG_OSD0_POST)
    f, rate, ms, lat = _score_and_time(code, dec, batches, args.steps, args.warmup, "BP + OSD-0")
    q, qp, n = float(f.mean()), float(f_plain.mean()), f.size
    two_sigma = 2 * float(np.sqrt(max(q, 1 / n) * (1 - q) / n + max(qp, 1 / n) * (1 - qp) / n))
    return {"bp_max_iter": args.max_iter, "value": round(rate, 1), "unit": "shots/s", "ms_per_step": round(ms, 4),
            "ler": round(q, 6), "ler_bp_lsd": round(qp, 6), "ler_difference_two_sigma": round(two_sigma, 6),
            "equal_ler": bool(abs(q - qp) <= two_sigma),
            "mcnemar_vs_bp_lsd": {"only_osd_fails": int(np.sum(f & ~f_plain)),
                                  "only_lsd_fails": int(np.sum(~f & f_plain))},
            "bp_lsd_speedup": round(plain_rate / rate, 3), "shots_scored": int(n)}


def osd_cs_leg(code, bcode, batches, args, plain_rate, order=7, mu=16):
    """Higher-order post-processing on the same batches: BP followed by global OSD-CS of order
    `order` (the BP+OSD-CS comparator of Sec. 2.3 and Appendix C) against BP followed by LSD-mu
    whose local reprocessing is OSD-CS of the same order (Appendix D), both timed like the
    headline; the paired counts compare the two forms shot by shot."""
    from paper_2406_18655_amd import binding
    B = batches[0][1].shape[0]
    g = binding.Decoder(bcode, code.priors, B, max_iter=args.max_iter, flags=binding.FLAG_OSD0_POST,
                        osd_method=binding.OSD_CS, osd_order=order)
    f_g, rate_g, ms_g, _ = _score_and_time(code, g, batches, args.steps, args.warmup, f"BP + OSD-CS-{order}")
    del g
    loc = binding.Decoder(bcode, code.priors, B, max_iter=args.max_iter, lsd_order=mu, osd_method=binding.OSD_CS,
                          osd_order=order)
    f_l, rate_l, ms_l, _ = _score_and_time(code, loc, batches, args.steps, args.warmup, f"BP + LSD-{mu} CS-{order}")
    del loc
    n = f_g.size
    q_g, q_l = float(f_g.mean()), float(f_l.mean())
    two_sigma = 2 * float(np.sqrt(max(q_g, 1 / n) * (1 - q_g) / n + max(q_l, 1 / n) * (1 - q_l) / n))
    return {"order": order, "bp_max_iter": args.max_iter, "shots_scored": int(n),
            "global": {"value": round(rate_g, 1), "unit": "shots/s", "ms_per_step": round(ms_g, 4),
                       "ler": round(q_g, 6), "bp_lsd0_speedup": round(plain_rate / rate_g, 3)},
            "lsd_mu_local": {"lsd_order": mu, "value": round(rate_l, 1), "unit": "shots/s",
                             "ms_per_step": round(ms_l, 4), "ler": round(q_l, 6)},
            "ler_difference_two_sigma": round(two_sigma, 6),
            "mcnemar_local_vs_global": {"only_global_fails": int(np.sum(f_g & ~f_l)),
                                        "only_local_fails": int(np.sum(~f_g & f_l))}}


def record_traffic(fetch, write, cfetch, cwrite, path):
    """HBM bytes per launch of the fused BP + LSD kernel: the median FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) over its dispatches, each scaled by what the same counter reads for a
    plain device copy of known size (mean over the calibration copies)."""
    import csv

    def per_dispatch(fn, needle):
        v = [float(r["Counter_Value"]) for r in csv.DictReader(open(fn)) if needle in r.get("Kernel_Name", "")]
        return v

    f_k = float(np.median(per_dispatch(fetch, "bp_lds_kernel<6, 3, true, 2, false>")))
    w_k = float(np.median(per_dispatch(write, "bp_lds_kernel<6, 3, true, 2, false>")))
    # the 1 GiB copies (the calibration run's last, tiny copy returns a flag to the host)
    cf = [v for v in per_dispatch(cfetch, "copyBuffer") if v > 1024.0]
    cw = [v for v in per_dispatch(cwrite, "copyBuffer") if v > 1024.0]
    nbytes = 1 << 30
    f_fac = nbytes / 1024.0 / float(np.mean(cf))
    w_fac = nbytes / 1024.0 / float(np.mean(cw))
    rec = {"kernel": "bp_lds_kernel<6,3,true,2,false> (BP + LSD-0 in one kernel)",
           "workload": "bb144_codecap_p0.05_bp50_lsd0, 65536 shots per launch",
           "kernel_source_hash": _kernel_hash(),
           "bytes_per_launch": round(1024.0 * (f_k * f_fac + w_k * w_fac)),
           "fetch_kib_per_launch_raw": round(f_k, 2), "write_kib_per_launch_raw": round(w_k, 2),
           "copy_calibration": {"bytes": nbytes, "fetch_kib_raw": round(float(np.mean(cf)), 1),
                                "write_kib_raw": round(float(np.mean(cw)), 1),
                                "fetch_factor": round(f_fac, 4), "write_factor": round(w_fac, 4)}}
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def stream_leg(code, bcode, args):
    """Per-request latency of the decode service on the headline code: the service's maximum
    throughput (every request arriving at once), then Poisson arrivals at 50 % and 90 % of it;
    latency = completion - arrival per request, host staging and PCIe both ways included."""
    from paper_2406_18655_amd import binding
    from paper_2406_18655_amd.workloads import sample
    N = args.stream_requests
    e, S = sample(code, 2 * N, seed=args.seed + 777)

    import torch

    def run(arrivals, pool, device=False):
        srv = binding.Server(16 << 30)
        cid, lanes = srv.add_code(bcode, code.priors, batch_shots=16384, max_lanes=3, max_iter=args.max_iter)
        if device:
            pd = torch.from_numpy(np.ascontiguousarray(pool)).cuda()
            out = torch.empty((pool.shape[0], code.n), dtype=torch.uint8, device="cuda")
            srv.submit_many_device(cid, pd, out, np.arange(pool.shape[0], dtype=np.uint64), arrivals)
        else:
            out = np.zeros((pool.shape[0], code.n), dtype=np.uint8)
            srv.submit_many(cid, pool, out, np.arange(pool.shape[0], dtype=np.uint64), arrivals)
        srv.start()
        srv.wait(pool.shape[0], timeout_s=300)
        comp = srv.completions()
        srv.close()
        lat = comp["done_us"] - comp["arrival_us"]
        span = (comp["done_us"].max() - comp["arrival_us"].min()) * 1e-6
        return lat, pool.shape[0] / span, comp["batch_size"].mean()

    _, max_rate, _ = run(np.zeros(2 * N), S)
    res = {"code": "[[144,12,12]] p=0.05, BP 50 + LSD-0", "requests_per_point": N,
           "max_throughput_shots_per_s": round(max_rate, 1), "points": []}
    rng = np.random.default_rng(args.seed)
    for frac in (0.5, 0.9):
        rate = frac * max_rate
        arr = np.cumsum(rng.exponential(1e6 / rate, size=N))
        lat, thr, mb = run(arr, S[:N])
        res["points"].append({"offered_frac_of_max": frac, "offered_shots_per_s": round(rate, 1),
                              "served_shots_per_s": round(thr, 1),
                              "p50_us": round(float(np.percentile(lat, 50)), 1),
                              "p99_us": round(float(np.percentile(lat, 99)), 1),
                              "mean_batch": round(float(mb), 1)})
    res["latency_includes"] = "host staging, PCIe copies both ways, scheduler polling"
    # device-resident requests (syndromes and corrections stay in HBM): no staging, no PCIe
    _, max_dev, _ = run(np.zeros(2 * N), S, device=True)
    dev = {"max_throughput_shots_per_s": round(max_dev, 1), "points": []}
    for frac in (0.5, 0.9):
        rate = frac * max_dev
        arr = np.cumsum(rng.exponential(1e6 / rate, size=N))
        lat, thr, mb = run(arr, S[:N], device=True)
        dev["points"].append({"offered_frac_of_max": frac, "offered_shots_per_s": round(rate, 1),
                              "served_shots_per_s": round(thr, 1),
                              "p50_us": round(float(np.percentile(lat, 50)), 1),
                              "p99_us": round(float(np.percentile(lat, 99)), 1),
                              "mean_batch": round(float(mb), 1)})
    res["device_resident"] = dev
    return res


_STREAMS = []


def two_stream_rate(code, decs, batches, steps):
    """Whole-job shots/s with consecutive batches on two streams, one decoder (and one launch per
    batch) each: a launch's BP ramp and LSD tail overlap the next launch.  Context only.  The
    streams are created once: HIP spreads new streams over its hardware queues in turn, and two
    streams that share a queue run their kernels one after the other."""
    import torch
    B = batches[0][1].shape[0]
    while len(_STREAMS) < len(decs):
        _STREAMS.append(torch.cuda.Stream())
    streams = _STREAMS[:len(decs)]
    outs = [torch.empty((B, code.n), dtype=torch.uint8, device="cuda") for _ in decs]
    def run(k0, n):
        for k in range(k0, k0 + n):
            i = k % len(decs)
            with torch.cuda.stream(streams[i]):
                decs[i].decode_into(batches[k % len(batches)][1], outs[i], None)
    run(0, 2 * len(decs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(0, steps)
    torch.cuda.synchronize()
    return steps * B / (time.perf_counter() - t0)


def _score_and_time(code, dec, batches, steps, warmup, label):
    """Logical failures of `dec` on every batch (untimed, each correction checked against its
    syndrome), then `steps` timed decodes of the batches in turn with the inputs in HBM."""
    import torch
    from paper_2406_18655_amd.workloads import logical_failures, syndromes
    B = batches[0][1].shape[0]
    corr = torch.empty((B, code.n), dtype=torch.uint8, device="cuda")
    fails = []
    for e, s in batches:
        dec.decode_into(s, corr, None)
        c = corr.cpu().numpy()
        if not (syndromes(code, c) == s.cpu().numpy()).all():
            print(f"{label}: correction does not satisfy its syndrome", file=sys.stderr)
            sys.exit(3)
        fails.append(logical_failures(code, e, c))
    for k in range(warmup):
        dec.decode_into(batches[k % len(batches)][1], corr, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        dec.decode_into(batches[k % len(batches)][1], corr, None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = pipelined_latencies(dec, batches, corr, steps)
    return np.concatenate(fails), steps * B / wall, wall * 1e3 / steps, lat


def _kernel_hash(root=None):
    """Hash of the fused kernel's sources with comments and whitespace removed: the stored HBM
    traffic stays valid across comment-only edits and is dropped when the code changes."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("qlsd_bp.hip", "qlsd_internal.h", "qlsd_lsd_dev.h"):
        with open(os.path.join(root or HERE, "paper_2406_18655_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update("".join(text.split()).encode())
    return h.hexdigest()[:16]


def cpu_baseline(code, errors, S, args):
    """The CPU oracle (float64 BP + LSD, OpenMP over shots) on batch 0, as it stands."""
    import oracle
    from paper_2406_18655_amd.workloads import logical_failures
    oc = oracle.Code.from_dense(code.H)
    lam = oracle.llr_from_priors(code.priors)
    host = host_cpu()
    # one worker per physical core available to this process, within the CPU share the GPU host
    # gives one GPU (OMP_NUM_THREADS there)
    threads = min(x for x in (host["physical_cores"], host["available_cpus"],
                              int(os.environ.get("OMP_NUM_THREADS", "0")) or None) if x)
    mu = args.lsd_order
    omega = oracle.omega_from_llr(lam) if mu > 0 else None
    if args.workload == "dem":  # the float64 oracle takes ~ms per DEM shot: a bounded sample
        S, errors = S[:2048], errors[:2048]
    # one full pass over the sample gives the oracle's LER on the same shots
    t0 = time.perf_counter()
    corr, st, it, _ = oracle.decode_batch(oc, lam, S, args.max_iter, mu=mu, omega=omega, nthreads=threads)
    dt = time.perf_counter() - t0
    done, tot = S.shape[0], dt
    while tot < args.cpu_seconds:
        t0 = time.perf_counter()
        oracle.decode_batch(oc, lam, S, args.max_iter, mu=mu, omega=omega, nthreads=threads)
        tot += time.perf_counter() - t0
        done += S.shape[0]
    ler_ref = logical_failures(code, errors, corr)
    # single-thread rate on a slice of the same sample (about 3 s)
    k = max(1, min(S.shape[0], int(3.0 * S.shape[0] / (dt * threads))))
    t0 = time.perf_counter()
    oracle.decode_batch(oc, lam, S[:k], args.max_iter, mu=mu, omega=omega, nthreads=1)
    one = k / (time.perf_counter() - t0)
    base = {"value": round(done / tot, 1), "unit": "shots/s", "cores": threads, "kind": "oracle",
            "sample": f"first {S.shape[0]} shots of batch 0 decoded {done // S.shape[0]}x, {tot:.1f} s",
            "single_thread_value": round(one, 1), "host": host}
    return base, ler_ref


def host_cpu():
    """CPU model and counts of the host this runs on (from /proc/cpuinfo and the affinity mask)."""
    model, cores, cur = None, set(), {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    cur["p"] = v
                elif k == "core id":
                    cores.add((cur.get("p"), v))
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"model": model, "physical_cores": len(cores) or None, "logical_cpus": os.cpu_count(),
            "available_cpus": avail, "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def serve_main(args):
    """Continuous-batching service over HGP(3,4) n=16/24/32, the BB code and the synthetic DEM
    (uniform mix), Poisson arrivals at each rate; latency = completion - arrival per request."""
    if args.serve_hw_queues > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.serve_hw_queues)  # read when HIP initialises below
    import torch
    from paper_2406_18655_amd import binding
    from paper_2406_18655_amd.workloads import bivariate_bicycle, random_34_hgp, synthetic_dem, sample
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    mix = [("hgp34_n16", random_34_hgp(16, p=0.03), 30, 0, 4096),
           ("hgp34_n24", random_34_hgp(24, p=0.03), 30, 0, 2048),
           ("hgp34_n32", random_34_hgp(32, p=0.03), 30, 0, 1024),
           ("bb144", bivariate_bicycle(p=0.05), 50, 0, 4096),
           ("dem936x8800", synthetic_dem(), 100, 10, 512)]
    from paper_2406_18655_amd.binding import DeviceSampler
    per_code = args.serve_requests // len(mix)
    pools = []
    for k, (name, code, T, mu, bs) in enumerate(mix):  # request syndromes, drawn on the GPU, held on the host
        e, S = DeviceSampler(code).sample(per_code, args.seed + 100 + k)
        pools.append(S.cpu().numpy())
        del e, S
    torch.cuda.synchronize()
    print(f"[serve] {per_code} requests per code sampled", file=sys.stderr, flush=True)
    wdir = os.path.join(HERE, "paper_2406_18655_amd", "weights")
    learned_lanes = {"bb144": (10, "bb144_mix_T10.npy"), "dem936x8800": (30, "dem_T30.npy")}
    for ordering, rate in [(o, float(x)) for o in args.serve_ordering.split(",") for x in args.serve_rates.split(",")]:
        rng = np.random.default_rng(args.seed)
        srv = binding.Server(64 << 30)
        outs, cids = [], []
        for k, (name, code, T, mu, bs) in enumerate(mix):
            bc = binding.Code.from_dense(code.H)
            learned = ordering == "learned" and name in learned_lanes
            cid, lanes = srv.add_code(bc, code.priors, batch_shots=bs, max_lanes=3,
                                      max_iter=learned_lanes[name][0] if learned else T, lsd_order=mu)
            if learned:
                srv.set_net(cid, binding.Net(bc, code.priors, np.load(os.path.join(wdir, learned_lanes[name][1]))))
            arr = np.cumsum(rng.exponential(1e6 / (rate / len(mix)), size=per_code))
            out = np.zeros((per_code, code.n), dtype=np.uint8)
            srv.submit_many(cid, pools[k], out, np.arange(per_code, dtype=np.uint64), arr)
            outs.append(out)
            cids.append(cid)
        total = per_code * len(mix)
        srv.start()
        srv.wait(total, timeout_s=600)
        comp = srv.completions()
        srv.close()
        lat = comp["done_us"] - comp["arrival_us"]
        span_s = (comp["done_us"].max() - comp["arrival_us"].min()) * 1e-6
        codes = {}
        for k, (name, *_r) in enumerate(mix):
            sel = comp["code_id"] == cids[k]
            codes[name] = {"p50_us": round(float(np.percentile(lat[sel], 50)), 1),
                           "p99_us": round(float(np.percentile(lat[sel], 99)), 1),
                           "mean_batch": round(float(comp["batch_size"][sel].mean()), 1)}
        print(json.dumps({"metric": "streaming decode latency over a mixed-code Poisson load",
                          "offered_shots_per_s": rate, "requests": int(total),
                          "throughput_shots_per_s": round(total / span_s, 1),
                          "p50_us": round(float(np.percentile(lat, 50)), 1),
                          "p99_us": round(float(np.percentile(lat, 99)), 1),
                          "per_code": codes,
                          "ordering": "plain BP+LSD" if ordering == "plain" else
                                      "[[144,12,12]]: BP 10 + learned refinement + LSD; DEM: BP 30 + learned "
                                      "refinement + LSD-10; others plain",
                          "latency_includes": "host staging, PCIe copies, scheduler polling"}), flush=True)


def sweep_main(args):
    """Logical error rate and throughput of plain BP (50) + LSD-0 and of the learned form across
    the code-capacity noise sweep; inputs resident in HBM during the timed decodes."""
    import torch
    import oracle
    from paper_2406_18655_amd import binding
    from paper_2406_18655_amd.workloads import bivariate_bicycle, sample, logical_failures, syndromes
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    sizes = [65536] * 15 + [16960]
    w = np.load(os.path.join(HERE, "paper_2406_18655_amd", "weights", "bb144_mix_T10.npy"))
    for p in (0.01, 0.02, 0.04, 0.05, 0.06):
        code = bivariate_bicycle(p=p)
        bc = binding.Code.from_dense(code.H)
        plain = binding.Decoder(bc, code.priors, 65536, max_iter=50)
        learned = binding.Decoder(bc, code.priors, 65536, max_iter=10)
        net = binding.Net(bc, code.priors, w)
        binding.attach_net(learned, net)
        res = {}
        e0 = s0 = None
        for name, dec in (("plain", plain), ("learned", learned)):
            fails, ms, start = 0, 0.0, 0
            for k, B in enumerate(sizes):
                e, S = sample(code, B, seed=args.seed + 1000 * int(round(p * 100)), start=start)
                start += B
                s = torch.from_numpy(S).cuda()
                out = torch.empty((B, code.n), dtype=torch.uint8, device="cuda")
                dec.decode_into(s, out)  # warm
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                dec.decode_into(s, out)
                b.record()
                torch.cuda.synchronize()
                ms += a.elapsed_time(b)
                c = out.cpu().numpy()
                if not (syndromes(code, c) == S).all():
                    print("correction does not satisfy its syndrome", file=sys.stderr)
                    sys.exit(3)
                f = logical_failures(code, e, c)
                fails += int(f.sum())
                if k == 0 and name == "plain":
                    e0, s0, f0 = e, S, f
            n = sum(sizes)
            q = fails / n
            res[name] = {"ler": q, "sigma": float(np.sqrt(max(q, 1 / n) * (1 - q) / n)),
                         "shots_per_s": round(n / (ms * 1e-3), 1)}
        oc = oracle.Code.from_dense(code.H)
        corr, st, it, _ = oracle.decode_batch(oc, oracle.llr_from_priors(code.priors), s0, 50,
                                              nthreads=min(16, os.cpu_count() or 1))
        fo = logical_failures(code, e0, corr)
        q = max(fo.mean(), 1 / fo.size)
        two_sigma = 2 * float(np.sqrt(q * (1 - q) / fo.size))
        print(json.dumps({"workload": "bb144_codecap_sweep_bp50_lsd0", "p": p, "shots": sum(sizes), **res,
                          "oracle_first_launch": {"shots": int(fo.size), "ler_oracle": float(fo.mean()),
                                                  "ler_gpu": float(f0.mean()), "two_sigma": two_sigma,
                                                  "matched": bool(abs(f0.mean() - fo.mean()) <= two_sigma)},
                          "learned_weights": "bb144_mix_T10.npy"}), flush=True)


def window_main(args):
    """Multi-round decoding: the 12-round memory DEM of the headline code (936 detectors, 2736
    faults) decoded by the (w=3, c=1) overlapping-window scheme and, for comparison, as one
    12-round history; shots drawn by the library's sampler, inputs in HBM while timed."""
    import torch
    from paper_2406_18655_amd import binding
    from paper_2406_18655_amd.workloads import bivariate_bicycle, round_dem
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    cycles, B, reps = 12, 16384, 8
    for p in (0.01, 0.02, 0.025, 0.03):
        dem = round_dem(bivariate_bicycle(p=p), cycles, p, p)
        bc = binding.Code.from_dense(dem.H)
        ds = binding.DeviceSampler(dem)
        legs = {"window_3_1": binding.WindowDecoder(bc, dem.priors, dem.det_round, 3, 1, B, max_iter=30),
                "full_history": binding.Decoder(bc, dem.priors, B, max_iter=30)}
        res = {}
        for name, dec in legs.items():
            fails, ms = 0, 0.0
            out = torch.empty((B, dem.n), dtype=torch.uint8, device="cuda")
            for r in range(reps):
                e, s = ds.sample(B, args.seed + 31 * r)
                dec.decode_into(s, out)  # warm
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                dec.decode_into(s, out)
                b.record()
                torch.cuda.synchronize()
                ms += a.elapsed_time(b)
                if not torch.equal(ds.syndromes(out), s):
                    print(f"{name}: correction does not satisfy its syndrome", file=sys.stderr)
                    sys.exit(3)
                fails += int(ds.failures(e, out).sum().item())
            n = reps * B
            q = fails / n
            res[name] = {"ler_total": q, "sigma": float(np.sqrt(max(q, 1 / n) * (1 - q) / n)),
                         "per_cycle": 1.0 - (1.0 - q) ** (1.0 / cycles),
                         "shots_per_s": round(n / (ms * 1e-3), 1)}
        print(json.dumps({"workload": f"bb144_memory_{cycles}rounds_phenomenological", "p": p,
                          "H": f"{dem.m}x{dem.n}", "shots": reps * B, "bp_max_iter": 30, "lsd_order": 0,
                          "windows": legs["window_3_1"].windows, **res}), flush=True)


def cluster_stats_main(args):
    """Distributions of nu (clusters per shot), kappa (largest cluster) and kappa_alpha (size-
    weighted mean cluster size) for LSD's final clusters and for the optimal factorization
    (connected components of the true error in the fault graph), both on the shots BP does not
    solve, plus the optimal factorization over all shots; Bethe-lattice estimates for the fault-
    graph degree theta (the two forms the paper prints, Appendices A and B)."""
    import torch
    from paper_2406_18655_amd import binding
    from paper_2406_18655_amd.workloads import bivariate_bicycle, synthetic_dem
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)

    def dist(x):
        x = np.asarray(x, dtype=np.float64)
        if x.size == 0:
            return None
        return {"mean": round(float(x.mean()), 4), "p50": float(np.percentile(x, 50)),
                "p90": float(np.percentile(x, 90)), "p99": float(np.percentile(x, 99)), "max": float(x.max())}

    def summary(st):
        st = st.astype(np.float64)
        ka = np.where(st[:, 2] > 0, st[:, 3] / np.maximum(st[:, 2], 1), 0.0)
        return {"nu": dist(st[:, 0]), "kappa": dist(st[:, 1]), "kappa_alpha": dist(ka)}

    cases = [("bb144", bivariate_bicycle(p=p), p, 0) for p in (0.01, 0.02, 0.04, 0.05, 0.06)]
    cases.append(("dem936x8800", synthetic_dem(), None, 10))
    for name, code, p, mu in cases:
        B = 65536 if name == "dem936x8800" else 262144
        bc = binding.Code.from_dense(code.H)
        ds = binding.DeviceSampler(code)
        e, s = ds.sample(B, args.seed + 4242)
        dec = binding.Decoder(bc, code.priors, B, max_iter=30, lsd_order=mu)
        llr, hard, info = dec.bp(s)
        torch.cuda.synchronize()
        fail = np.nonzero((binding.parse_info(info)["status"] & 1) == 0)[0]
        idx = torch.from_numpy(fail).cuda()
        _, _, st = dec.lsd_stats(s[idx].contiguous(), llr[idx].contiguous())
        opt = binding.error_clusters(bc, e)
        torch.cuda.synchronize()
        st, opt = st.cpu().numpy(), opt.cpu().numpy()
        F = (code.H.T.astype(np.int64) @ code.H.astype(np.int64)) > 0
        np.fill_diagonal(F, False)
        deg = F.sum(1)
        theta = float(deg.max())
        pbar = float(code.priors.mean())
        bethe = {"theta": theta, "theta_mean": round(float(deg.mean()), 2), "p": pbar,
                 "appendix_A": round(pbar / (1 - pbar * (theta - 1)), 5) if pbar * (theta - 1) < 1 else None,
                 "appendix_B": round((1 + pbar) / (1 - (theta - 1) * pbar), 5) if pbar * (theta - 1) < 1 else None}
        print(json.dumps({"workload": name, "p": p, "shots": B, "bp_max_iter": 30, "lsd_order": mu,
                          "bp_failures": int(len(fail)),
                          "lsd": summary(st), "optimal_on_bp_failures": summary(opt[fail]),
                          "optimal_all_shots": summary(opt[opt[:, 2] > 0]), "bethe": bethe}), flush=True)


def copy_calibration(nbytes):
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give the factor that turns
    the decoder kernels' counter readings into bytes."""
    import torch
    x = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3, "equal": bool(torch.equal(x, y))}), flush=True)


if __name__ == "__main__":
    _a = parse()
    if _a.record_counters:
        record_counters(_a.record_counters[0], _a.record_counters[1], _a.counters_json)
    elif _a.record_traffic:
        record_traffic(*_a.record_traffic, _a.traffic_json)
    elif _a.cluster_stats:
        cluster_stats_main(_a)
    elif _a.window:
        window_main(_a)
    elif _a.copy_calibration:
        copy_calibration(_a.copy_calibration)
    elif _a.sweep:
        sweep_main(_a)
    elif _a.serve:
        serve_main(_a)
    else:
        main()
