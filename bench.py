"""Benchmark: ms per boosting round of Viola-Jones AdaBoost on one MI355X.

Workload (default): 5,000 + 10,000 synthetic 24x24 windows (seeded stand-in for
the face / non-face training set), all 162,336 Haar features, FP32 weights
with FP64 accumulation in the scan.  A step is one boosting round: the scan
of every feature's sorted keys against the current weights, the argmin over
features, the threshold, beta / alpha and the weight update.  The one-time
preparation (integral images, feature values, per-feature sort) runs before
the timed region and is reported separately as init_ms.

The scan's launch schedule is the one measured fastest at init (--schedule -1,
the default) or a fixed one.  Beside the round time the line carries the
scan's HBM roofline (algorithmic key bytes over its live-measured device
time, and the copy-calibrated rocprofv3 traffic when it was taken on the same
code and schedule), a stream probe (the same key reads with no arithmetic),
the same workload in the other precision modes (FP32 weights with
compensated FP32 sums, FP64, plain FP32; per-kernel device times over 50
rounds), the batched-jobs measurement (32 uneven jobs by default,
jobs*rounds/s, against the same jobs run one at a time through the
single-job path) and the FP64 oracle's round time on the host cores over 20
of the 200 rounds.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "ms per boosting round (162k Haar × 15k imgs); batched jobs·rounds/s vs plain"
def profiled_traffic(kind: str, precision: str, schedule: int):
    """HBM bytes per scan launch from the committed rocprofv3 counter summary,
    or None when it is missing or was taken on a different scan source,
    precision or schedule."""
    from paper_1306_1467_amd.profsum import scan_source_hash
    path = os.path.join(ROOT, "profiles", f"stump_scan_{kind}_counters.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("scan_source_hash") != scan_source_hash() or d.get("precision") != precision:
        return None
    return d.get("schedules", {}).get(str(schedule), {}).get("bytes_per_launch")


def cpu_baseline(images, labels, n_features: int, rounds: int, rounds_1t: int):
    """The FP64 oracle's round time on the host cores: `rounds` rounds with
    every host thread and `rounds_1t` rounds with one thread, over the first
    `n_features` features (0: all) of the same windows."""
    import numpy as np
    import oracle
    F = oracle.feature_count(24, 24)
    feats = oracle.enumerate_features(24, 24)
    nf = F if n_features <= 0 or n_features >= F else n_features
    pick = np.arange(F) if nf == F else np.sort(np.random.default_rng(0).choice(F, nf, replace=False))
    threads = oracle.max_threads()
    t_prep = time.perf_counter()
    ii = oracle.integrals(images, threads)
    vals = oracle.feature_values(ii, feats[pick], threads)
    order = oracle.sort_features(vals, threads)
    t_prep = time.perf_counter() - t_prep
    w = oracle.init_weights(labels)
    scratch = np.zeros(nf, oracle.STUMP_DTYPE)
    oracle.boost_round(vals, order, labels, w, 1e-10, threads, scratch)   # warm caches
    t0 = time.perf_counter()
    for _ in range(rounds):
        oracle.boost_round(vals, order, labels, w, 1e-10, threads, scratch)
    dt = (time.perf_counter() - t0) / rounds
    t0 = time.perf_counter()
    for _ in range(rounds_1t):
        oracle.boost_round(vals, order, labels, w, 1e-10, 1, scratch)
    dt1 = (time.perf_counter() - t0) / max(rounds_1t, 1)
    scale = F / nf
    what = "all" if nf == F else f"{nf:,} sampled"
    return {"value": round(dt * 1e3 * scale, 2), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"{rounds} oracle rounds over {what} of {F:,} features x {len(labels):,} windows"
                      + ("" if nf == F else f", scaled by {scale:.3f}")
                      + " (one-time value/sort preparation excluded)",
            "one_thread_ms": round(dt1 * 1e3 * scale, 1), "one_thread_rounds": rounds_1t,
            "prep_s": round(t_prep * scale, 2), "host_cpu": _cpu_model(), "host_threads": os.cpu_count()}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_single(args, torch, vb, synth):
    spec = synth.workload_jobs("faces15k")[0]
    images, labels = spec.make()
    vb.boost_tune_cache_clear()
    t0 = time.perf_counter()
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=args.precision,
                    schedule_id=args.schedule)
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t0) * 1e3
    # the schedule in use (under the measured choice: the tuner's pick, timed during init)
    schedule, tune_ms = tr.schedule()
    tuning = {"requested": args.schedule, "chosen": schedule,
              "best_scan_ms_by_schedule": {str(k): round(m, 4) for k, m in enumerate(tune_ms) if m > 0}}
    F, n = tr.F, tr.n
    if args.warmup:
        vb.boost_train(tr.ctx, args.warmup, False)
    tr.stream.synchronize()
    # timed region: K rounds replayed from the captured HIP graph; HIP events on
    # the library's stream bracket the region
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(tr.stream):
        ev0.record()
    vb.boost_train(tr.ctx, args.steps, False)
    with torch.cuda.stream(tr.stream):
        ev1.record()
    tr.stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    graph_ms = ev0.elapsed_time(ev1) / args.steps
    # per-round distribution (outside the timed region): HIP events around
    # each single-round graph launch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    with torch.cuda.stream(tr.stream):
        evs[0].record()
    for r in range(args.steps):
        vb.boost_train(tr.ctx, 1, False)
        with torch.cuda.stream(tr.stream):
            evs[r + 1].record()
    tr.stream.synchronize()
    per_round = sorted(evs[r].elapsed_time(evs[r + 1]) for r in range(args.steps))
    pct = lambda q: per_round[min(len(per_round) - 1, int(q * len(per_round)))]
    rec = tr.round()
    # the strong classifier of 200 stumps on the training windows (outside the timed region)
    stumps = tr.train(200)
    tr.classify(stumps)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(tr.stream):
        c0.record()
    for _ in range(5):
        tr.classify(stumps)
    with torch.cuda.stream(tr.stream):
        c1.record()
    tr.stream.synchronize()
    classify_ms = c0.elapsed_time(c1) / 5
    correct = int((tr.classify(stumps)[0].cpu().numpy() == labels).sum())
    tr.close()
    # per-kernel device times: the same rounds with HIP events around each
    # kernel on the library's stream (direct launches)
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=args.precision,
                    schedule_id=schedule, flags=vb.BOOST_FLAG_TIMING)
    if args.warmup:
        vb.boost_train(tr.ctx, args.warmup, False)
    vb.boost_reset_timing(tr.ctx)
    t1 = time.perf_counter()
    vb.boost_train(tr.ctx, args.steps, False)
    tr.stream.synchronize()
    timed_ms = (time.perf_counter() - t1) * 1e3 / args.steps
    scan_ms, upd_ms, nr, _ = vb.boost_get_timing(tr.ctx)
    probe_ms = vb.boost_probe_stream(tr.ctx, 10)   # the same key reads with no arithmetic
    tr.close()
    scan_avg = scan_ms / nr
    alg_bytes = F * n * 2
    achieved = alg_bytes / (scan_avg * 1e-3) / 1e9
    traffic = profiled_traffic("faces15k", args.precision, schedule)
    out = {
        "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
        "graph_event_ms_per_round": round(graph_ms, 4),
        "round_ms_p10_p50_p90": [round(pct(0.1), 4), round(pct(0.5), 4), round(pct(0.9), 4)],
        "event_instrumented_ms_per_round": round(timed_ms, 4),
        "init_ms": round(init_ms, 1),
        "scan_ms_avg": round(scan_avg, 4),
        "update_ms_avg": round(upd_ms / nr, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                                         "copy-calibrated)",
                     "traffic_GBps": None if traffic is None else round(traffic / (scan_avg * 1e-3) / 1e9, 1),
                     "kernel": f"k_scan (schedule {schedule})", "alg_bytes_per_launch": alg_bytes},
        "last_round": {"feature": int(rec.feature), "error_raw": rec.error_raw, "polarity": int(rec.polarity),
                       "threshold": int(rec.threshold)},
        "strong_classifier": {"stumps": 200, "windows": n, "ms": round(classify_ms, 4),
                              "training_accuracy": round(correct / n, 4)},
        "stream_probe": {"ms": round(probe_ms, 4), "key_GBps": round(alg_bytes / (probe_ms * 1e-3) / 1e9, 1),
                         "scan_time_over_probe": round(probe_ms / scan_avg, 4)},
        "schedule_tuning": tuning, "schedule": schedule,
        "F": F, "n": n,
    }
    return out, images, labels


def run_precision_sweep(args, torch, vb, images, labels, F: int, n: int):
    """The same workload in the other precision modes: per-kernel device
    times (HIP events around each kernel, direct launches) over a few rounds,
    each under the measured schedule choice."""
    out = {}
    modes = [m for m in args.sweep_precisions.split(",") if m and m != args.precision]
    for prec in modes:
        tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=prec,
                        schedule_id=vb.BOOST_SCHEDULE_AUTO, flags=vb.BOOST_FLAG_TIMING)
        schedule, _ = tr.schedule()
        vb.boost_train(tr.ctx, 3, False)
        vb.boost_reset_timing(tr.ctx)
        recs = vb.boost_train(tr.ctx, args.sweep_rounds, True)
        tr.stream.synchronize()
        scan_ms, upd_ms, nr, _ = vb.boost_get_timing(tr.ctx)
        tr.close()
        del tr
        scan_avg = scan_ms / nr
        out[prec] = {"schedule": schedule, "rounds": nr, "scan_ms_avg": round(scan_avg, 4),
                     "update_ms_avg": round(upd_ms / nr, 4), "ms_per_round": round((scan_ms + upd_ms) / nr, 4),
                     "scan_hbm_frac": round(F * n * 2 / (scan_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "last_error_raw": float(recs[-1]["error_raw"])}
    return out


def run_batched(name, args, torch, vb, synth):
    """Jobs of a batched workload trained together (one scan + one update
    launch per round for all jobs) against the same jobs trained one at a
    time through the single-job path, same precision and schedule."""
    import numpy as np
    specs = synth.workload_jobs(name)
    data = [s.make() for s in specs]
    rounds = args.batch_rounds or specs[0].rounds
    prec = args.batch_precision
    # plain: each job alone; one untimed round first (graph capture), as below
    t_plain = 0.0
    plain = []
    for images, labels in data:
        tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=prec,
                        schedule_id=args.batch_schedule)
        vb.boost_train(tr.ctx, 1, False)
        tr.stream.synchronize()
        t0 = time.perf_counter()
        plain.append(vb.boost_train(tr.ctx, rounds, True))
        t_plain += time.perf_counter() - t0
        tr.close()
        del tr
        torch.cuda.empty_cache()
    t0 = time.perf_counter()
    bt = vb.BatchTrainer([(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data], precision=prec,
                         schedule_id=args.batch_schedule)
    bt.sync()
    init_s = time.perf_counter() - t0
    bt.train(1, False)
    bt.sync()
    t0 = time.perf_counter()
    recs = bt.train(rounds, True)
    t_batch = time.perf_counter() - t0
    same = all(recs[:, k].tobytes() == plain[k].tobytes() for k in range(len(data)))
    chosen = bt.schedule()
    keys = sum(vb.boost_feature_count(vb.feature_set(s.size)) * s.n for s in specs)
    jr = len(data) * rounds
    bt.close()
    del bt
    torch.cuda.empty_cache()
    sizes = sorted({s.size for s in specs})
    return {"workload": f"{len(data)} jobs, " + "/".join(f"{z}x{z}" for z in sizes) + " windows"
                        + f", {min(s.n for s in specs):,}-{max(s.n for s in specs):,} windows per job",
            "jobs": len(data), "rounds": rounds, "precision": prec, "keys_per_round": keys,
            "batched_jobs_rounds_per_s": round(jr / t_batch, 2),
            "plain_jobs_rounds_per_s": round(jr / t_plain, 2),
            "speedup_vs_plain": round(t_plain / t_batch, 3),
            "batched_ms_per_round": round(t_batch * 1e3 / rounds, 3),
            "batched_key_GBps": round(keys * 2 * rounds / t_batch / 1e9, 1),
            "batched_init_s": round(init_s, 2),
            "schedule": {"requested": args.batch_schedule,
                         "key14": {"schedule": chosen[0][0], "segs_per_wg": chosen[0][1]},
                         "key15": {"schedule": chosen[1][0], "segs_per_wg": chosen[1][1]}},
            "stumps_identical_to_plain": bool(same)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp32_wide")
    ap.add_argument("--schedule", type=int, default=-1,
                    help="scan launch schedule of the single-job workload (-1: measured choice at init)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-features", type=int, default=0, help="oracle features (0: all)")
    ap.add_argument("--cpu-rounds", type=int, default=20)
    ap.add_argument("--cpu-rounds-1t", type=int, default=1)
    ap.add_argument("--sweep-precisions", default="fp32_kahan,fp64,fp32",
                    help="other precision modes timed on the same workload (empty: none)")
    ap.add_argument("--sweep-rounds", type=int, default=50)
    ap.add_argument("--batched", default="batch32",
                    help="comma list of batched workloads to measure (batch32: 32 uneven jobs of 24x24 windows, "
                         "batch64: 64 jobs of 16-28 px windows); empty for none")
    ap.add_argument("--batch-rounds", type=int, default=0, help="rounds per batched job (0: the workload's own)")
    ap.add_argument("--batch-precision", default="fp32_wide")
    ap.add_argument("--batch-schedule", type=int, default=-1,
                    help="schedule of the batched and the plain per-job runs (-1: measured choice at init)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="run one device copy of this many GiB first (counter calibration)")
    ap.add_argument("--prep-only", action="store_true",
                    help="only the one-time preparation of the headline workload (fixed schedule 0, no tuning), "
                         "then exit: the run a profile of the preparation kernels needs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: vjboost runs on one GPU only; multi-GPU runs are not supported "
              "(the path would shard features across GPUs: each scans its share and one all-reduce-min "
              "picks the stump)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1306_1467_amd import synth
    from paper_1306_1467_amd import vjboost as vb
    vb.lib()
    if args.copy_calibration_gib > 0:
        nb = int(args.copy_calibration_gib * 2 ** 30)
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.prep_only:
        images, labels = synth.workload_jobs("faces15k")[0].make()
        t0 = time.perf_counter()
        tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=args.precision, schedule_id=0)
        torch.cuda.synchronize()
        print(json.dumps({"prep_only": True, "init_ms": round((time.perf_counter() - t0) * 1e3, 1),
                          "features": tr.F, "windows": tr.n}), flush=True)
        tr.close()
        return
    res, images, labels = run_single(args, torch, vb, synth)
    line = {
        "metric": METRIC,
        "value": res["ms_per_step"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32_wide": "f32 weights, f64 accumulation", "fp32_kahan": "f32 two-sum",
                  "fp32": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "162,336 Haar features x 15,000 windows 24x24 (5,000 pos + 10,000 neg), "
                               "one boosting round per step", "precision": args.precision,
                   "schedule": res["schedule"], "schedule_requested": args.schedule, "features": res["F"],
                   "windows": res["n"]},
        "init_ms": res["init_ms"],
        "graph_event_ms_per_round": res["graph_event_ms_per_round"],
        "round_ms_p10_p50_p90": res["round_ms_p10_p50_p90"],
        "event_instrumented_ms_per_round": res["event_instrumented_ms_per_round"],
        "scan_ms_avg": res["scan_ms_avg"],
        "update_ms_avg": res["update_ms_avg"],
        "roofline": res["roofline"],
        "last_round": res["last_round"],
        "stream_probe": res["stream_probe"],
        "strong_classifier": res["strong_classifier"],
        "schedule_tuning": res["schedule_tuning"],
    }
    if args.sweep_precisions:
        line["precision_sweep"] = run_precision_sweep(args, torch, vb, images, labels, res["F"], res["n"])
    for name in [c.strip() for c in args.batched.split(",") if c.strip()]:
        line[f"batched_{name}"] = run_batched(name, args, torch, vb, synth)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(images, labels, args.cpu_features, args.cpu_rounds, args.cpu_rounds_1t)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
