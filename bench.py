"""Benchmark: ms per boosting round of Viola-Jones AdaBoost on one MI355X.

Headline workload: 5,000 + 10,000 synthetic 24x24 windows (a seeded stand-in
for the face / non-face training set), all 162,336 Haar features, FP32
weights scanned with compensated (Kahan-style) FP32 prefix sums -- the
precision the headline configuration names.  A step is one boosting round:
the scan of every feature's sorted keys against the current weights, the
argmin over features, the threshold, beta / alpha and the FP64 weight
update.  The one-time preparation (integral images, feature values,
per-feature sort) runs before the timed region and is reported separately
(init_ms, tuned and with the tuning cache warm).

Beside the round time the line carries:
  roofline         the headline scan kernel's algorithmic key bytes over its
                   live-measured device time against 8 TB/s, and the
                   copy-calibrated rocprofv3 HBM traffic when a counter record
                   of the same scan code, precision and schedule is committed;
  variants         the same workload with FP32 weights accumulated in FP64
                   (the library's exact mode), with its own roofline;
  precision_sweep  the FP64 and plain FP32 modes (per-kernel device times);
  precision_report every mode against the FP64 oracle over K teacher-forced
                   full-size rounds (every feature, both polarities), on the
                   headline data and on a non-separable set;
  batched_*        32 uneven jobs (batch32) and 64 mixed-window jobs (batch64,
                   in the compensated and the FP64-accumulated modes):
                   jobs*rounds/s against the same jobs run one at a time;
  cpu_baseline*    the FP64 oracle timed on the host cores: the headline round
                   over all features, and bounded samples of both batched
                   workloads;
  strong_classifier  training and held-out error of the 200-stump classifier.
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
DTYPE = {"fp32_kahan": "f32", "fp32_wide": "f32 weights, f64 sums", "fp32": "f32", "fp64": "f64"}
PRECISION_NAME = {"fp32_kahan": "FP32 weights, compensated FP32 prefix sums (Fast2Sum), FP64 candidates",
                  "fp32_wide": "FP32 weights accumulated in FP64 (exact sums)",
                  "fp64": "FP64 weights and sums", "fp32": "FP32 weights, plain FP32 sums"}


def profiled_traffic(kind: str, precision: str, schedule: int):
    """HBM bytes per scan launch from the committed rocprofv3 counter record,
    or None when it is missing or was taken on a different scan source,
    precision or schedule."""
    from paper_1306_1467_amd.profsum import scan_source_hash
    path = os.path.join(ROOT, "profiles", f"stump_scan_{kind}_counters.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    records = d.get("records", [d])
    h = scan_source_hash()
    for r in records:
        if r.get("scan_source_hash") == h and r.get("precision") == precision:
            got = r.get("schedules", {}).get(str(schedule), {}).get("bytes_per_launch")
            if got is not None:
                return got
    return None


def progress(msg: str):
    """One line per finished step on stderr (the JSON result line is the only stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_tables(images, features=None, threads: int = 0):
    # threads: OpenMP threads of every oracle call (0: the current setting)
    """The oracle's one-time preparation: values and per-feature orders."""
    import oracle
    W = images.shape[2]
    feats = oracle.enumerate_features(W, images.shape[1]) if features is None else features
    t0 = time.perf_counter()
    ii = oracle.integrals(images, threads)
    vals = oracle.feature_values(ii, feats, threads)
    order = oracle.sort_features(vals, threads)
    return vals, order, time.perf_counter() - t0


def cpu_baseline(labels, tables, rounds: int, rounds_1t: int, threads: int):
    """The FP64 oracle's round time on the host cores over every feature of
    the headline workload: `rounds` rounds with `threads` host threads and
    `rounds_1t` with one thread."""
    import numpy as np
    import oracle
    vals, order, prep_s = tables
    F, n = vals.shape
    w = oracle.init_weights(labels)
    scratch = np.zeros(F, oracle.STUMP_DTYPE)
    oracle.boost_round(vals, order, labels, w, 1e-10, threads, scratch)   # warm caches
    t0 = time.perf_counter()
    for _ in range(rounds):
        oracle.boost_round(vals, order, labels, w, 1e-10, threads, scratch)
    dt = (time.perf_counter() - t0) / rounds
    t0 = time.perf_counter()
    for _ in range(rounds_1t):
        oracle.boost_round(vals, order, labels, w, 1e-10, 1, scratch)
    dt1 = (time.perf_counter() - t0) / max(rounds_1t, 1)
    return {"value": round(dt * 1e3, 2), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"{rounds} oracle rounds over all {F:,} features x {n:,} windows "
                      "(one-time value/sort preparation excluded)",
            "one_thread_ms": round(dt1 * 1e3, 1), "one_thread_rounds": rounds_1t,
            "prep_s": round(prep_s, 2), "host_cpu": _cpu_model(), "host_threads": os.cpu_count()}


def cpu_baseline_batched(name, specs, data, pick, n_features: int, rounds: int, threads: int):
    """The oracle on a bounded sample of a batched workload: the jobs `pick`,
    each over a seeded sample of n_features features, `rounds` rounds each;
    every job's round time is scaled by (its feature count / the sample), and
    the rate is jobs*rounds/s over those jobs.  The whole workload's rate is
    estimated from the per-key time of the sample."""
    import numpy as np
    import oracle
    t_job = []
    keys_sampled = 0
    t_sampled = 0.0
    for k in pick:
        images, labels = data[k]
        s = specs[k]
        feats = oracle.enumerate_features(s.size, s.size)
        F = len(feats)
        nf = min(n_features, F)
        sel = np.sort(np.random.default_rng(1000 + k).choice(F, nf, replace=False))
        vals, order, _ = oracle_tables(images, feats[sel], threads)
        w = oracle.init_weights(labels)
        scratch = np.zeros(nf, oracle.STUMP_DTYPE)
        t0 = time.perf_counter()
        for _ in range(rounds):
            oracle.boost_round(vals, order, labels, w, 1e-10, threads, scratch)
        dt = (time.perf_counter() - t0) / rounds
        t_job.append(dt * F / nf)
        keys_sampled += nf * len(labels)
        t_sampled += dt
        del vals, order
    s_per_key = t_sampled / keys_sampled
    import oracle as _o
    all_keys = sum(_o.feature_count(s.size, s.size) * s.n for s in specs)
    return {"value": round(len(pick) / sum(t_job), 3), "unit": "jobs·rounds/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(pick)} of {len(specs)} {name} jobs ({', '.join(str(k) for k in pick)}), "
                      f"{n_features:,} sampled features each, {rounds} rounds per job, each job's round time "
                      "scaled by its feature count over the sample",
            "job_round_s": [round(t, 4) for t in t_job],
            "est_full_workload_jobs_rounds_per_s": round(len(specs) / (s_per_key * all_keys), 4)}


def single_job(args, torch, vb, images, labels, precision: str, steps: int, warmup: int):
    """One precision mode on the headline workload: init (tuned, and again
    with the tuning cache warm), the timed graph replay, the per-round
    distribution, per-kernel device times and the stream probe."""
    vb.boost_tune_cache_clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=precision,
                    schedule_id=args.schedule)
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t0) * 1e3
    schedule, tune_ms = tr.schedule()
    tuning = {"requested": args.schedule, "chosen": schedule,
              "best_scan_ms_by_schedule": {str(k): round(m, 4) for k, m in enumerate(tune_ms) if m > 0}}
    F, n = tr.F, tr.n
    if warmup:
        vb.boost_train(tr.ctx, warmup, False)
    tr.stream.synchronize()
    # timed region: `steps` rounds replayed from the captured HIP graph; HIP
    # events on the library's stream bracket the region
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(tr.stream):
        ev0.record()
    vb.boost_train(tr.ctx, steps, False)
    with torch.cuda.stream(tr.stream):
        ev1.record()
    tr.stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    graph_ms = ev0.elapsed_time(ev1) / steps
    # per-round distribution (outside the timed region)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    with torch.cuda.stream(tr.stream):
        evs[0].record()
    for r in range(steps):
        vb.boost_train(tr.ctx, 1, False)
        with torch.cuda.stream(tr.stream):
            evs[r + 1].record()
    tr.stream.synchronize()
    per_round = sorted(evs[r].elapsed_time(evs[r + 1]) for r in range(steps))
    pct = lambda q: per_round[min(len(per_round) - 1, int(q * len(per_round)))]
    tr.close()
    # init again with the choice in the tuning cache (no timing of candidates)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=precision,
                    schedule_id=args.schedule, flags=vb.BOOST_FLAG_TIMING)
    torch.cuda.synchronize()
    init_hit_ms = (time.perf_counter() - t0) * 1e3
    # per-kernel device times: HIP events around each kernel (direct launches)
    if warmup:
        vb.boost_train(tr.ctx, warmup, False)
    vb.boost_reset_timing(tr.ctx)
    t1 = time.perf_counter()
    vb.boost_train(tr.ctx, steps, False)
    tr.stream.synchronize()
    timed_ms = (time.perf_counter() - t1) * 1e3 / steps
    scan_ms, upd_ms, nr, _ = vb.boost_get_timing(tr.ctx)
    probe_ms = vb.boost_probe_stream(tr.ctx, 10)   # the same key reads with no arithmetic
    tr.close()
    torch.cuda.empty_cache()
    scan_avg = scan_ms / nr
    alg_bytes = F * n * 2
    achieved = alg_bytes / (scan_avg * 1e-3) / 1e9
    traffic = profiled_traffic("faces15k", precision, schedule)
    return {
        "precision": precision,
        "ms_per_step": round(elapsed * 1e3 / steps, 4),
        "graph_event_ms_per_round": round(graph_ms, 4),
        "round_ms_p10_p50_p90": [round(pct(0.1), 4), round(pct(0.5), 4), round(pct(0.9), 4)],
        "event_instrumented_ms_per_round": round(timed_ms, 4),
        "init_ms": {"tuned": round(init_ms, 1), "tuning_cache_hit": round(init_hit_ms, 1)},
        "scan_ms_avg": round(scan_avg, 4),
        "update_ms_avg": round(upd_ms / nr, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                                         "copy-calibrated)",
                     "traffic_GBps": None if traffic is None else round(traffic / (scan_avg * 1e-3) / 1e9, 1),
                     "kernel": f"k_scan<{ {'fp32': 0, 'fp32_kahan': 1, 'fp64': 2, 'fp32_wide': 3}[precision] }, ...> "
                               f"(schedule {schedule})",
                     "alg_bytes_per_launch": alg_bytes},
        "stream_probe": {"ms": round(probe_ms, 4), "key_GBps": round(alg_bytes / (probe_ms * 1e-3) / 1e9, 1),
                         "scan_time_over_probe": round(probe_ms / scan_avg, 4)},
        "schedule_tuning": tuning, "schedule": schedule, "F": F, "n": n,
    }


def run_precision_sweep(args, torch, vb, images, labels, F: int, n: int, modes):
    """Other precision modes on the same workload: per-kernel device times
    (HIP events around each kernel, direct launches), measured schedule."""
    out = {}
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
        torch.cuda.empty_cache()
        scan_avg = scan_ms / nr
        out[prec] = {"schedule": schedule, "rounds": nr, "scan_ms_avg": round(scan_avg, 4),
                     "update_ms_avg": round(upd_ms / nr, 4), "ms_per_round": round((scan_ms + upd_ms) / nr, 4),
                     "scan_hbm_frac": round(F * n * 2 / (scan_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "last_error_raw": float(recs[-1]["error_raw"])}
    return out


def precision_report(torch, vb, datasets, modes, rounds: int, threads: int = 0):
    """Every mode against the FP64 oracle over `rounds` teacher-forced rounds
    per dataset: the oracle runs its own trajectory; each round the GPU gets
    the oracle's normalised weights, and every feature's two minimal errors,
    the chosen stump and its error are compared.  Relative errors forgive the
    oracle's own rounding (4 n 2^-53 absolute); a (0, 0) pair counts 0."""
    import numpy as np
    import oracle
    U64 = 2.0 ** -53
    out = {}
    for dname, images, labels, tables in datasets:
        vals, order, _ = tables
        n = len(labels)
        floor = 4.0 * n * U64
        traj = []
        w = oracle.init_weights(labels)
        scratch = np.zeros(vals.shape[0], oracle.STUMP_DTYPE)
        for _ in range(rounds):
            wn = w / w.sum()
            rec, st = oracle.boost_round(vals, order, labels, w, 1e-10, threads, scratch)
            errs = np.sort(np.partition(st["err"], 1)[:2])
            traj.append((wn, rec, st["err_pos"].copy(), st["err_neg"].copy(), float(errs[1] - errs[0])))

        def rel(g, r):
            d = np.maximum(np.abs(g - r) - floor, 0.0)
            o = np.zeros_like(d)
            nz = r > 0
            o[nz] = d[nz] / r[nz]
            o[~nz] = np.where(d[~nz] > 0, np.inf, 0.0)
            return o
        res = {}
        for mode in modes:
            tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=mode,
                            schedule_id=vb.BOOST_SCHEDULE_AUTO)
            mx_feat, mx_best, agree, ties, mx_abs = 0.0, 0.0, 0, 0, 0.0
            per_round = []
            for wn, orec, ep, en, gap in traj:
                tr.set_weights(wn)
                g, ferr = tr.round(feature_err=True)
                ferr = ferr.cpu().numpy()
                rf = float(max(rel(ferr[:, 0], ep).max(), rel(ferr[:, 1], en).max()))
                rb = float(rel(np.array([g.error_raw]), np.array([orec.err_raw]))[0])
                same = (g.feature, g.polarity, g.threshold) == (orec.feature, orec.polarity, orec.theta)
                tie = gap <= 1e-6 * max(orec.err_raw, floor)
                mx_feat, mx_best = max(mx_feat, rf), max(mx_best, rb)
                mx_abs = max(mx_abs, float(max(np.abs(ferr[:, 0] - ep).max(), np.abs(ferr[:, 1] - en).max())))
                agree += int(same)
                ties += int((not same) and tie)
                per_round.append(rf)
            tr.close()
            del tr
            torch.cuda.empty_cache()
            res[mode] = {"rounds": len(traj), "max_rel_feature_error": mx_feat, "max_rel_best_error": mx_best,
                         "max_abs_feature_error": mx_abs, "stumps_equal": agree, "differ_at_ties": ties,
                         "per_round_max_rel_feature_error": per_round}
        out[dname] = {"windows": n, "features": int(vals.shape[0]),
                      "eps_range": [min(t[1].err_raw for t in traj), max(t[1].err_raw for t in traj)],
                      "modes": res}
    return out


def run_batched(name, precision, args, torch, vb, specs, data):
    """Jobs of a batched workload trained together (persistent scans from a
    work queue + one update launch per round, graph-replayed) against the same
    jobs trained one at a time through the single-job path, same precision
    and schedule policy."""
    rounds = args.batch_rounds or specs[0].rounds
    t_plain = 0.0
    plain = []
    for images, labels in data:
        tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=precision,
                        schedule_id=args.batch_schedule)
        vb.boost_train(tr.ctx, 1, False)   # graph capture, untimed
        tr.stream.synchronize()
        t0 = time.perf_counter()
        plain.append(vb.boost_train(tr.ctx, rounds, True))
        t_plain += time.perf_counter() - t0
        tr.close()
        del tr
        torch.cuda.empty_cache()
    vb.boost_tune_cache_clear()
    t0 = time.perf_counter()
    bt = vb.BatchTrainer([(torch.from_numpy(i), torch.from_numpy(l)) for i, l in data], precision=precision,
                         schedule_id=args.batch_schedule)
    bt.sync()
    init_s = time.perf_counter() - t0
    lib_init_s, alloc_s = bt.init_s, bt.alloc_s
    bt.train(1, False)
    bt.sync()
    t0 = time.perf_counter()
    recs = bt.train(rounds, True)
    t_batch = time.perf_counter() - t0
    same = all(recs[:, k].tobytes() == plain[k].tobytes() for k in range(len(data)))
    chosen = bt.schedule()
    bt_ws = bt.ws_bytes
    keys = sum(vb.boost_feature_count(vb.feature_set(s.size)) * s.n for s in specs)
    jr = len(data) * rounds
    bt.close()
    del bt
    torch.cuda.empty_cache()
    sizes = sorted({s.size for s in specs})
    return {"workload": f"{len(data)} jobs, " + "/".join(f"{z}x{z}" for z in sizes) + " windows"
                        + f", {min(s.n for s in specs):,}-{max(s.n for s in specs):,} windows per job",
            "jobs": len(data), "rounds": rounds, "precision": precision, "keys_per_round": keys,
            "batched_jobs_rounds_per_s": round(jr / t_batch, 2),
            "plain_jobs_rounds_per_s": round(jr / t_plain, 2),
            "speedup_vs_plain": round(t_plain / t_batch, 3),
            "batched_ms_per_round": round(t_batch * 1e3 / rounds, 3),
            "batched_key_GBps": round(keys * 2 * rounds / t_batch / 1e9, 1),
            "batched_init_s": round(lib_init_s, 3),
            "batched_init_detail": {"boost_batch_init_s": round(lib_init_s, 3),
                                    "workspace_alloc_s": round(alloc_s, 3),
                                    "workspace_GB": round(bt_ws / 1e9, 1),
                                    "constructor_total_s": round(init_s, 3),
                                    "tuning": "cold (tuning cache cleared first)"},
            "schedule": {"requested": args.batch_schedule,
                         "key14": {"schedule": chosen[0][0], "segs_per_wg": chosen[0][1]},
                         "key15": {"schedule": chosen[1][0], "segs_per_wg": chosen[1][1]}},
            "stumps_identical_to_plain": bool(same)}


def retrain_report(torch, vb, images, labels, precision: str, n0: int = 10000, fracs=(0.01, 0.1, 0.5)):
    """Incremental retraining: a context prepared on n0 windows of the
    headline workload, extended by m = frac * n0 more (boost_extend, which
    reuses the old windows' key order), against a fresh boost_init on the same
    n0 + m windows.  Library times only (the workspace allocations are the
    caller's); schedule fixed, so no tuning in either.  The extended context's
    sorted keys (a sample of features) and first 3 rounds must equal the
    fresh one's."""
    import numpy as np
    p = np.random.default_rng(957).permutation(len(labels))
    img, lab = np.ascontiguousarray(images[p]), np.ascontiguousarray(labels[p])
    sched = 9
    base = vb.Trainer(torch.from_numpy(img[:n0]), torch.from_numpy(lab[:n0]), precision=precision,
                      schedule_id=sched)
    out = {"base_windows": n0, "precision": precision, "schedule": sched, "base_init_ms": round(base.init_s * 1e3, 2),
           "cases": []}
    for f in fracs:
        m = int(round(f * n0))
        union_img, union_lab = img[:n0 + m], lab[:n0 + m]
        ext = base.extend(torch.from_numpy(img[n0:n0 + m]), torch.from_numpy(lab[n0:n0 + m]))
        fresh = vb.Trainer(torch.from_numpy(union_img), torch.from_numpy(union_lab), precision=precision,
                           schedule_id=sched)
        same = True
        for j0 in (0, fresh.F // 3, fresh.F - 2048):
            oe, fe = ext.sorted(j0, 2048)
            of, ff = fresh.sorted(j0, 2048)
            same &= bool(torch.equal(oe, of) and torch.equal(fe, ff))
        same &= ext.train(3).tobytes() == fresh.train(3).tobytes()
        out["cases"].append({"added_windows": m, "added_frac": f, "merged": ext.merged(),
                             "extend_ms": round(ext.init_s * 1e3, 2), "fresh_init_ms": round(fresh.init_s * 1e3, 2),
                             "speedup": round(fresh.init_s / ext.init_s, 2), "identical_to_fresh": same})
        progress(f"retrain +{m} windows: extend {ext.init_s * 1e3:.1f} ms, fresh {fresh.init_s * 1e3:.1f} ms")
        for t in (ext, fresh):
            t.close()
        del ext, fresh
        torch.cuda.empty_cache()
    base.close()
    del base
    torch.cuda.empty_cache()
    return out


def classifier_report(torch, vb, images, labels, himg, hlab, precision: str, rounds: int):
    """The strong classifier of `rounds` stumps: training-error curve and the
    error on held-out windows (the same recipe, seeded apart)."""
    tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=precision,
                    schedule_id=vb.BOOST_SCHEDULE_AUTO)
    recs = tr.train(rounds)
    curve = tr.error_curve(recs).cpu().numpy()
    tr.close()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    _, _, hcurve = vb.classify(himg, recs, hlab)
    ev1.record()
    torch.cuda.synchronize()
    hcurve = hcurve.cpu().numpy()
    n, m = len(labels), len(hlab)
    at = [t for t in (1, 10, 50, 100, 200) if t <= rounds]
    return {"stumps": rounds, "training_windows": n, "held_out_windows": m,
            "training_error": round(float(curve[-1]) / n, 6), "held_out_error": round(float(hcurve[-1]) / m, 6),
            "after_rounds": at,
            "training_error_after": [round(float(curve[t - 1]) / n, 6) for t in at],
            "held_out_error_after": [round(float(hcurve[t - 1]) / m, 6) for t in at],
            "held_out_classify_ms": round(ev0.elapsed_time(ev1), 3)}


def flipped_job(synth, seed=25, n_pos=5000, n_neg=10000):
    """A non-separable set of the headline shape: contrast 60, 8 % of the
    labels flipped by a seeded draw."""
    import numpy as np
    images, labels = synth.make_job((seed, 0), n_pos, n_neg, size=24, r0=8, contrast=60.0)
    flip = np.random.default_rng(seed).random(len(labels)) < 0.08
    return images, np.where(flip, 1 - labels, labels).astype(np.uint8)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp32_kahan", help="headline precision mode")
    ap.add_argument("--variants", default="fp32_wide",
                    help="other modes measured like the headline, with their own roofline (empty: none)")
    ap.add_argument("--schedule", type=int, default=-1,
                    help="scan launch schedule of the single-job workload (-1: measured choice at init)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rounds", type=int, default=20)
    ap.add_argument("--cpu-rounds-1t", type=int, default=1)
    ap.add_argument("--cpu-batch-features", type=int, default=8192,
                    help="sampled features per job of the batched workloads' oracle baselines")
    ap.add_argument("--sweep-precisions", default="fp64,fp32",
                    help="further modes timed on the same workload (empty: none)")
    ap.add_argument("--sweep-rounds", type=int, default=50)
    ap.add_argument("--precision-rounds", type=int, default=20,
                    help="teacher-forced full-size rounds per dataset of the precision report (0: none)")
    ap.add_argument("--batched", default="batch32,batch64",
                    help="comma list of batched workloads (batch32: 32 uneven jobs of 24x24 windows, "
                         "batch64: 64 jobs of 16-28 px windows); empty for none")
    ap.add_argument("--batch-precision", default="",
                    help="modes of the batched runs (comma list; default: the headline mode for batch32, "
                         "the headline mode and fp32_wide for batch64)")
    ap.add_argument("--batch-rounds", type=int, default=0, help="rounds per batched job (0: the workload's own)")
    ap.add_argument("--batch-schedule", type=int, default=-1,
                    help="schedule of the batched and the plain per-job runs (-1: measured choice at init)")
    ap.add_argument("--classifier-rounds", type=int, default=200, help="0 skips the strong-classifier report")
    ap.add_argument("--no-retrain", action="store_true", help="skip the incremental-retraining timings")
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
    images, labels = synth.workload_jobs("faces15k")[0].make()
    host_threads = 0
    if not args.no_cpu_baseline or args.precision_rounds > 0:
        import oracle
        host_threads = oracle.max_threads()   # every host thread; the oracle calls below pass it explicitly
    if args.prep_only:
        t0 = time.perf_counter()
        tr = vb.Trainer(torch.from_numpy(images), torch.from_numpy(labels), precision=args.precision, schedule_id=0)
        torch.cuda.synchronize()
        print(json.dumps({"prep_only": True, "init_ms": round((time.perf_counter() - t0) * 1e3, 1),
                          "features": tr.F, "windows": tr.n}), flush=True)
        tr.close()
        return
    res = single_job(args, torch, vb, images, labels, args.precision, args.steps, args.warmup)
    progress(f"headline {args.precision}: {res['ms_per_step']} ms per round")
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
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": "162,336 Haar features x 15,000 windows 24x24 (5,000 pos + 10,000 neg), "
                               "one boosting round per step", "precision": args.precision,
                   "precision_detail": PRECISION_NAME[args.precision],
                   "schedule": res["schedule"], "schedule_requested": args.schedule, "features": res["F"],
                   "windows": res["n"]},
        "roofline": res["roofline"],
    }
    for k in ("init_ms", "graph_event_ms_per_round", "round_ms_p10_p50_p90", "event_instrumented_ms_per_round",
              "scan_ms_avg", "update_ms_avg", "stream_probe", "schedule_tuning"):
        line[k] = res[k]
    variants = [v.strip() for v in args.variants.split(",") if v.strip() and v.strip() != args.precision]
    if variants:
        line["variants"] = {}
        for v in variants:
            r = single_job(args, torch, vb, images, labels, v, args.steps, args.warmup)
            line["variants"][v] = {k: r[k] for k in ("precision", "ms_per_step", "graph_event_ms_per_round",
                                                     "round_ms_p10_p50_p90", "init_ms", "scan_ms_avg",
                                                     "update_ms_avg", "roofline", "stream_probe", "schedule")}
            line["variants"][v]["precision_detail"] = PRECISION_NAME[v]
            progress(f"variant {v}: {r['ms_per_step']} ms per round")
    sweep = [m for m in args.sweep_precisions.split(",") if m and m != args.precision and m not in variants]
    if sweep:
        line["precision_sweep"] = run_precision_sweep(args, torch, vb, images, labels, res["F"], res["n"], sweep)
        progress("precision sweep done")
    if args.classifier_rounds > 0:
        himg, hlab = synth.make_job((1, 1), 1000, 2000)
        line["strong_classifier"] = classifier_report(torch, vb, images, labels, himg, hlab, args.precision,
                                                      args.classifier_rounds)
        # the headline set is separable by single features (zero error from
        # the first stump on); the flipped-label set shows a real curve
        fimg, flab = flipped_job(synth)
        fh_img, fh_lab = flipped_job(synth, seed=26, n_pos=1000, n_neg=2000)
        line["strong_classifier_flipped_labels"] = dict(
            classifier_report(torch, vb, fimg, flab, fh_img, fh_lab, args.precision, args.classifier_rounds),
            data="contrast 60, 8 % of labels flipped (training and held-out alike)")
        progress("strong classifier done")
    if not args.no_retrain:
        line["incremental_retraining"] = retrain_report(torch, vb, images, labels, args.precision)
    headline_tables = None
    if args.precision_rounds > 0 or not args.no_cpu_baseline:
        headline_tables = oracle_tables(images, None, host_threads)
        progress("oracle tables of the headline data built")
    if args.precision_rounds > 0:
        modes = [args.precision] + [m for m in ("fp32_wide", "fp64", "fp32") if m != args.precision]
        fimg, flab = flipped_job(synth)
        line["precision_report"] = precision_report(torch, vb, [("headline", images, labels, headline_tables)],
                                                    modes, args.precision_rounds, host_threads)
        progress("precision report: headline data done")
        ftables = oracle_tables(fimg, None, host_threads)
        line["precision_report"].update(precision_report(
            torch, vb, [("contrast60_flipped8pct", fimg, flab, ftables)], modes, args.precision_rounds, host_threads))
        del ftables
        progress("precision report: flipped-label data done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(labels, headline_tables, args.cpu_rounds, args.cpu_rounds_1t, host_threads)
        progress("oracle baseline of the headline round done")
    else:
        line["cpu_baseline"] = None
    del headline_tables
    for name in [c.strip() for c in args.batched.split(",") if c.strip()]:
        specs = synth.workload_jobs(name)
        data = [s.make() for s in specs]
        if args.batch_precision:
            modes = [m.strip() for m in args.batch_precision.split(",") if m.strip()]
        else:
            modes = [args.precision] + (["fp32_wide"] if name == "batch64" and args.precision != "fp32_wide" else [])
        for m in modes:
            key = f"batched_{name}" if m == modes[0] else f"batched_{name}_{m}"
            line[key] = run_batched(name, m, args, torch, vb, specs, data)
            progress(f"{name} {m}: {line[key]['speedup_vs_plain']}x plain")
        if not args.no_cpu_baseline:
            order = sorted(range(len(specs)), key=lambda k: specs[k].n * vb.boost_feature_count(
                vb.feature_set(specs[k].size)))
            pick = list(range(len(specs))) if name == "batch32" else order[:4] + order[-2:]
            line[f"cpu_baseline_{name}"] = cpu_baseline_batched(name, specs, data, pick, args.cpu_batch_features, 2,
                                                                host_threads)
            progress(f"oracle baseline of {name} done")
        del data
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
