#!/usr/bin/env python3
"""Throughput of the ENS traveltime-parameter search on one MI355X.

One step = one pass of the whole path over the workload: bind the
device-resident traces into the library's store (quantising them to binary16
for the 16-bit workloads), then the search (initial populations, every
generation of every ENS stage, the neighbour exchange), the gradient polish
where the workload has one, and the binary64 re-scoring of every winner.
Prints one JSON line.

Workloads (synthetic Ricker gathers, synth.WORKLOADS): crs_diff (default:
2048 CMPs x 96 offsets x 2000 samples at 2 ms, CRS operator, NP 32 x NG 40 +
ENS, binary16 traces, 10 adjoint-polish steps), crs_ens, cmp_small,
crs_uneven, crs_precision.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "semblance evals/s & ZO samples/s at <=1e-3 semblance gap; % of HBM peak"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X vector binary32 (counts packed dual-FMA issue)
# per-CU vector-memory path (texture addresser / L1 return): 64 B per clock,
# 256 CUs at 2.4 GHz; derived from unit counts, matching the ~60 B per busy
# cycle the TA counters show for the search kernel's window loads
VMEM_PATH_PEAK_GBS = 256 * 64 * 2.4
CSRC = os.path.join(ROOT, "paper_2304_11399_amd", "csrc")
KERNEL_SOURCES = ("device.h", "eval.h", "launch.h", "search.h", "kernels.hip", "search_f32.hip",
                  "search_f16.hip", "search_bf16.hip")
DT_CODE = {"f32": 0, "f16": 1, "bf16": 2}


def flops_per_pair(op, window):
    """Arithmetic of the definition per (candidate, participating trace).

    Traveltime with per-candidate constants folded (mo = al dm + be dm^2 +
    ga h^2: 5; q = n0^2 + mo: 1; sqrt: 1; dtau = mo / (tau + n0): 2; floor
    and fraction: 2) = 11 (CMP: mo = ga h^2: 1 -> 7); per window sample the
    interpolation (1-f) u_k + f u_k+1 (3) and the sums s_k += a, E += a^2 (3),
    plus 1 for 1-f.
    """
    tt = 11 if op == 3 else 7
    return tt + 6 * window + 1


def kernel_sources_sha(root=ROOT):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(root, "paper_2304_11399_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_profile(workload, kernel, shape, root=ROOT):
    """The committed rocprofv3 summary of the dominant kernel (HBM bytes per
    launch from FETCH_SIZE/WRITE_SIZE, VALU/TA busy, L2 hit rate), or None when
    the kernel sources, the kernel or its launch shape differ from the
    profiled ones."""
    path = os.path.join(root, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != kernel_sources_sha(root) or rec.get("kernel") != kernel:
        return None
    if rec.get("shape") != shape:
        return None
    return rec


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="crs_diff")
    ap.add_argument("--store", default=None, help="f32, f16 or bf16 (default: the workload's)")
    ap.add_argument("--waves", type=int, default=0, help="trace slices per population (0: auto)")
    ap.add_argument("--order", type=int, default=0,
                    help="work-item order: 1 XCD-contiguous, 2 costliest first, "
                         "3 costliest first within XCD-contiguous shares (0: measure)")
    ap.add_argument("--occupancy", type=int, default=0,
                    help="search kernel registers: 1 as compiled, 2 held to 64 (0: measure)")
    ap.add_argument("--packing", type=int, default=0,
                    help="exploration workgroups: 1 one population per lane group, 2/4/8 "
                         "populations packed over that many waves (0: measure)")
    ap.add_argument("--gather", type=int, default=0,
                    help="1: binary32 windows staged per trace in LDS (0: read directly)")
    ap.add_argument("--graph", action="store_true", help="replay the trace steps as a HIP graph")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the equal-accuracy comparison of the variants")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gap", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="CPU work per oracle timing (all cores, then one core)")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-clock seconds after which the remaining comparison rows are "
                         "skipped (and listed as skipped)")
    return ap.parse_args()


def cpu_baseline(g, wl, de, bounds, seconds):
    """The oracle (binary64 C, OpenMP) on a bounded sample of the workload, on
    every host core it is given and on one core."""
    import numpy as np

    import oracle
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    if wl["de"]["ens_enabled"]:
        mid = g.n_cmp // 2 - 2
        t0, t1 = g.nt // 4, g.nt // 4 + min(500, g.nt // 2)
        de_s = dict(de, n_bucket=4, polish_steps=0)
    else:
        t0, t1 = 0, g.nt
        de_s = de

    def timed(limit):
        start = time.perf_counter()
        n = ev = k = 0
        while True:
            if wl["de"]["ens_enabled"]:
                # successive 4-CMP buckets from the middle of the line
                c0 = (mid + 4 * k) % max(1, g.n_cmp - 3)
                cmp_out = np.arange(c0, c0 + 4, dtype=np.int32)
                tt1 = t1
            else:
                cmp_out = np.arange(g.n_cmp, dtype=np.int32)
                tt1 = t1
            _, _, e = L.search(bounds, de_s, wl["search_seed"], cmp_out=cmp_out, t_begin=t0,
                               t_end=tt1)
            n += cmp_out.size * (tt1 - t0)
            ev += e
            k += 1
            if time.perf_counter() - start >= limit:
                break
        return n, ev, k, time.perf_counter() - start

    lib = oracle.lib()
    threads = int(lib.or_num_threads())
    n, ev, k, sec = timed(seconds)
    lib.or_set_num_threads(1)
    if wl["de"]["ens_enabled"]:
        t1_all = t1
        t1 = t0 + min(100, t1 - t0)     # a narrower band of t keeps the one-core leg short
    n1, ev1, k1, sec1 = timed(seconds)
    lib.or_set_num_threads(threads)
    if wl["de"]["ens_enabled"]:
        what = (f"ENS (no polish) over {k} 4-CMP bucket(s) from CMP {mid} x t {t0}..{t1_all - 1}")
        what1 = f"{k1} 4-CMP bucket(s) x t {t0}..{t1 - 1}"
    else:
        what, what1 = f"plain DE over the whole line, {k} time(s)", f"{k1} time(s)"
    return {"value": round(n / sec, 3), "unit": "ZO samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}: {n} ZO samples, {ev} evaluations, {sec:.1f} s, {ev / sec:.4g} evals/s",
            "one_core": {"value": round(n1 / sec1, 3), "unit": "ZO samples/s", "cores": 1,
                         "sample": f"{what1}: {n1} ZO samples, {ev1} evaluations, {sec1:.1f} s, "
                                   f"{ev1 / sec1:.4g} evals/s"}}


def variants_for(name, wl):
    """(method, storage, search configuration) rows of the equal-accuracy
    comparison.  crs_diff: the binary16 + polish claim, the binary16 search with the
    adjoint polish against the per-sample binary32 search the paper compares
    with, with ENS in binary32 and in binary16 without polish between them."""
    de0 = dict(wl["de"])
    plain0 = dict(de0, ens_enabled=0, polish_steps=0, n_skip=0)
    if name == "crs_diff":
        # most telling rows first (a time budget may cut the list short): the
        # configured budget, the per-sample binary32 search at it, the smaller
        # ENS budget with and without binary16 storage and polish, then the rest
        nop = dict(de0, polish_steps=0)
        small = dict(np_lo=16, np_hi=16, ng_f=20)
        return [("ens_f16_polish", "f16", dict(de0)),
                ("plain_f32", "f32", dict(plain0)),
                ("ens_f16_polish", "f16", dict(de0, **small)),
                ("ens_f16", "f16", dict(nop, **small)),
                ("ens_f32", "f32", dict(nop, **small)),
                ("plain_f32", "f32", dict(plain0, **small)),
                ("ens_f16_polish", "f16", dict(de0, np_lo=16, np_hi=16, ng_f=10)),
                ("ens_f32", "f32", dict(nop)),
                ("ens_f16", "f16", dict(nop)),
                ("plain_f32", "f32", dict(plain0, ng_f=80))]
    if name == "crs_ens":
        return [("ens", "f32", dict(de0)),
                ("ens", "f32", dict(de0, np_lo=16, np_hi=16, ng_f=20)),
                ("ens", "f32", dict(de0, np_lo=16, np_hi=16, ng_f=10)),
                ("ens_skip2", "f32", dict(de0, n_skip=2)),
                ("ens_skip2", "f32", dict(de0, np_lo=16, np_hi=16, ng_f=20, n_skip=2)),
                ("ens_jade", "f32", dict(de0, adapt=1, CR=0.5)),
                ("ens_jade", "f32", dict(de0, np_lo=16, np_hi=16, ng_f=20, adapt=1, CR=0.5)),
                ("plain_jade", "f32", dict(plain0, ng_f=40, adapt=1, CR=0.5)),
                ("plain_jade", "f32", dict(plain0, adapt=1, CR=0.5)),
                ("plain", "f32", dict(plain0, np_lo=16, np_hi=16, ng_f=20)),
                ("plain", "f32", dict(plain0, ng_f=40)),
                ("plain", "f32", dict(plain0))]
    if name == "cmp_small":
        # the configured budget is NP 16 x NG 30; more generations do not close
        # the gap (the populations settle on side maxima), a larger population does
        return [("plain", "f32", dict(de0)),
                ("plain", "f32", dict(de0, ng_f=60)),
                ("plain", "f32", dict(de0, np_lo=24, np_hi=24, ng_f=20)),
                ("plain", "f32", dict(de0, np_lo=24, np_hi=24))]
    return []


def compare_equal_accuracy(ctxs, bounds, wl, g, seed, note, main=None, deadline=None):
    """Each row's throughput and gap; the fastest row of each method whose mean
    gap to the reference maxima is <= 1e-3 is that method's throughput at
    equal accuracy.  main = (store, de, seconds, S64) of the timed steps: the
    row with that configuration takes their mean step time (bind + search +
    re-score) instead of a run of its own.  Rows not started by `deadline`
    (time.perf_counter()) are listed as skipped."""
    import torch
    rows, skipped = [], []
    variants = variants_for(wl["name"], wl)
    for k, (kind, store, de) in enumerate(variants):
        if main is not None and store == main[0] and de == main[1]:
            sec, S64 = main[2], main[3]
            note(f"compare {k + 1}/{len(variants)} {kind} {de['np_lo']}x{de['ng_f']}: "
                 f"{1e3 * sec:.1f} ms (the timed steps)")
            n_evals = main[4]
        elif deadline is not None and time.perf_counter() > deadline:
            skipped.append({"method": kind, "np": de["np_lo"], "ng": de["ng_f"], "store": store})
            note(f"compare {k + 1}/{len(variants)} {kind} {de['np_lo']}x{de['ng_f']}: skipped (time)")
            continue
        else:
            c = ctxs[store]
            for attempt in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = c.search(bounds, de, seed, rescore_fp64=True)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                if c.stats()["tune_ms"] == 0:  # no launch-shape measurement inside the clock
                    break
            S64, n_evals = out["S64"].cpu().numpy(), out["n_evals"]
            note(f"compare {k + 1}/{len(variants)} {kind} {de['np_lo']}x{de['ng_f']}: {1e3 * sec:.1f} ms")
        gap = gap_stats(wl["name"], S64, g.nt, g)
        rows.append({"method": kind, "np": de["np_lo"], "ng": de["ng_f"],
                     "n_skip": de.get("n_skip", 0), "adapt": de.get("adapt", 0),
                     "store": store, "polish": de.get("polish_steps", 0),
                     "ms": round(1e3 * sec, 2), "zo_samples_per_s": round(g.n_cmp * g.nt / sec, 1),
                     "evals": n_evals, "gap_mean": gap["mean"] if gap else None,
                     "frac_le_1e-3": gap["frac_le_1e-3"] if gap else None})
    best = {}
    for r in rows:
        if r["gap_mean"] is not None and r["gap_mean"] <= 1e-3:
            b = best.get(r["method"])
            if b is None or r["zo_samples_per_s"] > b["zo_samples_per_s"]:
                best[r["method"]] = r

    def ratio(a, b):
        if a in best and b in best:
            return round(best[a]["zo_samples_per_s"] / best[b]["zo_samples_per_s"], 3)
        return None
    res = {"runs": rows, "best_at_gap_le_1e-3": best, "skipped_for_time": skipped}
    if wl["name"] == "crs_diff":
        res["ens_f16_polish_over_plain_f32_zo_samples_per_s"] = ratio("ens_f16_polish", "plain_f32")
        res["ens_f16_over_plain_f32"] = ratio("ens_f16", "plain_f32")
        res["ens_f32_over_plain_f32"] = ratio("ens_f32", "plain_f32")
        res["ens_f16_polish_over_ens_f32"] = ratio("ens_f16_polish", "ens_f32")
    elif wl["name"] == "crs_ens":
        res["ens_over_plain_zo_samples_per_s"] = ratio("ens", "plain")
        res["ens_skip2_over_plain_zo_samples_per_s"] = ratio("ens_skip2", "plain")
        res["ens_jade_over_plain_jade_zo_samples_per_s"] = ratio("ens_jade", "plain_jade")
    return res


def gap_stats(name, S64, nt, g):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"sref_{name}.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    fp = float((g.traces.astype(np.float64) ** 2).sum())
    if abs(fp / float(ref["fingerprint"]) - 1.0) > 1e-9:
        return {"error": "reference maxima were made for other data"}
    found = S64.reshape(-1)[ref["cmp"].astype(np.int64) * nt + ref["t"]]
    gap = np.maximum(ref["S_ref"] - found, 0.0)
    return {"n": int(gap.size), "mean": float(gap.mean()), "p50": float(np.median(gap)),
            "p95": float(np.quantile(gap, 0.95)), "max": float(gap.max()),
            "frac_le_1e-3": float((gap <= 1e-3).mean()),
            "mean_S": float(found.mean()), "rms_S": float(np.sqrt((found ** 2).mean()))}


def main():
    t_start = time.perf_counter()
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        msg = ("the library runs on one GPU: the search shards by bucket across GPUs "
               "by design but no multi-GPU path is built; run with --gpus 1")
        print(json.dumps({"metric": METRIC, "error": msg, "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2304_11399_amd as ens
    from synth import base_bounds, make_workload

    def note(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    g, wl = make_workload(args.workload)
    wl = dict(wl, name=args.workload)
    store = args.store or wl["store"]
    de, bounds = dict(wl["de"]), base_bounds(wl)
    stream = torch.cuda.Stream() if args.graph else torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        ctx = ens.Context(stream)
        ctx.set_tuning(waves_per_sample_group=args.waves, use_graph=int(args.graph),
                       item_order=args.order, occupancy=args.occupancy, packing=args.packing, gather=args.gather)
        # the one-time host-to-device upload, outside the steps
        torch.cuda.synchronize()
        t_up = time.perf_counter()
        traces = torch.from_numpy(g.traces).cuda()
        torch.cuda.synchronize()
        upload_ms = 1e3 * (time.perf_counter() - t_up)
        P_d = g.n_cmp * g.nt

        def bind():
            ctx.bind(traces, g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"], wl["window"], wl["ap_lo"],
                     wl["ap_hi"], store=store)

        def step():
            bind()
            return ctx.search(bounds, de, wl["search_seed"], rescore_fp64=True)

        note(f"{args.workload}: {args.warmup} warm-up step(s), launch shapes measured in the first")
        for _ in range(args.warmup):
            out = step()
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        bind()
        torch.cuda.synchronize()
        bind_ms = 1e3 * (time.perf_counter() - t_b)
        note(f"warm-up done; timing {args.steps} step(s)")
        t0 = time.perf_counter()
        for k in range(args.steps):
            out = step()
            # each step ends in a stream synchronisation (the search reads its
            # counters back), so this line costs the clock a print
            note(f"step {k + 1}/{args.steps} done")
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ms_step = 1e3 * sec / args.steps
        note(f"{ms_step:.1f} ms per step")
        evals = out["n_evals"]
        S64 = out["S64"].cpu().numpy()

        # one more step with per-launch event timing, outside the timed region
        ctx.set_tuning(waves_per_sample_group=args.waves, collect_timing=1, item_order=args.order,
                       occupancy=args.occupancy, packing=args.packing, gather=args.gather)
        step()
        st = ctx.stats()
        ctx.set_tuning(waves_per_sample_group=args.waves, item_order=args.order,
                       occupancy=args.occupancy, packing=args.packing, gather=args.gather)
        # quality outputs of the last step, outside the timed region: the
        # zero-offset stack along the winners and the coherence-panel RMS
        torch.cuda.synchronize()
        t_st = time.perf_counter()
        stack, coherence_rms = ctx.stack(out["params"], out["S"])
        stack_ms = 1e3 * (time.perf_counter() - t_st)
        stack_info = {"ms": round(stack_ms, 3), "coherence_rms": round(coherence_rms, 6),
                      "stack_rms": round(float(stack.double().pow(2).mean().sqrt().item()), 6)}
        comparison = None
        if not args.no_compare and not args.no_gap and variants_for(args.workload, wl):
            ctxs = {store: ctx}
            for s in {v[1] for v in variants_for(args.workload, wl)} - {store}:
                c = ens.Context(stream)
                c.bind(traces, g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"], wl["window"], wl["ap_lo"],
                       wl["ap_hi"], store=s)
                ctxs[s] = c
            comparison = compare_equal_accuracy(
                ctxs, bounds, wl, g, wl["search_seed"], note,
                main=(store, de, sec / args.steps, S64, evals), deadline=t_start + args.budget_s)

    if wl["de"]["ens_enabled"]:
        expect = ens.evals_ens(P_d, de["np_lo"], de["ng_f"], de["np_bf"], de["ng_bf"],
                               de["n_cycle"], de.get("n_skip", 0))
    else:
        expect = ens.evals_jade(P_d, de["np_lo"], de["ng_f"])
    assert de["np_lo"] != de["np_hi"] or evals == expect, (evals, expect)

    # roofline of the dominant kernel: the exploration trace-step launches
    ex = st["explore"]
    elem = 4 if store == "f32" else 2
    W = wl["window"]
    per_launch_s = ex["device_ms"] / 1e3 / ex["launches"]
    bytes_per_launch = ex["sum_m"] * (W + 1) * elem / ex["launches"]
    flops_per_launch = ex["sum_m"] * flops_per_pair(wl["op"], W) / ex["launches"]
    gbs = bytes_per_launch / per_launch_s / 1e9
    tflops = flops_per_launch / per_launch_s / 1e12
    if ex.get("packed"):
        kname = ("k_search_packed_dense" if ex.get("dense") else "k_search_packed") + \
            f"<{wl['op']}, {DT_CODE[store]}, {W}>"
    elif args.gather == 1 and store == "f32" and not de.get("adapt", 0):
        kname = f"k_search_tiles<{wl['op']}, {W}, 0>"
    else:
        kname = ("k_search_dense" if ex.get("dense") else "k_search") + \
            f"<{wl['op']}, {DT_CODE[store]}, {W}, 0>"
    shape = {"waves": ex.get("waves"), "item_order": ex.get("item_order"), "dense": ex.get("dense"),
             "packed": ex.get("packed", 0)}
    prof = measured_profile(args.workload, f"void ens::{kname}(ens::SearchArgs)", shape)
    traffic = None if prof is None else round(prof["traffic_bytes_per_launch"])
    roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tflops / FP32_PEAK_TFLOPS, 4), "traffic": traffic,
            "flops_per_pair": flops_per_pair(wl["op"], W),
            "algorithmic_bytes_per_launch": round(bytes_per_launch),
            "kernel": kname, "shape": shape,
            "launches": ex["launches"], "avg_launch_ms": round(ex["device_ms"] / ex["launches"], 4),
            # the same gathers against the per-CU vector-memory path every window
            # load passes through (the second limit of the kernel)
            "vector_memory_path": {"achieved": round(gbs, 1), "peak": round(VMEM_PATH_PEAK_GBS, 1),
                                   "unit": "GB/s", "frac": round(gbs / VMEM_PATH_PEAK_GBS, 4)},
            # algorithmic gather bytes over time: served by L1/L2/MALL, not by
            # HBM (the measured HBM bytes are "traffic"); not an HBM fraction
            "cache_served_gather_gbs": round(gbs, 1)}
    if prof is not None:
        roof["measured"] = {k: prof[k] for k in ("hbm_gbs", "valu_cycles_per_instr", "ta_busy", "l2_hit",
                                                 "profile") if k in prof}

    gap = None if args.no_gap else gap_stats(args.workload, S64, g.nt, g)
    line = {
        "metric": METRIC,
        "value": round(P_d * args.steps / sec, 3),
        "unit": "ZO samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "store": store,
        "arithmetic": ("binary32 window interpolation and sums" if store != "f16" else
                       "binary16 sample pairs times binary16 weights, exact products summed "
                       "in binary32 (traveltimes on a 2^-11-sample grid); binary32 sums"),
        "data": "synthetic",
        "config": {"workload": args.workload, "n_cmp": g.n_cmp, "offsets": int(g.cmp_ptr[1]),
                   "nt": g.nt, "dt": g.dt, "op": "CRS" if wl["op"] == 3 else "CMP", "window": W,
                   "aperture": [wl["ap_lo"], wl["ap_hi"]], "np": [de["np_lo"], de["np_hi"]],
                   "ng": de["ng_f"], "ens": bool(de["ens_enabled"]), "n_cycle": de["n_cycle"],
                   "n_bucket": de["n_bucket"], "polish_steps": de["polish_steps"],
                   "store": store, "zo_samples": P_d, "parallelism": "1 GPU"},
        "evals_per_s": round(evals * args.steps / sec, 1),
        "evals_per_step": evals,
        "upload_ms": round(upload_ms, 2),
        "bind_ms": round(bind_ms, 2),
        "gap": gap,
        "gap_ok": None if not gap or "mean" not in gap else bool(gap["mean"] <= 1e-3),
        "roofline": roof,
        "stats": st,
        "stack": stack_info,
        "equal_accuracy": comparison,
    }
    if not args.no_cpu_baseline:
        note("CPU baseline (the oracle on a bounded sample, all cores then one core)")
        line["cpu_baseline"] = cpu_baseline(g, wl, de, bounds, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
