"""Benchmark: unique languages enumerated per second on one MI355X.

A step solves one batch of synthetic single instances (alphabet {0,1}, target
expression of cost 10..14, 10 positive and 10 negative strings of length
0..7, seeds 0..31, under the cost functions (1,1,1,1,1) and (1,1,5,1,2))
with one rei_solve_batch call on the current stream (one workgroup per
instance runs its whole search; instances that outgrow their preallocated
rows finish on the per-chunk path).  Instances are staged (rei_create: host
staging + upload) before the timed region, so their tables are resident in
HBM when timing starts.  The same instances solved one after the other with
rei_solve are timed as well (sequential_value).

value = sum over the batch of unique languages enumerated / wall time of the
batch.  The JSON line also carries the time-to-minimal-regex distribution,
the dominant kernel's roofline figures (HIP events recorded by the library
around each launch, on the stream the kernel runs on) and the CPU oracle's
rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per work unit of each kernel class:
# a generator must probe the dedup table once per candidate; a probe is a
# random access, and the smallest HBM transaction is 64 bytes.
PROBE_BYTES = 64

# HBM bytes per launch of the dominant kernel, from FETCH_SIZE / WRITE_SIZE
# counter runs calibrated on a 1 GiB copy (profiles/hbm_traffic_counters.md),
# by (workload, kernel class).  Only valid for the kernels as they were
# measured: an entry is removed when its kernel changes.
TRAFFIC_BYTES = {
    ("row1", "gen_concat"): 295079584,
    ("single", "solve_batch"): 40402152,
    ("single", "gen_pieces"): 4097032,
    ("single", "gen_concat"): 3652345,
    ("batched", "solve_batch"): 545672132,
    ("batched", "gen_pieces"): 3831192,
    ("batched", "gen_concat"): 2344806,
}


def workload(name: str):
    from paper_2305_18575_amd import instances
    if name == "single":
        out = []
        for costs in ((1, 1, 1, 1, 1), (1, 1, 5, 1, 2)):
            for seed in range(32):
                out.append(instances.single_instance(seed, costs))
        desc = ("single instance: alphabet {0,1}, target cost 10-14, 10+10 strings of length 0-7, "
                "seeds 0-31 x cost functions (1,1,1,1,1) and (1,1,5,1,2), 64 solves per step")
        return out, desc
    if name == "plain":
        out = [instances.plain_instance(s) for s in range(200)]
        return out, "plain instance: alphabet {0,1}, target cost 1-8, 4+4 strings of length 1-5, seeds 0-199"
    if name == "batched":
        out = instances.batched_instances(0, 4096)
        return out, ("batched: 4096 instances from master seed 0, alphabet of 2-4 symbols, 2-16 positive and "
                     "2-16 negative strings of length 0-6, target cost 4-12, cost function (1,1,1,1,1), "
                     "max_cost = target cost")
    if name == "sweep":
        out = []
        for kind, seeds in (("type1", (0, 2)), ("type2", (1, 2))):
            gen = instances.type1_instance if kind == "type1" else instances.type2_instance
            for seed in seeds:
                for costs in instances.PAPER_COST_FUNCTIONS:
                    out.append(gen(seed, costs=costs, max_cost=1000))
        return out, ("cost-function sweep: Type 1 seeds 0 and 2, Type 2 seeds 1 and 2 (paper's generators, "
                     "alphabet {0,1}), each under the paper's 12 cost functions, 25 GB language cache")
    if name == "row1":
        t = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_examples.json")))["table1_row1"]
        inst = instances.Instance(t["alphabet"], t["pos"], t["neg"], "", 0, 0, "row1",
                                  (1, 1, 1, 1, 1), 30)
        return [inst], "Table 1 row 1 specification (10+12 strings), cost function (1,1,1,1,1)"
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--max-errors", type=int, default=0)
    ap.add_argument("--serving-requests", type=int, default=200,
                    help="requests per serving run (0 = skip the serving measurement)")
    ap.add_argument("--sequential", action="store_true",
                    help="time rei_solve per instance as the step instead of rei_solve_batch")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the batched solver's tuning (profiling runs: every launch the same kind)")
    ap.add_argument("--no-compare", action="store_true",
                    help="do not also time the other mode (batched vs sequential)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, copy this many MiB device to device once: a kernel of "
                         "known traffic that calibrates FETCH_SIZE / WRITE_SIZE counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the search is "
              "not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2305_18575_amd as rei

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    insts, desc = workload(args.workload)
    # the sweep mirrors the paper's 25 GB memory restriction and is timed per
    # solve (its instances are not batchable: costs up to 30 per constructor)
    cache = (25 << 30) if args.workload == "sweep" else (64 << 30)
    if args.workload == "sweep":
        args.sequential = True
    handles = []
    for it in insts:
        h = rei.Instance(it.alphabet, it.pos, it.neg, it.costs, it.max_cost, cache_bytes=cache)
        if args.max_errors:
            h.set_max_errors(args.max_errors)
        handles.append(h)
    stream = torch.cuda.current_stream().cuda_stream
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step_sequential():
        if args.workload == "sweep":
            # 48 solves with 25 GB caches do not fit HBM side by side: each
            # instance frees its cache after its solve
            out = []
            for h in handles:
                out.append(h.solve(stream))
                h.trim()
            return out
        return [h.solve(stream) for h in handles]

    def step_batch():
        return rei.solve_batch(handles, stream)

    step = step_sequential if args.sequential else step_batch

    def timed(fn, k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = [fn() for _ in range(k)]
        torch.cuda.synchronize()
        return out, time.perf_counter() - t

    for _ in range(args.warmup):
        step()
    tuned = None
    if not args.sequential and args.warmup and not args.no_tune:
        # launch shape of the batched solver, chosen by measurement (untimed)
        tuned = rei.tune_batch(handles, stream)
    # Python's cyclic collector scans every object torch created at import;
    # a full pass inside the timed region costs tens of milliseconds that
    # belong to no step.  Objects made so far are moved out of its reach.
    gc.collect()
    gc.freeze()

    def kernel_classes():
        out = {}
        for k, name in enumerate(rei.KERNEL_CLASSES):
            n = ms = units = 0
            for h in handles:
                a, b, c = h.kernel_stats(k)
                n += a
                ms += b
                units += c
            out[name] = {"launches": n, "ms": ms, "units": units}
        return out

    # One untimed step with the generator classes and the batched solver
    # timed names the dominant kernel; the timed steps then record events on
    # its launches only (events on a launch cost it a few microseconds).
    for h in handles:
        h.set_profiling(True)
    step()
    torch.cuda.synchronize()
    classes = kernel_classes()
    gen = {k: v for k, v in classes.items() if k.startswith("gen_") or k == "solve_batch"}
    dom = max(gen, key=lambda k: gen[k]["ms"])
    for h in handles:
        h.set_profiling_class(dom)
    results, elapsed = timed(step, args.steps)
    for h in handles:
        h.set_profiling(False)
    other = step_batch if args.sequential else step_sequential
    same = None
    other_value = None
    if not args.no_compare:
        other()
        other_results, other_elapsed = timed(other, args.steps)
        key = lambda r: (r.status, r.cost, r.regex, tuple(r.unique), tuple(r.candidates))
        same = all(key(a) == key(b) for ra, rb in zip(results, other_results) for a, b in zip(ra, rb))
        other_value = sum(r.total_unique for batch in other_results for r in batch) / other_elapsed

    uniq = sum(r.total_unique for batch in results for r in batch)
    value = uniq / elapsed
    solve_ms = sorted(r.seconds_solve * 1e3 for batch in results for r in batch)

    def pct(p):
        return solve_ms[min(len(solve_ms) - 1, int(p * len(solve_ms)))]

    # the dominant kernel's launches over the timed steps (HIP events)
    d = kernel_classes()[dom]
    avg_ms = d["ms"] / max(1, d["launches"])
    bytes_per_launch = PROBE_BYTES * d["units"] / max(1, d["launches"])
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = TRAFFIC_BYTES.get((args.workload, dom)) if not args.max_errors else None
    # the events a launch records also span its dispatch and completion; an
    # empty kernel launched the same way shows how much (context for
    # comparing with a kernel trace; achieved keeps the raw events)
    overhead_us = rei.timing_overhead_us()
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
                "algorithmic_bytes_per_launch": round(bytes_per_launch),
                "avg_launch_us": round(avg_ms * 1e3, 3), "event_overhead_us": round(overhead_us, 3),
                "launches": d["launches"],
                "candidates_per_launch": round(d["units"] / max(1, d["launches"]), 1)}

    serving_out = None
    if args.serving_requests:
        from paper_2305_18575_amd import serving as S
        specs = S.request_mix(2024, args.serving_requests)
        hs = S.stage(rei, specs)
        for h in hs:  # first solve allocates each instance's buffers
            h.solve(stream)
        base_arr = S.poisson_arrivals(2024, len(hs), 1.0)
        seq_res, _, _ = S.run_sequential(rei, hs, base_arr * 0.0, stream)
        # capacity of the sequential solver: requests per second of pure service
        t = time.perf_counter()
        for h in hs:
            h.solve(stream)
        capacity = len(hs) / (time.perf_counter() - t)
        runs = []
        for mult in (1.0, 2.0):
            qps = capacity * mult
            arr = base_arr / qps
            res, lat, ips = S.run_served(rei, hs, arr, budget=128 << 30)
            sres, slat, sips = S.run_sequential(rei, hs, arr, stream)
            runs.append({"qps": round(qps, 2), "served": {"instances_per_sec": round(ips, 2),
                                                          **{k: round(v, 3) for k, v in S.percentiles(lat).items()}},
                         "sequential": {"instances_per_sec": round(sips, 2),
                                        **{k: round(v, 3) for k, v in S.percentiles(slat).items()}},
                         "identical_results": all(S.same(a, b) for a, b in zip(res, seq_res))})
        serving_out = {"requests": len(hs), "mix": "60% plain / 30% large (max cost 10) / 10% single",
                       "sequential_capacity_per_sec": round(capacity, 2), "runs": runs}
        for h in hs:
            h.close()

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        t1 = time.perf_counter()
        cu = 0
        done = 0
        while time.perf_counter() - t1 < args.cpu_seconds and done < 40 * len(insts):
            it = insts[done % len(insts)]
            r = oracle.solve(it.alphabet, it.pos, it.neg, it.costs, it.max_cost, 1 << 40,
                             args.max_errors, threads)
            cu += sum(r.unique)
            done += 1
        ct = time.perf_counter() - t1
        cpu = {"value": round(cu / ct, 3), "unit": "languages/s", "cores": threads, "kind": "oracle",
               "sample": f"{done} solves of the same instance list in order ({ct:.1f} s)"}

    line = {
        "metric": "unique languages enumerated/sec",
        "value": round(value, 3),
        "unit": "languages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "instances_per_step": len(insts),
                   "mode": "rei_solve per instance" if args.sequential else "rei_solve_batch",
                   "batch_tuning": tuned},
        ("batched_value" if args.sequential else "sequential_value"):
            None if other_value is None else round(other_value, 3),
        "batched_over_sequential": None if other_value is None else
            round((other_value / value) if args.sequential else (value / other_value), 3),
        "identical_results": same,
        "instances_per_sec": round(len(insts) * args.steps / elapsed, 3),
        "time_to_minimal_regex_ms": {"mean": round(sum(solve_ms) / len(solve_ms), 4),
                                     "p50": round(pct(0.5), 4), "p99": round(pct(0.99), 4)},
        "roofline": roofline,
        "serving": serving_out,
        "cpu_baseline": cpu,
        # every generator class and the batched solver, from the untimed
        # profiled step before the timed ones
        "kernels_profiled_step": {k: {"launches": v["launches"], "ms": round(v["ms"], 3), "units": v["units"]}
                                  for k, v in classes.items()},
    }
    if args.workload == "sweep":
        # per cost function, as in the paper's cost-function comparison
        per = {}
        for it, r in zip(insts, results[-1]):
            d = per.setdefault(",".join(map(str, it.costs)), {"solves": 0, "ok": 0, "out_of_memory": 0,
                                                               "seconds": 0.0, "candidates": 0})
            d["solves"] += 1
            d["ok"] += r.status == "OK"
            d["out_of_memory"] += r.status == "OUT_OF_MEMORY"
            d["seconds"] = round(d["seconds"] + r.seconds_solve, 4)
            d["candidates"] += sum(r.candidates)
        line["per_cost_function"] = per
        tot_c = sum(sum(r.candidates) for r in results[-1])
        line["candidates_per_sec"] = round(tot_c / (elapsed / args.steps), 1)
    print(json.dumps(line), flush=True)
    for h in handles:
        h.close()


if __name__ == "__main__":
    main()
