"""Benchmark: unique languages enumerated per second on one MI355X.

Default workload (the large configuration): four seeded specifications
(seeds 0..3) over the alphabet {0,1,2}, each with 20 positive and 20 negative
strings of length 0..10 drawn from a target expression of cost 14..18, cost
function (1,1,1,1,1), searched up to the target's cost with a 200 GB
language-cache budget.  A step solves the four with one rei_solve_batch call
on the current stream (word-width groups that the batched solver's tuner
sends to the per-chunk path run there, concurrently); the specifications are staged
(rei_create: host staging + upload) before the timed region, so their tables
are resident in HBM when timing starts.

value = unique languages enumerated in a step (sum over the instances and
their levels) / wall time of the step, over the timed steps (no timing
events on any launch).  The dominant kernel class's launch durations come
from as many steps again, run right after with HIP events on that class's
launches.

The JSON line also carries, per instance, the per-level unique and candidate
counts and the time to the minimal expression (rei_create + rei_solve, the
two parts separately); the dominant kernel's roofline figures against the
published HBM and integer-ALU peaks and against peaks measured in the same
run (copy, random table probes, bitwise ALU loop); the other configurations
(single instances as one batch, the 4096-instance batch replayed as one
graph launch, the serving sweep); and the CPU oracle's rate on a bounded
sample of the same workload with 1 thread and with the host's CPU share.
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
# 256 CUs x 64 integer lanes per clock x 2.4 GHz = 39.3 T 32-bit lane
# operations per second; each does 32 bitwise operations
VALU_PEAK_BITOPS = 256 * 64 * 2.4e9 * 32
# a dedup probe is one random access; the smallest HBM transaction is 64 B
PROBE_BYTES = 64

# HBM bytes per launch of the dominant kernel from FETCH_SIZE / WRITE_SIZE
# counter runs (rocprofv3 --pmc), calibrated on a plain copy of known size,
# by (workload, kernel class); stored, since a counter run is a separate
# profiler invocation.  The profile each figure comes from is named beside it.
# An entry is removed when its kernel changes.
TRAFFIC = {
    ("large", "gen_pieces"): (3310269, "profiles/large_workload_kernels.md (16-word launches of the timed and event steps)"),
    ("row1", "gen_concat"): (369546757, "profiles/table1_row1_kernels.md (launches of the timed and event steps)"),
    ("single", "solve_batch"): (57411487, "profiles/single_workload_kernels.md (both word widths' launches of the timed and event steps)"),
}


def infix_closure(strings):
    out = set()
    for w in strings:
        for i in range(len(w) + 1):
            for j in range(i, len(w) + 1):
                out.add(w[i:j])
    return out


def guide_size(inst) -> int:
    """S: entries of the guide table, all cuts w = u v of every infix w."""
    return sum(len(w) + 1 for w in infix_closure(list(inst.pos) + list(inst.neg)))


def workload(name: str):
    from paper_2305_18575_amd import instances
    if name == "large":
        out = [instances.large_instance(s) for s in range(4)]
        desc = ("large: alphabet {0,1,2}, target cost 14-18, 20+20 strings of length 0-10 (461-700 infixes, "
                "8-16 words per language), seeds 0-3, cost function (1,1,1,1,1), max_cost = target cost, "
                "200 GB language cache; 4 solves per step")
        return out, desc, 200 << 30
    if name == "single":
        out = []
        for costs in ((1, 1, 1, 1, 1), (1, 1, 5, 1, 2)):
            for seed in range(32):
                out.append(instances.single_instance(seed, costs))
        desc = ("single instance: alphabet {0,1}, target cost 10-14, 10+10 strings of length 0-7, "
                "seeds 0-31 x cost functions (1,1,1,1,1) and (1,1,5,1,2), 64 solves per step")
        return out, desc, 64 << 30
    if name == "plain":
        out = [instances.plain_instance(s) for s in range(200)]
        return out, "plain instance: alphabet {0,1}, target cost 1-8, 4+4 strings of length 1-5, seeds 0-199", 8 << 30
    if name == "batched":
        out = instances.batched_instances(0, 4096)
        return out, ("batched: 4096 instances from master seed 0, alphabet of 2-4 symbols, 2-16 positive and "
                     "2-16 negative strings of length 0-6, target cost 4-12, cost function (1,1,1,1,1), "
                     "max_cost = target cost"), 1 << 30
    if name == "wide":
        out = [instances.wide_instance(s, 12) for s in range(4)]
        return out, ("wide: 20+20 ternary strings of length <= 12 drawn as Type 1 benchmarks (1219-1234 "
                     "infixes, 32 words per language), seeds 0-3, max_cost 12"), 64 << 30
    if name == "sweep":
        out = []
        for kind, seeds in (("type1", (0, 2)), ("type2", (1, 2))):
            gen = instances.type1_instance if kind == "type1" else instances.type2_instance
            for seed in seeds:
                for costs in instances.PAPER_COST_FUNCTIONS:
                    out.append(gen(seed, costs=costs, max_cost=1000))
        return out, ("cost-function sweep: Type 1 seeds 0 and 2, Type 2 seeds 1 and 2 (paper's generators, "
                     "alphabet {0,1}), each under the paper's 12 cost functions, 25 GB language cache"), 25 << 30
    if name == "row1":
        t = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_examples.json")))["table1_row1"]
        inst = instances.Instance(t["alphabet"], t["pos"], t["neg"], "", 0, 0, "row1", (1, 1, 1, 1, 1), 30)
        return [inst], "Table 1 row 1 specification (10+12 strings), cost function (1,1,1,1,1)", 64 << 30
    raise SystemExit(f"unknown workload {name}")


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / (1 << 20), 1)
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "ram_gib": ram}


def cpu_share() -> int:
    """Threads the oracle may use: the CPUs this process may run on, capped
    by the thread count the environment allots (OMP_NUM_THREADS)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(insts, cache, seconds, max_errors=0):
    """The oracle as written, timed on this host: the workload's instances in
    order (whole passes, at least one instance) for about ``seconds``, once
    with one thread and once with the host's CPU share (the oracle splits
    each chunk of candidates across its threads)."""
    import oracle
    from paper_2305_18575_amd import instances as I

    def leg(threads):
        t1 = time.perf_counter()
        cu = done = 0
        while True:
            it = insts[done % len(insts)]
            cap = I.row_cap(cache, I.n_infixes(list(it.pos) + list(it.neg)))
            r = oracle.solve(it.alphabet, it.pos, it.neg, it.costs, it.max_cost, cap, max_errors, threads)
            cu += sum(r.unique)
            done += 1
            if time.perf_counter() - t1 >= seconds or done >= 40 * len(insts):
                break
        ct = time.perf_counter() - t1
        return {"value": round(cu / ct, 3), "cores": threads, "solves": done, "seconds": round(ct, 2)}

    t = cpu_share()
    one = leg(1)
    many = leg(t) if t > 1 else one
    return {"value": many["value"], "unit": "languages/s", "cores": t, "kind": "oracle",
            "sample": f"{many['solves']} solves of the workload's instances in order ({many['seconds']} s), "
                      f"threads = the host's CPU share",
            "single_thread": one, "host": host_info()}


def measured_peaks(rei):
    out = {}
    r, s = rei.measure_peak("copy", 4 << 30)
    out["copy_GBps"] = round(r / 1e9, 1)
    r, s = rei.measure_peak("probe", 4 << 30)
    out["probe_4GiB_table_Gps"] = round(r / 1e9, 2)
    r, s = rei.measure_peak("probe", 64 << 20)
    out["probe_64MiB_table_Gps"] = round(r / 1e9, 2)
    r, s = rei.measure_peak("probe_atomic", 4 << 30)
    out["probe_atomic_4GiB_table_Gps"] = round(r / 1e9, 2)
    r, s = rei.measure_peak("bitwise")
    out["bitwise_Tbitops"] = round(r * 32 / 1e12, 1)
    return out


def kernel_classes(rei, handles):
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


def timed(step, k):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = [step() for _ in range(k)]
    torch.cuda.synchronize()
    return out, time.perf_counter() - t


def roofline(rei, handles, insts, dom, peaks, workload_name, max_errors, overhead_us):
    """Figures of the dominant kernel class over the event steps (HIP events
    the library records at each of its launches' own start and end)."""
    d = kernel_classes(rei, handles)[dom]
    # the events' own span (an empty kernel's, measured in the same run) is
    # taken off each launch's: what is left agrees with the kernel trace
    overhead_s = overhead_us * 1e-6
    avg_events_s = d["ms"] / max(1, d["launches"]) * 1e-3
    avg_s = max(avg_events_s - overhead_s, 0.5 * avg_events_s)
    cand = d["units"] / max(1, d["launches"])
    bytes_per_launch = PROBE_BYTES * cand
    achieved = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    tr = TRAFFIC.get((workload_name, dom)) if not max_errors else None
    out = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": tr[0] if tr else None,
           "traffic_source": tr[1] if tr else None,
           "algorithmic_bytes_per_launch": round(bytes_per_launch), "candidates_per_launch": round(cand, 1),
           "avg_launch_us": round(avg_s * 1e6, 3), "avg_launch_us_with_events": round(avg_events_s * 1e6, 3),
           "launches": d["launches"],
           "probes_per_sec": round(cand / avg_s, 1) if avg_s > 0 else 0.0}
    if peaks:
        out["frac_of_measured_copy"] = round(achieved / peaks["copy_GBps"], 4)
        out["probe_frac_of_measured_4GiB_table"] = round(cand / avg_s / 1e9 / peaks["probe_4GiB_table_Gps"], 4)
    if dom in ("gen_concat", "gen_star"):
        # the fold over the guide table: per candidate S ANDs and S ORs of
        # single bits (concatenation: a cut's prefix in x and suffix in y;
        # star: one pass over cuts, shorter suffixes first)
        k = rei.KERNEL_CLASSES.index(dom)
        bits = sum(h.kernel_stats(k)[2] * 2 * guide_size(it) for h, it in zip(handles, insts))
        rate = bits / max(1, d["launches"]) / avg_s if avg_s > 0 else 0.0
        out["valu"] = {"bound": "alu", "achieved": round(rate / 1e12, 3), "peak": round(VALU_PEAK_BITOPS / 1e12, 1),
                       "unit": "T bit-terms/s", "frac": round(rate / VALU_PEAK_BITOPS, 6),
                       "bit_terms_per_launch": round(bits / max(1, d["launches"]))}
        if peaks:
            out["valu"]["frac_of_measured_bitwise"] = round(rate / 1e12 / peaks["bitwise_Tbitops"], 6)
    return out


def run_extra(rei, name, steps, stream):
    """Another configuration in the same run: its value and step time (a
    batch of the configuration's instances per step)."""
    insts, desc, cache = workload(name)
    hs = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in insts]
    rei.solve_batch(hs, stream)
    tuned = rei.tune_batch(hs, stream)
    res, el = timed(lambda: rei.solve_batch(hs, stream), steps)
    uniq = sum(r.total_unique for batch in res for r in batch)
    out = {"workload": desc, "value": round(uniq / el, 3), "unit": "languages/s",
           "ms_per_step": round(el / steps * 1e3, 3), "instances_per_sec": round(len(hs) * steps / el, 1),
           "batch_tuning": tuned}
    for h in hs:
        h.close()
    return out


def same_result(a, b) -> bool:
    return (a.status, a.cost, a.regex, a.unique, a.candidates) == (b.status, b.cost, b.regex, b.unique, b.candidates)


def run_batched_graph(rei, steps, stream):
    """The batched configuration three ways on the same 4096 instances: one
    rei_solve_batch call per step (one launch per word width), one replay of
    the captured graph per step (persistent launches, one graph launch), and
    one sequential pass of rei_solve; results compared."""
    insts, desc, cache = workload("batched")
    hs = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in insts]
    rei.solve_batch(hs, stream)
    tuned = rei.tune_batch(hs, stream)
    multi, el_multi = timed(lambda: rei.solve_batch(hs, stream), steps)
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    seq = [h.solve(stream) for h in hs]
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t
    g = rei.BatchGraph(hs)
    g.run(stream)  # first replay (untimed)
    graph, el_graph = timed(lambda: g.run(stream), steps)
    uniq = sum(r.total_unique for r in graph[-1])
    out = {"workload": desc, "value": round(uniq * steps / el_graph, 3), "unit": "languages/s",
           "mode": "captured graph, one replay per step",
           "instances_beside_the_graph": g.outside(),
           "ms_per_step": round(el_graph / steps * 1e3, 3),
           "instances_per_sec": round(len(hs) * steps / el_graph, 1),
           "multi_launch": {"value": round(uniq * steps / el_multi, 3), "ms_per_step": round(el_multi / steps * 1e3, 3),
                            "batch_tuning": tuned},
           "sequential": {"value": round(uniq / seq_s, 3), "ms_per_pass": round(seq_s * 1e3, 3)},
           "identical_results": all(same_result(a, b) and same_result(a, c)
                                    for a, b, c in zip(graph[-1], multi[-1], seq))}
    g.close()
    for h in hs:
        h.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-peaks", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other configurations measured beside the headline")
    ap.add_argument("--max-errors", type=int, default=0)
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="arrivals per serving load point (0 = skip the serving sweep)")
    ap.add_argument("--sequential", action="store_true",
                    help="time rei_solve per instance as the step instead of rei_solve_batch")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the batched solver's tuning (profiling runs: every launch the same kind)")
    ap.add_argument("--tune-save", default="",
                    help="after tuning, write the process's tuning tables to this JSON file (rei_tune_save); "
                         "a later run with REI_TUNE_FILE set to it and --no-tune repeats the same launch settings")
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
    insts, desc, cache = workload(args.workload)
    if args.workload == "sweep":
        args.sequential = True  # 48 solves with 25 GB caches: one at a time, trimmed after each
    # The process's first rei_create also pays one-time set-up (the HIP
    # runtime's first allocations, the library's code object, the tuning
    # file): a throwaway instance takes it, so that each instance's stage
    # time below is its own staging and upload.
    rei.Instance("01", ["0"], ["1"], (1, 1, 1, 1, 1), 4).close()
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
        out = []
        for h in handles:
            out.append(h.solve(stream))
            if args.workload == "sweep":
                h.trim()
        return out

    def step_batch():
        return rei.solve_batch(handles, stream)

    step = step_sequential if args.sequential else step_batch
    for _ in range(args.warmup):
        step()
    tuned = None
    if not args.sequential and args.warmup and not args.no_tune:
        # launch shapes chosen by measurement (untimed): the per-chunk path's
        # chunk sizes and concatenation shape per word width (timed on at
        # most 16 of the instances: the tuner solves each one 60 times), then
        # the batched solver's threads per instance and hand-off size
        tuned = {"grid": rei.tune_grid(handles[:16], stream)}
        tuned.update(rei.tune_batch(handles, stream))
        if args.tune_save:
            rei.tune_save(args.tune_save)
    # Python's cyclic collector scans every object torch created at import;
    # a full pass inside the timed region costs tens of milliseconds that
    # belong to no step.  Objects made so far are moved out of its reach.
    gc.collect()
    gc.freeze()

    # One untimed step with the generator classes and the batched solver
    # timed names the dominant kernel; the timed steps then record events on
    # its launches only (events on a launch cost it a few microseconds).
    for h in handles:
        h.set_profiling(True)
    step()
    torch.cuda.synchronize()
    classes = kernel_classes(rei, handles)
    gen = {k: v for k, v in classes.items() if k.startswith("gen_") or k == "solve_batch"}
    dom = max(gen, key=lambda k: gen[k]["ms"])
    for h in handles:
        h.set_profiling(False)
    # the events' own cost, measured on an empty kernel (its launches are
    # the last before the timed steps in a kernel trace of this run)
    event_overhead_us = rei.timing_overhead_us()
    results, elapsed = timed(step, args.steps)
    # The dominant class's launch durations: the same number of steps again,
    # with HIP events that each of its launches records at its own start and
    # end (on the launch's stream).  Events cost a launch several
    # microseconds, so the steps that give the headline carry none.
    for h in handles:
        h.set_profiling_class(dom)
    timed(step, args.steps)
    for h in handles:
        h.set_profiling(False)

    uniq = sum(r.total_unique for batch in results for r in batch)
    value = uniq / elapsed
    last = results[-1]
    ttm = sorted((r.seconds_stage + r.seconds_solve) * 1e3 for batch in results for r in batch)

    def pct(a, p):
        return a[min(len(a) - 1, int(p * len(a)))]

    per_instance = None
    if len(insts) <= 16:
        per_instance = [{"seed": it.seed, "ic": r.ic_size, "words": r.cs_words, "status": r.status,
                         "cost": r.cost, "regex": r.regex, "first_level": r.first_level,
                         "unique_per_level": r.unique, "candidates_per_level": r.candidates,
                         "stage_ms": round(r.seconds_stage * 1e3, 3), "solve_ms": round(r.seconds_solve * 1e3, 3),
                         "time_to_minimal_regex_ms": round((r.seconds_stage + r.seconds_solve) * 1e3, 3)}
                        for it, r in zip(insts, last)]

    peaks = None if args.no_peaks else measured_peaks(rei)
    roof = roofline(rei, handles, insts, dom, peaks, args.workload, args.max_errors, event_overhead_us)
    roof["event_overhead_us"] = round(event_overhead_us, 3)
    if peaks:
        roof["measured_peaks"] = peaks

    extras = None
    if not args.no_extras and args.workload == "large":
        extras = {"single": run_extra(rei, "single", 20, stream),
                  "batched": run_batched_graph(rei, 5, stream)}

    serving_out = None
    if args.serving_requests:
        from paper_2305_18575_amd import serving as S
        serving_out = S.sweep(rei, args.serving_requests, stream=stream)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(insts, cache, args.cpu_seconds, args.max_errors)

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
                   "cache_bytes": cache, "batch_tuning": tuned},
        "instances_per_sec": round(len(insts) * args.steps / elapsed, 3),
        "time_to_minimal_regex_ms": {"definition": "rei_create + rei_solve (stage + solve)",
                                     "mean": round(sum(ttm) / len(ttm), 4),
                                     "p50": round(pct(ttm, 0.5), 4), "p99": round(pct(ttm, 0.99), 4)},
        "per_instance": per_instance,
        "roofline": roof,
        "other_configs": extras,
        "serving": serving_out,
        "cpu_baseline": cpu,
        "kernels_profiled_step": {k: {"launches": v["launches"], "ms": round(v["ms"], 3), "units": v["units"]}
                                  for k, v in classes.items() if v["launches"]},
    }
    if args.workload == "sweep":
        per = {}
        for it, r in zip(insts, last):
            d = per.setdefault(",".join(map(str, it.costs)), {"solves": 0, "ok": 0, "out_of_memory": 0,
                                                               "seconds": 0.0, "candidates": 0})
            d["solves"] += 1
            d["ok"] += r.status == "OK"
            d["out_of_memory"] += r.status == "OUT_OF_MEMORY"
            d["seconds"] = round(d["seconds"] + r.seconds_solve, 4)
            d["candidates"] += sum(r.candidates)
        line["per_cost_function"] = per
    line["candidates_per_sec"] = round(sum(sum(r.candidates) for r in last) / (elapsed / args.steps), 1)
    print(json.dumps(line), flush=True)
    for h in handles:
        h.close()


if __name__ == "__main__":
    main()
