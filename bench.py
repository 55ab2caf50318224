#!/usr/bin/env python3
"""Benchmark of synchronous relaxation for the n-fold way Ising simulation on
one MI355X.

One step = the whole path over the medium workload: reset every lattice to
its initial spins (random +-1 from the seed, on the device), then relax and
commit every window up to the horizon, then read the observables -- for each
of the three temperatures (1024x1024 periodic, J=1, h=0.1, T in {1.5, 2.269,
3.0}, 4096 subdomains of 16x16, window 0.5, horizon 100).  Lattices live in
HBM for the whole run; the timed region holds only device work and the
host's window loop.

Printed: ONE JSON line with committed flips/s (value), iterations per window,
the relaxation kernel's roofline figure, the batched-vs-plain comparison over
uneven lattices, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue ceiling: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per
# SIMD every 4 cycles (16 lanes per cycle).
PEAK_WAVE_INSTR = 256 * 4 * 2.4e9 / 4
LDS_PEAK_GBPS = 256 * 128 * 2.4e9 / 1e9       # 128 B per clock per CU
# Algorithmic serial-chain work per processed event (wave instructions):
# class choice ~25, site choice ~40, re-classing 5 sites ~50, weight scan ~16,
# next-tick division ~30, record / draw ~25, amortised Philox + fixed-point log
# (64 lanes) ~10.
WAVE_INSTR_PER_EVENT = 200
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-persistent-only", action="store_true",
                    help="batch leg: only the persistent launch, no plain comparison (profiling the "
                         "persistent kernel: rocprofv3's kernel trace has crashed in the runtime while "
                         "eight host threads launched graphs)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-medium", action="store_true",
                    help="skip the headline leg (profiling the other legs alone)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sequential-only", action="store_true",
                    help="medium leg without the concurrent run (profiling: launches do not overlap)")
    ap.add_argument("--sweep-horizon", type=float, default=200.0)
    ap.add_argument("--temps", default=None, help="comma list, default all three")
    ap.add_argument("--horizon", type=float, default=100.0,
                    help="shorter horizons only for profiler runs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="run only a device-to-device copy of MB megabytes (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1 "
                          "(sharding across GPUs is designed, not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_cs_0405053_amd as sr
    import workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.no_medium:
        side = {}
        if not args.no_batch:
            side["batched_vs_plain"] = bench_batch(sr, W, stream, torch, plain=not args.batch_persistent_only)
        if not args.no_serve:
            side["serving"] = bench_serve(sr, W, stream, n=args.serve_requests)
        if not args.no_sweep:
            side["large_window_sweep"] = bench_window_sweep(sr, W, stream, torch, args.sweep_horizon)
        print(json.dumps(side), flush=True)
        return
    temps = W.MEDIUM_TEMPS if not args.temps else tuple(float(x) for x in args.temps.split(","))
    ps = [W.medium(T=T, horizon=args.horizon) for T in temps]
    # one HIP stream per lattice (default priority); the plain form's window
    # loops of the lattices run concurrently from one host thread each
    streams = [torch.cuda.Stream() for _ in ps]
    sims = [sr.Sim(dict(p, log_mode="digest"), stream=st) for p, st in zip(ps, streams)]
    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(max_workers=len(sims))

    def run_one(s):
        s.reset()
        g = s.run()
        o = s.observables()
        return (g, o, s.digests()[0])

    def step():                       # the lattices concurrently (the headline)
        return list(pool.map(run_one, sims))

    def step_sequential():            # one lattice after the other
        return [run_one(s) for s in sims]

    def timed(fn, what):
        for i in range(args.warmup):
            log(f"warmup {what} step {i}")
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = []
        for i in range(args.steps):
            res.append(fn())
            log(f"timed {what} step {i} done")
        torch.cuda.synchronize()
        return res, (time.perf_counter() - t0) / max(args.steps, 1)

    results_seq, dt_seq = timed(step_sequential, "sequential")
    if args.sequential_only:
        results, dt = results_seq, dt_seq
    else:
        results, dt = timed(step, "concurrent")
    seq_same = all(np.array_equal(a[2], b[2]) for a, b in zip(results_seq[-1], results[-1]))

    flips = sum(o["flips"] for g, o, d in results[-1])
    processed = sum(o["events_processed"] for g, o, d in results[-1])
    gs = np.concatenate([g for g, o, d in results[-1]])
    # per-launch kernel times from the sequential run, where launches do not
    # overlap (HIP events on each lattice's stream)
    launches = sum(o["relax_launches"] for g, o, d in results_seq[-1])
    processed_seq = sum(o["events_processed"] for g, o, d in results_seq[-1])
    runs = sum(o["subdomain_runs"] for g, o, d in results_seq[-1])
    relax_ms = sum(o["relax_ms"] for g, o, d in results_seq[-1])
    repeat_exact = all(np.array_equal(a[2], b[2]) for r in results for a, b in zip(r, results[0]))
    nsub = results[-1][0][1]["n_sub"]
    lnN = math.log(nsub)

    avg_launch_s = relax_ms / 1e3 / max(launches, 1)
    instr_per_launch = WAVE_INSTR_PER_EVENT * processed / max(launches, 1)
    achieved = instr_per_launch / avg_launch_s / 1e9
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(PEAK_WAVE_INSTR / 1e9, 1),
                "unit": "Gwave-instr/s", "frac": round(achieved * 1e9 / PEAK_WAVE_INSTR, 4),
                "traffic": None, "kernel": "relax_graph_kernel",
                "avg_launch_us": round(avg_launch_s * 1e6, 2), "launches_per_step": launches,
                "measured_on": "sequential run (launches do not overlap)",
                # aggregate rate of the concurrent step: algorithmic work / wall time
                "concurrent_frac": round(WAVE_INSTR_PER_EVENT * processed / dt / PEAK_WAVE_INSTR, 4)}
    traffic_file = os.path.join(ROOT, "profiles", "relax_kernel_medium_traffic.json")
    # the profiles describe the default workload (horizon 100, three temperatures)
    if os.path.exists(traffic_file) and args.horizon == 100.0 and args.temps is None:
        import hashlib
        with open(traffic_file) as f:
            tr = json.load(f)
        with open(os.path.join(ROOT, "paper_cs_0405053_amd", "csrc", "sr_kernels.hip"), "rb") as f:
            cur = hashlib.sha256(f.read()).hexdigest()
        # counters describe one version of the kernel: stale once it changed
        if tr.get("kernel_source_sha256") == cur:
            roofline["traffic"] = tr.get("bytes_per_launch")
        if roofline["traffic"]:
            gbps = roofline["traffic"] / avg_launch_s / 1e9
            roofline["hbm_GBps"] = round(gbps, 1)
            roofline["hbm_frac"] = round(gbps / HBM_PEAK_GBPS, 4)
        # issued instructions (SQ_INSTS_* counters of the same kernel version)
        # per launch, over this run's launch time: the measured counterpart
        # of the algorithmic rate above
        ins_file = os.path.join(ROOT, "profiles", "relax_kernel_medium_instructions.json")
        if os.path.exists(ins_file):
            with open(ins_file) as f:
                ins = json.load(f)
            if ins.get("kernel_source_sha256") == cur:
                per = ins["instructions_per_launch"]
                roofline["issued"] = {
                    "Ginstr_per_s": round(per / avg_launch_s / 1e9, 1),
                    "valu_frac": round(ins["valu_per_launch"] / avg_launch_s / PEAK_WAVE_INSTR, 4),
                    "salu_frac": round(ins["salu_per_launch"] / avg_launch_s / PEAK_WAVE_INSTR, 4),
                    "instr_per_processed_event": round(per * launches / max(processed_seq, 1), 1),
                    "source": "profiles/relax_kernel_medium_instructions.json"}
                lds = ins.get("lds")
                if lds:
                    lds_bytes = (lds["idx_active_cycles_per_launch"] - lds["bank_conflict_cycles_per_launch"]) * \
                        lds["bytes_per_active_cycle"]
                    lds_gbps = lds_bytes / avg_launch_s / 1e9
                    roofline["lds_GBps"] = round(lds_gbps, 1)
                    roofline["lds_frac"] = round(lds_gbps / LDS_PEAK_GBPS, 4)

    line = {
        "metric": "committed flips/s + relax iters/window, batched vs plain, bit-exact on 1 GPU",
        "value": round(flips / dt, 1),
        "unit": "flips/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "medium: 1024x1024 periodic Ising, J=1, h=0.1, "
                               f"T in {list(temps)}, Metropolis, random +-1 start, 4096 "
                               f"subdomains of 16x16, window 0.5, horizon {args.horizon:g}; "
                               + ("plain form, one lattice after the other" if args.sequential_only
                                  else "plain form, the lattices on concurrent HIP streams"),
                   "lattices": len(sims), "horizon": args.horizon, "window": 0.5,
                   "streams": 1 if args.sequential_only else len(sims)},
        "committed_flips_per_step": int(flips),
        "processed_per_committed": round(processed / max(flips, 1), 3),
        "events_per_subdomain_run": round(processed / max(runs, 1), 2),
        "relax_iters_per_window": round(float(gs.mean()), 3),
        "relax_iters_per_window_max": int(gs.max()),
        "ln_N": round(lnN, 3),
        "thm2_ceiling_C2": round(2 * math.e * 13 * lnN + 1, 1),
        "boundary_events_f": boundary_f(sims, 20),
        "thm1_ceiling_C2": round(2 * math.e * lnN + 1, 1),
        "bit_exact_repeat": bool(repeat_exact),
        "medium_sequential": {"flips_per_s": round(flips / dt_seq, 1), "ms_per_step": round(dt_seq * 1e3, 2),
                              "bit_exact_vs_concurrent": bool(seq_same)},
        "roofline": roofline,
    }

    # the same three lattices in one persistent launch per step
    def step_batched():
        for s in sims:
            s.reset()
        sr.batch_run(sims, stream=stream)
        return [(s.observables(), s.digests()[0]) for s in sims]

    for i in range(args.warmup):
        step_batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        rb = step_batched()
        log(f"timed batched step {i} done")
    torch.cuda.synchronize()
    dtb = (time.perf_counter() - t0) / max(args.steps, 1)
    flips_b = sum(o["flips"] for o, d in rb)
    same_b = all(np.array_equal(d, r[2]) for (o, d), r in zip(rb, results[-1]))
    line["medium_batched"] = {"flips_per_s": round(flips_b / dtb, 1), "ms_per_step": round(dtb * 1e3, 2),
                              "bit_exact_vs_plain": bool(same_b and flips_b == flips)}
    line["medium_plain"] = {"flips_per_s": line["value"], "ms_per_step": line["ms_per_step"]}
    pool.shutdown()

    for s in sims:
        s.close()

    if not args.no_batch:
        try:
            line["batched_vs_plain"] = bench_batch(sr, W, stream, torch, plain=not args.batch_persistent_only)
        except Exception as e:   # reported, never hidden
            line["batched_vs_plain"] = {"error": repr(e)}
    if not args.no_serve:
        try:
            line["serving"] = bench_serve(sr, W, stream, n=args.serve_requests)
        except Exception as e:
            line["serving"] = {"error": repr(e)}
    if not args.no_sweep:
        try:
            line["large_window_sweep"] = bench_window_sweep(sr, W, stream, torch, args.sweep_horizon)
        except Exception as e:
            line["large_window_sweep"] = {"error": repr(e)}

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sr, W, stream, temps)
        if not args.no_batch and isinstance(line.get("batched_vs_plain"), dict):
            line["batched_vs_plain"]["cpu_baseline"] = cpu_baseline_batch(sr, W, stream)

    print(json.dumps(line), flush=True)


def copy_calibration(mb):
    """A plain device copy of known size, to scale the HBM byte counters."""
    import torch
    n = mb * (1 << 20)
    x = torch.ones(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": 3}))


def bench_batch(sr, W, stream, torch, n=512, horizon=50.0, nstreams=8, plain=True):
    """Uneven lattices: one persistent launch vs the plain form (one lattice
    per launch sequence), the latter both one lattice after the other and
    with `nstreams` lattices in flight on concurrent streams.  plain=False:
    the persistent launch alone."""
    import threading
    import numpy as np
    ps = W.batch(n=n, horizon=horizon)
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    sims = [sr.Sim(p, stream=streams[i % nstreams]) for i, p in enumerate(ps)]
    log(f"batch: {n} lattices created")

    def digests():
        return [s.digests()[0].copy() for s in sims]

    if not plain:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sr.batch_run(sims, stream=stream)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        flips_b = sum(s.observables()["flips"] for s in sims)
        log(f"batch: batched done in {t_batch:.2f}s")
        for s in sims:
            s.close()
        return {"workload": f"{n} lattices (persistent launch only)",
                "committed_flips": int(flips_b), "batched_flips_per_s": round(flips_b / t_batch, 1)}

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.run()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    flips = sum(s.observables()["flips"] for s in sims)
    dig_plain = digests()
    log(f"batch: plain done in {t_plain:.2f}s")

    for s in sims:
        s.reset()

    def worker(k):
        for s in sims[k::nstreams]:
            s.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = [threading.Thread(target=worker, args=(k,)) for k in range(nstreams)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    torch.cuda.synchronize()
    t_conc = time.perf_counter() - t0
    same_conc = all(np.array_equal(a, b) for a, b in zip(dig_plain, digests()))
    log(f"batch: plain on {nstreams} streams done in {t_conc:.2f}s")

    for s in sims:
        s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sr.batch_run(sims, stream=stream)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    flips_b = sum(s.observables()["flips"] for s in sims)
    same = all(np.array_equal(a, b) for a, b in zip(dig_plain, digests()))
    log(f"batch: batched done in {t_batch:.2f}s")
    spins = sum(s.observables()["Lx"] * s.observables()["Ly"] for s in sims)
    for s in sims:
        s.close()
    return {"workload": f"{n} lattices, L uniform on multiples of 16 in [32,512], T~U[1,3.5], "
                        "h~U[-0.2,0.2], tuned block/window, horizon 50",
            "spins": int(spins), "committed_flips": int(flips),
            "plain_flips_per_s": round(flips / t_plain, 1),
            f"plain_{nstreams}_streams_flips_per_s": round(flips / t_conc, 1),
            "batched_flips_per_s": round(flips_b / t_batch, 1),
            "speedup": round(t_plain / t_batch, 3),
            f"speedup_vs_plain_{nstreams}_streams": round(t_conc / t_batch, 3),
            "bit_exact": bool(same and same_conc and flips == flips_b)}


def bench_window_sweep(sr, W, stream, torch, horizon):
    """The 4096x4096 low-temperature lattice (all up, T = 1, h = 0.05, 16384
    subdomains of 32x32) at three step sizes: committed flips/s and
    iterations per window for each, and the final state, which must be the
    same for every window (the trajectory does not depend on the step)."""
    import numpy as np
    out, ref = {}, None
    same = True
    for w in W.LARGE_WINDOWS:
        s = sr.Sim(dict(W.large(window=w, horizon=horizon), log_mode="digest"), stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = s.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        o = s.observables()
        dg = s.digests()[0].copy()
        if ref is None:
            ref = (dg, o["M"], o["flips"])
        else:
            same &= bool(np.array_equal(dg, ref[0]) and o["M"] == ref[1] and o["flips"] == ref[2])
        out[f"window_{w:g}"] = {"committed_flips_per_s": round(o["flips"] / dt, 1), "seconds": round(dt, 3),
                                "windows": int(o["windows"]), "iters_per_window": round(float(g.mean()), 3),
                                "processed_per_committed": round(o["events_processed"] / max(o["flips"], 1), 3),
                                "avg_launch_us": round(1e3 * o["relax_ms"] / max(o["relax_launches"], 1), 2)}
        log(f"window sweep W={w}: {o['flips']} flips in {dt:.2f}s")
        s.close()
    out["workload"] = (f"4096x4096 periodic, J=1, h=0.05, T=1.0, all +1 start, 16384 subdomains of 32x32, "
                       f"horizon {horizon:g}, windows {list(W.LARGE_WINDOWS)}")
    out["committed_flips"] = int(ref[2])
    out["identical_across_windows"] = bool(same)
    return out


def bench_serve(sr, W, stream, n=64, rate=200.0, budget_gib=96, wpr=8, n_check=3):
    """Continuous batching under a Poisson request stream: a request is
    submitted once its arrival time has passed, every pump is one scheduling
    round (admission by device footprint, one budgeted persistent step over
    all admitted lattices, retirement).  Latency = completion - nominal
    arrival, on the server's clock."""
    import numpy as np
    reqs = W.serve_stream(n=n, rate=rate)
    srv = sr.Server(hbm_budget=budget_gib << 30, windows_per_round=wpr, stream=stream)
    t0 = time.perf_counter()            # the server's clock starts at creation
    got, ids, nxt = {}, {}, 0
    while len(got) < n:
        now = time.perf_counter() - t0
        while nxt < n and reqs[nxt]["t_arrive"] <= now:
            p = {k: v for k, v in reqs[nxt].items() if k not in ("t_arrive", "req_id")}
            ids[srv.submit(p)] = nxt
            nxt += 1
        if srv.pump() == 0 and nxt < n:
            time.sleep(max(0.0, min(0.01, reqs[nxt]["t_arrive"] - (time.perf_counter() - t0))))
        for r in srv.poll():
            got[ids[r["req_id"]]] = r
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    bad = [i for i, r in got.items() if r["status"] != 0]
    lat = np.array([got[i]["t_done"] - reqs[i]["t_arrive"] for i in range(n)])
    svc = np.array([got[i]["t_done"] - got[i]["t_start"] for i in range(n)])
    flips = sum(int(r["flips"]) for r in got.values())
    # a few requests again, alone, on the plain path: must equal their in-mix result
    small = sorted(range(n), key=lambda i: reqs[i]["Lx"] * reqs[i]["horizon"])[:n_check]
    same = True
    for i in small:
        p = {k: v for k, v in reqs[i].items() if k not in ("t_arrive", "req_id")}
        s = sr.Sim(p, stream=stream)
        s.run()
        o = s.observables()
        d = int(np.sum(s.digests()[0], dtype=np.uint64))
        s.close()
        same &= (d, o["flips"], o["M"]) == (got[i]["digest"], got[i]["flips"], got[i]["M"])
    last_arrival = reqs[-1]["t_arrive"]
    return {"workload": f"{n} requests, Poisson arrivals at {rate:g} req/s, L log-uniform in "
                        "[64,2048] (multiple of 16), T~U[1,3.5], h~U[-0.2,0.2], horizon~U[10,100], "
                        f"tuned block/window, HBM budget {budget_gib} GiB, {wpr} windows per round",
            "requests": n, "failed": len(bad),
            "offered_req_per_s": round(n / max(last_arrival, 1e-9), 1),
            "served_req_per_s": round(n / wall, 2),
            "stable": bool(n / wall >= 0.9 * n / max(last_arrival, 1e-9)),
            "committed_flips_per_s": round(flips / wall, 1),
            "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
            "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
            "service_p50_s": round(float(np.percentile(svc, 50)), 3),
            "rounds": st["rounds"], "peak_active": st["peak_active"],
            "peak_gib": round(st["peak_bytes"] / 2**30, 2), "wall_s": round(wall, 2),
            "gpu_busy_frac": round(st["busy_s"] / max(wall, 1e-9), 3),
            "alone_equals_in_mix": bool(same), "alone_checked": n_check}


def boundary_f(sims, windows):
    """f of the paper's Theorem 1 (own events on boundary sites of one
    subdomain in one committed window, the largest over subdomains) for the
    first `windows` windows of each lattice, run one window at a time outside
    the timed steps."""
    fs = []
    for s in sims:
        s.reset()
        for _ in range(windows):
            if len(s.run(1)) == 0:
                break
            fs.append(s.observables()["last_f"])
    return {"mean": round(sum(fs) / max(len(fs), 1), 2), "max": max(fs) if fs else 0,
            "windows": len(fs)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sr, W, stream, temps, horizon=1.0):
    """The oracle DES (single thread by construction: global event order) on
    the first `horizon` time units of every temperature; the GPU's committed
    state at the same time is checked against it."""
    import numpy as np
    import oracle
    flips, secs, parity = 0, 0.0, True
    for T in temps:
        p = W.medium(T=T, horizon=horizon)
        t0 = time.perf_counter()
        ref = oracle.des(p, log=False)
        secs += time.perf_counter() - t0
        flips += ref["n_events"]
        s = sr.Sim(dict(p, log_mode="digest"), stream=stream)
        s.run()
        parity &= bool(np.array_equal(s.spins(), ref["spins"]) and
                       np.array_equal(s.digests()[0], ref["sub_digest"]))
        s.close()
        log(f"cpu baseline T={T}: {ref['n_events']} flips")
    return {"value": round(flips / secs, 1), "unit": "flips/s", "cores": 1, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"medium workload, each of T={list(temps)}, first {horizon} time units "
                      f"({flips} flips, {secs:.1f} s)",
            "gpu_matches_oracle_on_sample": parity}


def cpu_baseline_batch(sr, W, stream, n=512, horizon=0.5, check=3):
    """The oracle DES on every lattice of the batch workload over its first
    `horizon` time units, lattices in parallel on host threads (the C oracle
    runs outside the interpreter lock; each lattice is sequential by
    construction), with the blocks the tuner gives the GPU path (the
    trajectory does not depend on the window).  The GPU's state at the same
    time is checked against it on the first `check` lattices."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    ps = []
    for p in W.batch(n=n, horizon=horizon):
        bx, by, w = sr.tune(p)
        ps.append(dict(p, bx=bx, by=by, window=w))
    threads = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))))
    oracle.lib()                                   # load once, before the threads
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        refs = list(ex.map(lambda p: oracle.des(p, log=False), ps))
    secs = time.perf_counter() - t0
    flips = sum(r["n_events"] for r in refs)
    parity = True
    for p, ref in zip(ps[:check], refs[:check]):
        s = sr.Sim(dict(p, bx=0, by=0, window=0.0), stream=stream)
        s.run()
        parity &= bool(np.array_equal(s.spins(), ref["spins"]) and
                       np.array_equal(s.digests()[0], ref["sub_digest"]))
        s.close()
    log(f"cpu baseline batch: {flips} flips on {threads} threads in {secs:.1f} s")
    return {"value": round(flips / secs, 1), "unit": "flips/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"batch workload, all {n} lattices, first {horizon} time units ({flips} flips, {secs:.1f} s)",
            "gpu_matches_oracle_on_sample": parity}


if __name__ == "__main__":
    main()
