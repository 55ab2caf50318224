#!/usr/bin/env python3
"""Benchmark of synchronous relaxation for the n-fold way Ising simulation on
one MI355X: committed flips/s of the batched persistent form against the
plain one-lattice-per-launch form, bit-exact against the CPU oracle.

One step (the headline) = the batch workload: reset 512 independent periodic
2D lattices (L uniform on multiples of 16 in [32, 512], T ~ U[1, 3.5],
h ~ U[-0.2, 0.2], random +-1 starts, tuned blocks and windows) to their
initial spins on the device, then relax and commit every window of every
lattice up to horizon 50 in ONE persistent launch.  Lattices live in HBM for
the whole run; the timed region holds device work only.

Printed: ONE JSON line: committed flips/s of that step (value), the plain
form on 8 concurrent streams and one lattice after the other beside it, the
persistent kernel's roofline over the timed launches, iterations per window,
the medium workload (1024x1024 at three temperatures) in both forms with the
relaxation kernel's roofline, the step size of the paper's efficiency
analysis, the window sweep of the 4096x4096 lattice, continuous-batching
serving, every full run compared with the stored oracle results, and the CPU
oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))

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
# LDS: 128 bytes per cycle per CU
LDS_PEAK_GBPS = 256 * 128 * 2.4e9 / 1e9
METRIC = "committed flips/s + relax iters/window, batched vs plain, bit-exact on 1 GPU"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sha_file(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


KERNEL_SOURCES = ("sr_kernels.hip", "sr_device.h", "sr_internal.h", "sr_api.hip")


def kernel_source_sha():
    """SHA-256 of the persistent and relaxation kernels' sources and of the
    host code that sizes and launches them (checkpoint interval, tuner,
    grid), concatenated."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_cs_0405053_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_record(name):
    """A committed counter summary (profiles/<name>.json) if it was taken on
    the current kernel source, else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    return rec if rec.get("kernel_source_sha256") == kernel_source_sha() else None


def golden_check(family, sims, ids):
    """Compare finished simulations with the stored oracle results (SHA-256 of
    spins, per-subdomain digests, flips, carry; totals).  None if the family
    has no stored results."""
    import numpy as np
    import goldens as G
    if not G.available(family):
        return None
    recs = G.load(family)
    bad = []
    for cid, s in zip(ids, sims):
        rec = recs[cid]
        o = s.observables()
        dg, fl = s.digests()
        got = G.fingerprints(s.spins(), dg, fl, s.carry())
        tot = (o["flips"], o["M"], o["bond_sum"], f"{int(np.sum(dg, dtype=np.uint64)):016x}")
        if got != rec["sha256"] or tot != (rec["n_events"], rec["M"], rec["bond"], rec["digest"]):
            bad.append(cid)
    return {"compared": len(ids), "equal": len(ids) - len(bad), "first_bad": bad[:3]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparison of the batch")
    ap.add_argument("--no-medium", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-paper-step", action="store_true")
    ap.add_argument("--medium-steps", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--profile", choices=["batch", "medium-sequential", "medium-batched"], default=None,
                    help="run only one leg once, for a profiler (prints its JSON)")
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

    import torch
    import paper_cs_0405053_amd as sr
    import workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.profile:
        print(json.dumps(profile_leg(args.profile, sr, W, stream, torch)), flush=True)
        return

    line = {"metric": METRIC}
    line.update(bench_batch(sr, W, stream, torch, args))
    if not args.no_medium:
        try:
            line["medium"] = bench_medium(sr, W, stream, torch, args.medium_steps)
        except Exception as e:   # reported, never hidden
            line["medium"] = {"error": repr(e)}
    if not args.no_paper_step:
        try:
            line["paper_step_size"] = bench_paper_step(sr, W, stream)
        except Exception as e:
            line["paper_step_size"] = {"error": repr(e)}
    if not args.no_sweep:
        try:
            line["large_window_sweep"] = bench_window_sweep(sr, W, stream, torch)
        except Exception as e:
            line["large_window_sweep"] = {"error": repr(e)}
    if not args.no_serve:
        try:
            line["serving"] = bench_serve(sr, W, stream, n=args.serve_requests)
        except Exception as e:
            line["serving"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(sr, W, stream)
        if not args.no_medium:
            line["medium"]["cpu_baseline"] = cpu_baseline_medium(sr, W, stream)
    print(json.dumps(line), flush=True)


# ------------------------------------------------------------------ headline
def bench_batch(sr, W, stream, torch, args, nstreams=8):
    """The 512-lattice batch: K timed persistent launches (the headline), then
    the plain form over the same lattices once on `nstreams` concurrent
    streams and once one lattice after the other (graphs already built by an
    untimed plain run, whose extra time is reported as instantiation)."""
    import threading
    import numpy as np
    ps = W.batch()
    n = len(ps)
    sims = [sr.Sim(p, stream=stream) for p in ps]
    log(f"batch: {n} lattices created")

    def step():
        for s in sims:
            s.reset()
        sr.batch_run(sims, stream=stream)

    for i in range(args.warmup):
        step()
        log(f"warmup batched step {i}")
    torch.cuda.synchronize()
    # the persistent kernel's own duration: HIP events around each launch on
    # the launch stream, kept in every lattice's record (reset clears it, so
    # it is read after each step)
    kernel_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        kernel_ms.append(sims[0].observables()["relax_ms"])
        log(f"timed batched step {i} done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    obs = [s.observables() for s in sims]
    flips = sum(o["flips"] for o in obs)
    processed = sum(o["events_processed"] for o in obs)
    windows = sum(o["windows"] for o in obs)
    iters = sum(o["iterations"] for o in obs)
    spins = sum(o["Lx"] * o["Ly"] for o in obs)
    avg_launch_s = sum(kernel_ms) / 1e3 / max(len(kernel_ms), 1)
    dig_batched = [s.digests()[0].copy() for s in sims]
    gold = golden_check("batch", sims, [f"batch_{i:03d}" for i in range(n)])

    roof = {"bound": "alu", "kernel": "batch_kernel (persistent, 16x16 blocks)",
            "achieved": round(WAVE_INSTR_PER_EVENT * processed / avg_launch_s / 1e9, 2),
            "peak": round(PEAK_WAVE_INSTR / 1e9, 1), "unit": "Gwave-instr/s",
            "frac": round(WAVE_INSTR_PER_EVENT * processed / avg_launch_s / PEAK_WAVE_INSTR, 4),
            "traffic": None, "avg_launch_us": round(avg_launch_s * 1e6, 1),
            "processed_events_per_launch": int(processed),
            "algorithmic_wave_instr_per_event": WAVE_INSTR_PER_EVENT,
            "measured_on": "the timed persistent launches (HIP events on the launch stream)"}
    add_counters(roof, "batch_kernel_batch512", avg_launch_s, processed)

    out = {
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
        "config": {"workload": f"batch: {n} independent periodic 2D Ising lattices, L uniform on multiples "
                               "of 16 in [32,512], J=1, T~U[1,3.5], h~U[-0.2,0.2], Metropolis, random +-1 "
                               "starts, tuned 16x16 blocks and adapted windows, horizon 50; one persistent "
                               "launch per step",
                   "lattices": n, "spins": int(spins), "horizon": 50.0, "form": "batched persistent"},
        "committed_flips_per_step": int(flips),
        "processed_per_committed": round(processed / max(flips, 1), 3),
        "relax_iters_per_window": round(iters / max(windows, 1), 3),
        "windows_per_step": int(windows),
        "roofline": roof,
        "gpu_matches_oracle": gold,
    }
    if args.no_plain:
        for s in sims:
            s.close()
        return out

    # plain form: one lattice per launch sequence (window graphs), 8 host
    # threads on 8 streams; the first run builds each lattice's graphs
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    psims = [sr.Sim(p, stream=streams[i % nstreams]) for i, p in enumerate(ps)]

    def conc():
        def worker(k):
            for s in psims[k::nstreams]:
                s.reset()
                s.run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        th = [threading.Thread(target=worker, args=(k,)) for k in range(nstreams)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    t_first = conc()
    log(f"plain: first run on {nstreams} streams (graphs built) {t_first:.2f}s")
    t_conc = conc()
    log(f"plain: {nstreams} streams {t_conc:.2f}s")
    same_conc = all(np.array_equal(a, s.digests()[0]) for a, s in zip(dig_batched, psims))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for s in psims:
        s.reset()
        s.run()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    log(f"plain: one after the other {t_seq:.2f}s")
    same_seq = all(np.array_equal(a, s.digests()[0]) for a, s in zip(dig_batched, psims))
    for s in psims + sims:
        s.close()
    out["plain_8_streams"] = {"flips_per_s": round(flips / t_conc, 1), "seconds": round(t_conc, 3),
                              "bit_exact_vs_batched": bool(same_conc)}
    out["plain_sequential"] = {"flips_per_s": round(flips / t_seq, 1), "seconds": round(t_seq, 3),
                               "bit_exact_vs_batched": bool(same_seq)}
    out["plain_graph_instantiation_s"] = round(max(t_first - t_conc, 0.0), 3)
    out["speedup_vs_plain_8_streams"] = round(t_conc / dt, 3)
    out["speedup_vs_plain_sequential"] = round(t_seq / dt, 3)
    return out


def add_counters(roof, name, avg_launch_s, processed):
    """Counter-derived figures of the same kernel source (profiles/): HBM
    bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated), issued
    instructions per launch (SQ_INSTS_VALU / SALU) and LDS bytes per launch
    ((SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT) cycles x 128 B)."""
    tr = profile_record(f"{name}_traffic.json")
    if tr:
        roof["traffic"] = tr["bytes_per_launch"]
        roof["hbm_GBps"] = round(tr["bytes_per_launch"] / avg_launch_s / 1e9, 1)
        roof["hbm_frac"] = round(tr["bytes_per_launch"] / avg_launch_s / 1e9 / HBM_PEAK_GBPS, 4)
        roof["traffic_source"] = f"profiles/{name}_traffic.json"
    ins = profile_record(f"{name}_instructions.json")
    if ins:
        per = ins["instructions_per_launch"]
        roof["issued"] = {
            "Ginstr_per_s": round(per / avg_launch_s / 1e9, 1),
            "valu_frac": round(ins["valu_per_launch"] / avg_launch_s / PEAK_WAVE_INSTR, 4),
            "salu_frac": round(ins["salu_per_launch"] / avg_launch_s / PEAK_WAVE_INSTR, 4),
            "instr_per_processed_event": round(per / max(processed, 1), 1),
            "source": f"profiles/{name}_instructions.json"}
        lds = ins.get("lds")
        if lds:
            b = lds["bytes_per_launch"]
            roof["lds_GBps"] = round(b / avg_launch_s / 1e9, 1)
            roof["lds_frac"] = round(b / avg_launch_s / 1e9 / LDS_PEAK_GBPS, 4)


# ------------------------------------------------------------------ medium
def bench_medium(sr, W, stream, torch, steps):
    """1024x1024 at T in {1.5, 2.269, 3.0}, 4096 subdomains of 16x16, window
    0.5, horizon 100: plain form with the three lattices on concurrent
    streams, one after the other (the relaxation kernel's roofline: its
    launches do not overlap there), and batched in one persistent launch."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    ps = [W.medium(T=T) for T in W.MEDIUM_TEMPS]
    streams = [torch.cuda.Stream() for _ in ps]
    sims = [sr.Sim(dict(p, log_mode="digest"), stream=st) for p, st in zip(ps, streams)]
    pool = ThreadPoolExecutor(max_workers=len(sims))

    def one(s):
        s.reset()
        return s.run()

    def timed(fn, what):
        fn()                                 # untimed: builds graphs
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            fn()
        torch.cuda.synchronize()
        log(f"medium {what}: {steps} steps")
        return (time.perf_counter() - t) / steps

    dt_seq = timed(lambda: [one(s) for s in sims], "sequential")
    obs = [s.observables() for s in sims]
    launches = sum(o["relax_launches"] for o in obs)
    relax_ms = sum(o["relax_ms"] for o in obs)
    processed = sum(o["events_processed"] for o in obs)
    runs = sum(o["subdomain_runs"] for o in obs)
    flips = sum(o["flips"] for o in obs)
    gold = golden_check("medium", sims, [f"medium_T{T:g}" for T in W.MEDIUM_TEMPS])
    dig_plain = [s.digests()[0].copy() for s in sims]
    gs = np.concatenate([one(s) for s in sims])
    dt_conc = timed(lambda: list(pool.map(one, sims)), "concurrent")
    same_conc = all(np.array_equal(a, s.digests()[0]) for a, s in zip(dig_plain, sims))
    pool.shutdown()

    def batched():
        for s in sims:
            s.reset()
        sr.batch_run(sims, stream=stream)

    dt_b = timed(batched, "batched")
    b1 = sims[0].observables()               # the last step's one launch
    same_b = all(np.array_equal(a, s.digests()[0]) for a, s in zip(dig_plain, sims))
    b_launch_s = b1["relax_ms"] / 1e3 / max(b1["relax_launches"], 1)
    processed_b = sum(s.observables()["events_processed"] for s in sims)
    f_stats = boundary_f(sims, 20)
    for s in sims:
        s.close()

    avg_launch_s = relax_ms / 1e3 / max(launches, 1)
    achieved = WAVE_INSTR_PER_EVENT * processed / max(launches, 1) / avg_launch_s
    roof = {"bound": "alu", "kernel": "relax_graph_kernel<16,16,no-wrap>",
            "achieved": round(achieved / 1e9, 2), "peak": round(PEAK_WAVE_INSTR / 1e9, 1),
            "unit": "Gwave-instr/s", "frac": round(achieved / PEAK_WAVE_INSTR, 4), "traffic": None,
            "avg_launch_us": round(avg_launch_s * 1e6, 2), "launches_per_step": launches,
            "measured_on": "the sequential plain run (launches do not overlap)"}
    add_counters(roof, "relax_kernel_medium", avg_launch_s, processed / max(launches, 1))
    lnN = math.log(4096)
    return {
        "workload": "medium: 1024x1024 periodic Ising, J=1, h=0.1, T in [1.5, 2.269, 3.0], Metropolis, "
                    "random +-1 start, 4096 subdomains of 16x16, window 0.5, horizon 100",
        "committed_flips_per_step": int(flips),
        "plain_concurrent": {"flips_per_s": round(flips / dt_conc, 1), "ms_per_step": round(dt_conc * 1e3, 2),
                             "streams": len(sims), "bit_exact_vs_sequential": bool(same_conc)},
        "plain_sequential": {"flips_per_s": round(flips / dt_seq, 1), "ms_per_step": round(dt_seq * 1e3, 2)},
        "batched": {"flips_per_s": round(flips / dt_b, 1), "ms_per_step": round(dt_b * 1e3, 2),
                    "bit_exact_vs_plain": bool(same_b),
                    "roofline": {"bound": "alu", "kernel": "batch_kernel (persistent)",
                                 "achieved": round(WAVE_INSTR_PER_EVENT * processed_b / b_launch_s / 1e9, 2),
                                 "peak": round(PEAK_WAVE_INSTR / 1e9, 1), "unit": "Gwave-instr/s",
                                 "frac": round(WAVE_INSTR_PER_EVENT * processed_b / b_launch_s / PEAK_WAVE_INSTR, 4),
                                 "avg_launch_us": round(b_launch_s * 1e6, 1)}},
        "batched_vs_plain_concurrent": round(dt_conc / dt_b, 3),
        "processed_per_committed": round(processed / max(flips, 1), 3),
        "events_per_subdomain_run": round(processed / max(runs, 1), 2),
        "relax_iters_per_window": round(float(gs.mean()), 3),
        "relax_iters_per_window_max": int(gs.max()),
        "ln_N": round(lnN, 3),
        "boundary_events_f": f_stats,
        "roofline": roof,
        "gpu_matches_oracle": gold,
    }


def boundary_f(sims, windows):
    """f of the paper's Theorem 1 (own events on boundary sites of one
    subdomain in one iteration, the largest over subdomains and iterations)
    for the first `windows` windows of each lattice."""
    fs = []
    for s in sims:
        s.reset()
        for _ in range(windows):
            if len(s.run(1)) == 0:
                break
            fs.append(s.observables()["last_f"])
    return {"mean": round(sum(fs) / max(len(fs), 1), 2), "max": max(fs) if fs else 0,
            "windows": len(fs)}


# ------------------------------------------------------------------ Sec. 6
def bench_paper_step(sr, W, stream, windows=40):
    """The step size of the paper's efficiency analysis, T_max = ln N /
    (lambda |dG_i|) (Sec. 5), under which Theorems 1 and 2 bound f and g:
    for the medium lattice at T = 2.269 (N = 4096, |dG| = 60) and the large
    one (N = 16384, |dG| = 124), the first `windows` windows.  Reported: g, f
    and the committed events per subdomain and window, against ln N (the
    theorems' premise is about ln N events per PE per step); the theorem
    ceilings are given only where that premise holds within a factor 2."""
    out = {}
    cases = [("medium_T2.269", W.medium(T=2.269), 4096, 60), ("large", W.large(), 16384, 124)]
    for name, p, N, dG in cases:
        lnN = math.log(N)
        tmax = lnN / dG
        s = sr.Sim(dict(p, window=tmax, log_mode="digest"), stream=stream)
        gs, fs = [], []
        for _ in range(windows):
            g = s.run(1)
            if len(g) == 0:
                break
            gs.append(int(g[0]))
            fs.append(s.observables()["last_f"])
        o = s.observables()
        s.close()
        per_pe = o["flips"] / (N * max(len(gs), 1))
        holds = 0.5 <= per_pe / lnN <= 2.0
        e = {"window": round(tmax, 4), "windows": len(gs), "g_mean": round(sum(gs) / max(len(gs), 1), 2),
             "g_max": max(gs) if gs else 0, "f_mean": round(sum(fs) / max(len(fs), 1), 2),
             "f_max": max(fs) if fs else 0, "committed_events_per_pe_per_step": round(per_pe, 3),
             "ln_N": round(lnN, 3), "premise_within_2x": bool(holds)}
        if holds:
            e["thm1_f_ceiling_C2"] = round(2 * math.e * lnN + 1, 1)
            e["thm2_g_ceiling_C2"] = round(2 * math.e * 13 * lnN + 1, 1)
        out[name] = e
        log(f"paper step size {name}: g {e['g_mean']} f {e['f_mean']} events/PE/step {per_pe:.2f}")
    return out


# ------------------------------------------------------------------ large
def bench_window_sweep(sr, W, stream, torch, horizon=200.0):
    """The 4096x4096 low-temperature lattice (all up, T = 1, h = 0.05, 16384
    subdomains of 32x32) at three step sizes: committed flips/s and
    iterations per window for each; every window's final state is compared
    with the stored oracle result (the trajectory does not depend on the
    step)."""
    import numpy as np
    out, ref = {}, None
    same = True
    gold_all = []
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
        gold = golden_check("large", [s], ["large"]) if horizon == 200.0 else None
        if gold:
            gold_all.append(gold["equal"] == gold["compared"])
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
    out["gpu_matches_oracle_every_window"] = bool(gold_all and all(gold_all)) if gold_all else None
    return out


# ------------------------------------------------------------------ serving
def serve_run(sr, W, stream, n, rate, budget_gib=96, wpr=0):
    """One run of the Poisson request stream at `rate` req/s: a request is
    submitted once its arrival time has passed; the server keeps one
    persistent launch over the admitted lattices running and ends it at the
    next window boundaries when a request can join or a lattice finished
    (retire, admit by device footprint, relaunch).  Latency = completion -
    nominal arrival, on the server's clock."""
    import numpy as np
    reqs = W.serve_stream(n=n, rate=rate)
    srv = sr.Server(hbm_budget=budget_gib << 30, windows_per_round=wpr, stream=stream)
    t0 = time.perf_counter()
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
    lat = np.array([got[i]["t_done"] - reqs[i]["t_arrive"] for i in range(n)])
    flips = sum(int(r["flips"]) for r in got.values())
    last = reqs[-1]["t_arrive"]
    # bounded queue: the backlog does not grow over the run, i.e. the requests
    # that arrive last wait about as long as the first ones
    svc = np.array([got[i]["t_done"] - got[i]["t_start"] for i in range(n)])
    third = max(n // 3, 1)
    early, late = float(np.median(lat[:third])), float(np.median(lat[-third:]))
    failed = sum(1 for r in got.values() if r["status"] != 0)
    stable = bool(failed == 0 and late <= 2.0 * early + 0.25)
    return {"rate": rate, "requests": n, "failed": failed,
            "latency_first_third_p50_s": round(early, 3), "latency_last_third_p50_s": round(late, 3),
            "offered_req_per_s": round(n / max(last, 1e-9), 2), "served_req_per_s": round(n / wall, 2),
            "stable": stable, "committed_flips_per_s": round(flips / wall, 1),
            "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
            "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
            "service_p50_s": round(float(np.percentile(svc, 50)), 3),
            "rounds": st["rounds"], "peak_active": st["peak_active"], "restarts": st["restarts"],
            "peak_gib": round(st["peak_bytes"] / 2**30, 2), "wall_s": round(wall, 2),
            "gpu_busy_frac": round(st["busy_s"] / max(wall, 1e-9), 3)}, got, reqs


def bench_serve(sr, W, stream, n=256, rate=200.0, probe_n=96, probe_rates=(24.0, 16.0, 12.0, 8.0, 6.0, 4.0, 2.0)):
    """The 200 req/s stream (n requests, every result compared with the
    stored oracle results when n = 256), then the highest offered rate at
    which the queue stays bounded, from a short probe per rate."""
    import goldens as G
    main_run, got, reqs = serve_run(sr, W, stream, n, rate)
    log(f"serving {rate:g} req/s: served {main_run['served_req_per_s']} req/s, p99 {main_run['latency_p99_s']} s")
    gold = None
    if n == 256 and G.available("serve"):
        recs = G.load("serve")
        bad = []
        for i in range(n):
            r, rec = got[i], recs[f"serve_{i:03d}"]
            mine = (r["status"], r["flips"], r["M"], r["bond_sum"], f"{int(r['digest']):016x}")
            if mine != (0, rec["n_events"], rec["M"], rec["bond"], rec["digest"]):
                bad.append(i)
        gold = {"compared": n, "equal": n - len(bad), "first_bad": bad[:3]}
    main_run["gpu_matches_oracle"] = gold
    main_run["workload"] = (f"Poisson arrivals at {rate:g} req/s, L log-uniform in [64,2048] (multiple of 16), "
                            "T~U[1,3.5], h~U[-0.2,0.2], horizon~U[10,100], own seed, tuned block/window, "
                            "HBM budget 96 GiB, launches end at window boundaries when a request can join "
                            "or a lattice finished")
    best = None
    probes = []
    for r in probe_rates:
        pr, _, _ = serve_run(sr, W, stream, probe_n, r)
        probes.append({k: pr[k] for k in ("rate", "served_req_per_s", "stable", "latency_p50_s", "latency_p99_s")})
        log(f"serving probe {r:g} req/s: stable {pr['stable']}, p99 {pr['latency_p99_s']} s")
        if pr["stable"]:
            best = pr
            break
    main_run["highest_stable_rate"] = ({k: best[k] for k in ("rate", "requests", "served_req_per_s",
                                                             "latency_p50_s", "latency_p99_s")}
                                       if best else None)
    main_run["probes"] = probes
    return main_run


# ------------------------------------------------------------------ profiling legs
def profile_leg(which, sr, W, stream, torch):
    """One leg, run once, for rocprofv3 (kernel traces / counters)."""
    if which == "batch":
        sims = [sr.Sim(p, stream=stream) for p in W.batch()]
        sr.batch_run(sims, stream=stream)          # warm (first launch)
        for s in sims:
            s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sr.batch_run(sims, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        obs = [s.observables() for s in sims]
        r = {"leg": "batch", "launches": 2, "flips": sum(o["flips"] for o in obs),
             "processed": sum(o["events_processed"] for o in obs), "seconds": round(dt, 3)}
    else:
        sims = [sr.Sim(dict(W.medium(T=T), log_mode="digest"), stream=stream) for T in W.MEDIUM_TEMPS]
        if which == "medium-sequential":
            for s in sims:
                s.run()
        else:
            sr.batch_run(sims, stream=stream)
        torch.cuda.synchronize()
        obs = [s.observables() for s in sims]
        r = {"leg": which, "flips": sum(o["flips"] for o in obs),
             "processed": sum(o["events_processed"] for o in obs),
             "relax_launches": sum(o["relax_launches"] for o in obs)}
    for s in sims:
        s.close()
    return r


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


# ------------------------------------------------------------------ CPU oracle
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_batch(sr, W, stream, horizon=0.5, check=3):
    """The oracle DES on every lattice of the batch workload over its first
    `horizon` time units, lattices in parallel on host threads (the C oracle
    runs outside the interpreter lock; each lattice is sequential by
    construction), with the blocks the workload states.  The GPU's state at
    the same time is checked against it on the first `check` lattices."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    ps = []
    for p in W.batch(horizon=horizon):
        bx, by = W.tuned_block(p["Lx"], p["Ly"], p["T"])
        ps.append(dict(p, bx=bx, by=by, window=horizon))
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
            "sample": f"batch workload, all {len(ps)} lattices, first {horizon} time units "
                      f"({flips} flips, {secs:.1f} s)",
            "gpu_matches_oracle_on_sample": parity}


def cpu_baseline_medium(sr, W, stream, horizon=1.0):
    """The oracle DES (single thread by construction: global event order) on
    the first `horizon` time units of every medium temperature."""
    import numpy as np
    import oracle
    flips, secs, parity = 0, 0.0, True
    for T in W.MEDIUM_TEMPS:
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
    return {"value": round(flips / secs, 1), "unit": "flips/s", "cores": 1, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"medium workload, each of T={list(W.MEDIUM_TEMPS)}, first {horizon} time units "
                      f"({flips} flips, {secs:.1f} s)",
            "gpu_matches_oracle_on_sample": parity}


if __name__ == "__main__":
    main()
