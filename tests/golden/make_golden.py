#!/usr/bin/env python3
"""Write the stored oracle results of the full-size workloads.

Calls only the CPU oracle (``oracle.des``: the plain discrete-event
simulation that the converged relaxation reproduces, Sec. 4) on inputs from
``workloads.py``; nothing here touches the GPU library.  The trajectory does
not depend on the window (the window edge is not a break point, Sec. 5
"Subsequent steps"), so one DES run per lattice serves every window and the
tuned-window runs; the block does matter (it keys the random streams) and is
the one ``workloads.tuned_block`` states for tuned workloads.

Families (file ``<family>.json``):
  small    64x64, horizon 50
  medium   1024x1024, T in {1.5, 2.269, 3.0}, horizon 100
  large    4096x4096, 32x32 blocks, horizon 200
  batch    the 512 uneven lattices, horizon 50
  serve    the first 256 requests of the Poisson request stream

Usage: python tests/golden/make_golden.py [family ...] [--procs N]
Runs the lattices of a family in parallel processes, heaviest first.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import workloads as W  # noqa: E402
import goldens as G    # noqa: E402

SERVE_N = 256


def _clean(p):
    return {k: v for k, v in p.items() if k not in ("init_spins", "t_arrive", "req_id")}


def cases(family):
    """(id, params with an explicit block) of one family."""
    out = []
    if family == "small":
        out.append(("small", W.small()))
    elif family == "medium":
        for T in W.MEDIUM_TEMPS:
            out.append((f"medium_T{T:g}", W.medium(T=T)))
    elif family == "large":
        out.append(("large", W.large(window=1.0)))
    elif family == "batch":
        for i, p in enumerate(W.batch()):
            bx, by = W.tuned_block(p["Lx"], p["Ly"], p["T"])
            out.append((f"batch_{i:03d}", dict(p, bx=bx, by=by, window=1.0)))
    elif family == "serve":
        for i, p in enumerate(W.serve_stream(n=SERVE_N)):
            bx, by = W.tuned_block(p["Lx"], p["Ly"], p["T"])
            out.append((f"serve_{i:03d}", dict(_clean(p), bx=bx, by=by, window=1.0)))
    else:
        raise SystemExit(f"unknown family {family}")
    return out


def one(item):
    cid, p = item
    import oracle
    t0 = time.perf_counter()
    r = oracle.des(p, log=False)
    secs = time.perf_counter() - t0
    rec = {"id": cid, "params": _clean(p), "block": [p["bx"], p["by"]],
           "n_events": int(r["n_events"]), "M": int(r["M"]), "bond": int(r["bond"]),
           "digest": f"{int(r['digest']):016x}",
           "sha256": G.fingerprints(r["spins"], r["sub_digest"], r["sub_flips"], r["carry"][:, :3]),
           "oracle_seconds": round(secs, 2)}
    return rec


def run_family(family, procs):
    items = cases(family)
    # heaviest first (site-time), so the pool's tail is short
    items.sort(key=lambda it: -it[1]["Lx"] * it[1]["Ly"] * it[1]["horizon"])
    t0 = time.perf_counter()
    recs = []
    with ProcessPoolExecutor(procs) as ex:
        for rec in ex.map(one, items):
            recs.append(rec)
            print(f"{family}: {rec['id']} {rec['n_events']} events in {rec['oracle_seconds']} s "
                  f"({len(recs)}/{len(items)}, {time.perf_counter() - t0:.0f} s)", flush=True)
    recs.sort(key=lambda r: r["id"])
    head = {"generator": "tests/golden/make_golden.py", "family": family,
            "oracle": "oracle.des (plain DES, global tick order)"}
    with open(G.path(family) + ".tmp", "w") as f:     # one case per line
        f.write(json.dumps(head, sort_keys=True)[:-1] + ', "cases": [\n')
        f.write(",\n".join(json.dumps(r, sort_keys=True) for r in recs))
        f.write("\n]}\n")
    os.replace(G.path(family) + ".tmp", G.path(family))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("families", nargs="*", default=["small", "medium", "large", "batch", "serve"])
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    a = ap.parse_args()
    import oracle
    oracle.lib()
    for fam in a.families:
        run_family(fam, a.procs)


if __name__ == "__main__":
    main()
