"""The GPU path on the full-size workloads, bit for bit against stored
oracle results (tests/golden/*.json, written by tests/golden/make_golden.py
from the CPU oracle's DES alone).

* medium: 1024x1024, 4096 subdomains, T in {1.5, 2.269, 3.0}, window 0.5,
  full horizon 100, plain form;
* large: 4096x4096, 16384 subdomains of 32x32, all up, T = 1, full horizon
  200, at each window 0.25, 1 and 4 (the trajectory does not depend on the
  window);
* batch: all 512 uneven lattices in one persistent launch, tuned blocks and
  windows, horizon 50;
* serve: the 256 requests of the Poisson request stream through the
  continuous-batching server.

Compared: SHA-256 of the final spins, of the per-subdomain event digests,
flip counts and carries (j, anchor, acc), and the totals (events, M, bond
sum, lattice digest); served requests report totals only.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import goldens as G  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _need(family):
    if not G.available(family):
        pytest.skip(f"no stored oracle results for {family} (run tests/golden/make_golden.py {family})")
    return G.load(family)


def _check(sim, rec, what):
    o = sim.observables()
    dg, fl = sim.digests()
    got = G.fingerprints(sim.spins(), dg, fl, sim.carry())
    bad = [k for k in got if got[k] != rec["sha256"][k]]
    tot = (o["flips"], o["M"], o["bond_sum"], f"{int(np.sum(dg, dtype=np.uint64)):016x}")
    want = (rec["n_events"], rec["M"], rec["bond"], rec["digest"])
    assert not bad and tot == want, f"{what}: differs in {bad}; totals {tot} vs oracle {want}"


@pytest.mark.parametrize("T", W.MEDIUM_TEMPS)
def test_medium_full_horizon_equals_oracle(T):
    import paper_cs_0405053_amd as sr
    rec = _need("medium")[f"medium_T{T:g}"]
    p = W.medium(T=T)
    assert rec["params"]["seed"] == p["seed"]
    say("medium", T)
    s = sr.Sim(dict(p, log_mode="digest"))
    g = s.run()
    assert len(g) == 200
    _check(s, rec, f"medium T={T}")
    s.close()


@pytest.mark.parametrize("win", W.LARGE_WINDOWS)
def test_large_full_horizon_equals_oracle(win):
    import paper_cs_0405053_amd as sr
    rec = _need("large")["large"]
    say("large window", win)
    s = sr.Sim(dict(W.large(window=win), log_mode="digest"))
    s.run()
    _check(s, rec, f"large window {win}")
    s.close()


def test_batch512_persistent_equals_oracle():
    import paper_cs_0405053_amd as sr
    recs = _need("batch")
    ps = W.batch()
    sims = [sr.Sim(p) for p in ps]
    say("batch: 512 lattices created")
    sr.batch_run(sims)
    for i, (p, s) in enumerate(zip(ps, sims)):
        rec = recs[f"batch_{i:03d}"]
        o = s.observables()
        assert [o["bx"], o["by"]] == rec["block"], (i, o["bx"], rec["block"])
        _check(s, rec, f"batch lattice {i}")
    for s in sims:
        s.close()


def test_serve256_results_equal_oracle():
    import paper_cs_0405053_amd as sr
    recs = _need("serve")
    reqs = W.serve_stream(n=256)
    srv = sr.Server(hbm_budget=96 << 30)
    ids = {}
    for i, r in enumerate(reqs):
        p = {k: v for k, v in r.items() if k not in ("t_arrive", "req_id")}
        ids[srv.submit(p)] = i
    got = {}
    while len(got) < len(reqs):
        srv.pump()
        for r in srv.poll():
            got[ids[r["req_id"]]] = r
    srv.close()
    say("serve: 256 results")
    bad = []
    for i in range(len(reqs)):
        r, rec = got[i], recs[f"serve_{i:03d}"]
        mine = (r["status"], r["flips"], r["M"], r["bond_sum"], f"{int(r['digest']):016x}", [r["bx"], r["by"]])
        want = (0, rec["n_events"], rec["M"], rec["bond"], rec["digest"], rec["block"])
        if mine != want:
            bad.append((i, mine, want))
    assert not bad, bad[:5]
