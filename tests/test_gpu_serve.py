"""Serving (continuous batching) and the tuner.

Requests arrive while others run, are admitted by device footprint, share
persistent batch rounds, and each result must equal the same request run
alone.  A tuned simulation (block and first window from the tuner, step size
adapted after every window) must reach the oracle's trajectory bit for bit:
the step size is free in the Sec. 4 box and the trajectory does not depend
on it."""
import sys
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _sr():
    import paper_cs_0405053_amd as sr
    return sr


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def requests(n, seed, Lmax=192, hmax=3.0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = int(16 * rng.integers(4, Lmax // 16 + 1))
        out.append(W.params(L, L, 0, 0, T=float(rng.uniform(1.0, 3.5)), h=float(rng.uniform(-0.2, 0.2)),
                            window=0.0, horizon=float(rng.uniform(0.5, hmax)), seed=7000 + i,
                            log_mode="digest"))
    return out


def alone(sr, p):
    s = sr.Sim(p)
    s.run()
    o = s.observables()
    d = int(np.sum(s.digests()[0], dtype=np.uint64))
    s.close()
    return d, o["M"], o["bond_sum"], o["flips"]


def drain(srv, n, timeout=120.0):
    got = {}
    t0 = time.time()
    while len(got) < n:
        srv.pump()
        for r in srv.poll():
            got[r["req_id"]] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"only {len(got)} of {n} requests finished")
    return got


def test_served_results_equal_alone():
    sr = _sr()
    ps = requests(10, seed=1)
    srv = sr.Server(hbm_budget=8 << 30, windows_per_round=4)
    ids, got = [], {}
    for p in ps:
        ids.append(srv.submit(p))         # arrivals between rounds of the others
        srv.pump()
        for r in srv.poll():
            got[r["req_id"]] = r
    got.update(drain(srv, len(ps) - len(got)))
    st = srv.stats()
    srv.close()
    say("server stats", st)
    assert st["completed"] == len(ps) and st["failed"] == 0
    for rid, p in zip(ids, ps):
        r = got[rid]
        assert r["status"] == 0
        d, M, bond, flips = alone(sr, p)
        assert (r["digest"], r["M"], r["bond_sum"], r["flips"]) == (d, M, bond, flips), rid
        assert r["t_done"] >= r["t_start"] >= r["t_arrive"]


def test_budget_forces_queueing_and_stays_exact():
    sr = _sr()
    ps = requests(6, seed=2, Lmax=128)
    srv = sr.Server(hbm_budget=1 << 30, windows_per_round=2)
    info = []
    for p in ps:
        info.append(srv.submit(p))
    got = drain(srv, len(ps))
    st = srv.stats()
    srv.close()
    assert st["peak_bytes"] <= (1 << 30)
    for rid, p in zip(info, ps):
        d, M, bond, flips = alone(sr, p)
        assert (got[rid]["digest"], got[rid]["flips"]) == (d, flips)


def test_oversize_request_rejected():
    sr = _sr()
    srv = sr.Server(hbm_budget=1 << 20)
    with pytest.raises(sr.SRError) as e:
        srv.submit(W.params(512, 512, 0, 0, T=2.0, window=0.0, horizon=5.0, seed=1))
    assert e.value.code == sr.SR_ENOMEM
    srv.close()


def test_tuned_window_matches_oracle():
    sr = _sr()
    p = W.params(64, 64, 16, 16, T=2.5, h=0.1, window=0.0, horizon=6.0, seed=12, log_mode="full")
    s = sr.Sim(p)
    g = s.run()
    ref = oracle.des(dict(p, window=1.0))
    assert np.array_equal(s.spins(), ref["spins"])
    assert np.array_equal(s.digests()[0], ref["sub_digest"])
    for d in range(16):
        t, v = s.log(d)
        sel = ref["log_sub"] == d
        assert np.array_equal(t, ref["log_tick"][sel]) and np.array_equal(v, ref["log_site"][sel])
    assert len(g) > 0


def test_tuned_batch_equals_fixed_window_plain():
    sr = _sr()
    ps = requests(6, seed=5, Lmax=160)
    sims = [sr.Sim(p) for p in ps]
    sr.batch_run(sims)
    for p, s in zip(ps, sims):
        fixed = dict(p, window=0.5, bx=s.observables()["bx"], by=s.observables()["by"])
        d, M, bond, flips = alone(sr, fixed)
        o = s.observables()
        assert (int(np.sum(s.digests()[0], dtype=np.uint64)), o["M"], o["flips"]) == (d, M, flips)


def test_tuned_run_reports_every_window():
    """With a tuned step size the number of windows is not known ahead: the
    binding must return g for every committed window (and the C ABI must
    refuse a buffer when the count is unbounded)."""
    import ctypes as C
    sr = _sr()
    for p in requests(6, seed=9, Lmax=192):
        s = sr.Sim(p)
        first = s.observables()
        estimate = -(-first["horizon_ticks"] // first["window_ticks"])
        g = s.run()
        o = s.observables()
        assert o["tick"] == o["horizon_ticks"]
        assert len(g) == o["windows"] and int(g.sum()) == o["iterations"], (len(g), o)
        say("windows", o["windows"], "first-window estimate", estimate)
        s.close()
    s = sr.Sim(requests(1, seed=10)[0])
    buf = (C.c_int32 * 4)()
    assert sr.lib().sr_run_window(s.handle, -1, buf, None) == sr.SR_EINVAL
    s.close()


def test_arrival_joins_a_running_launch():
    # a short request submitted while a long one is on the device starts at
    # the long one's next window boundary and finishes long before it
    sr = _sr()
    long_p = W.params(512, 512, 0, 0, T=2.5, h=0.05, window=0.0, horizon=60.0, seed=4242, log_mode="digest")
    short_p = W.params(64, 64, 0, 0, T=2.0, h=0.1, window=0.0, horizon=1.0, seed=4243, log_mode="digest")
    srv = sr.Server(hbm_budget=8 << 30)
    a = srv.submit(long_p)
    srv.pump()                      # the long request's launch starts
    time.sleep(0.05)
    b = srv.submit(short_p)
    got = drain(srv, 2)
    st = srv.stats()
    srv.close()
    ra, rb = got[a], got[b]
    say("long", ra["t_start"], ra["t_done"], "short", rb["t_arrive"], rb["t_start"], rb["t_done"], st)
    assert ra["status"] == 0 and rb["status"] == 0
    assert rb["t_done"] < ra["t_done"]              # joined, did not wait for the long one
    assert st["rounds"] >= 2
    for rid, p in ((a, long_p), (b, short_p)):
        d, M, bond, flips = alone(sr, p)
        assert (got[rid]["digest"], got[rid]["M"], got[rid]["bond_sum"], got[rid]["flips"]) == (d, M, bond, flips)
