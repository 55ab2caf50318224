"""GPU path (HIP kernels behind the C ABI) against the CPU oracle, bit for bit.

For every case: final spins, the (tick, site) of every committed flip of every
subdomain, per-subdomain digests and flip counts, the carried random-stream
state (j, anchor, acc) at committed time, M and the bond sum -- all equal to
the oracle's DES; and the iteration count g of every window equal to the
literal CPU synchronous relaxation's (same Jacobi protocol: canonical
assumption, previous-iteration histories, stop when no boundary list changes).
"""
import sys

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


def check_against_oracle(p, with_sr_g=True, max_iters=2000):
    sr = _sr()
    say("case", {k: v for k, v in p.items() if k != "init_spins"})
    ref = oracle.des(p)
    sim = sr.Sim(dict(p, log_mode="full", max_iters=max_iters))
    g = sim.run()
    o = sim.observables()
    assert np.array_equal(sim.spins(), ref["spins"]), "final spins differ"
    nsub = o["n_sub"]
    for d in range(nsub):
        t, v = sim.log(d)
        sel = ref["log_sub"] == d
        rt, rv = ref["log_tick"][sel], ref["log_site"][sel]
        if not (np.array_equal(t, rt) and np.array_equal(v, rv)):
            n = min(len(t), len(rt))
            bad = np.nonzero((t[:n] != rt[:n]) | (v[:n] != rv[:n]))[0]
            i = int(bad[0]) if len(bad) else n
            raise AssertionError(f"subdomain {d}: first difference at event {i}: gpu "
                                 f"{t[i:i+3].tolist()} {v[i:i+3].tolist()} oracle "
                                 f"{rt[i:i+3].tolist()} {rv[i:i+3].tolist()} "
                                 f"(counts {len(t)} vs {len(rt)})")
    dg, fl = sim.digests()
    assert np.array_equal(fl, ref["sub_flips"])
    assert np.array_equal(dg, ref["sub_digest"])
    assert np.array_equal(sim.carry(), ref["carry"][:, :3])
    assert o["M"] == ref["M"] and o["bond_sum"] == ref["bond"]
    assert o["flips"] == ref["n_events"]
    assert o["tick"] == ref["horizon_ticks"]
    if with_sr_g:
        srr = oracle.sr(p)
        assert np.array_equal(g, srr["g"]), (g.tolist(), srr["g"].tolist())
    sim.close()
    return ref, g


CASES = [
    # Lx, Ly, bx, by, T, h, window, horizon, tick_bits, rule, init
    (16, 16, 8, 8, 1.5, 0.0, 1.0, 6.0, 28, "metropolis", "random"),      # 1 site / lane
    (32, 32, 16, 16, 3.0, 0.1, 0.5, 4.0, 28, "metropolis", "random"),    # 4 sites / lane
    (64, 64, 32, 32, 2.269, 0.05, 0.25, 2.0, 28, "metropolis", "random"),  # 16 sites / lane
    (32, 16, 8, 4, 2.5, -0.2, 1.0, 5.0, 28, "glauber", "random"),        # 32 sites, idle lanes
    (64, 32, 64, 16, 2.0, 0.0, 1.0, 2.0, 28, "metropolis", "random"),    # block spans x
    (32, 32, 16, 32, 2.0, 0.1, 1.0, 3.0, 28, "metropolis", "random"),    # block spans y
    (16, 16, 16, 16, 2.0, 0.1, 0.5, 5.0, 28, "metropolis", "random"),    # one subdomain
    (32, 32, 8, 8, 2.0, 0.0, 1.0, 4.0, 4, "metropolis", "random"),       # coarse ticks: ties
    (32, 16, 8, 8, 3.0, 0.2, 0.5, 3.0, 6, "glauber", "random"),          # ties, Lx/bx = 4
    (32, 32, 16, 16, 1.0, 0.05, 2.0, 8.0, 28, "metropolis", "up"),       # sparse, low T
    (48, 32, 16, 16, 2.5, 0.0, 0.75, 3.1, 28, "metropolis", "random"),   # ragged horizon
    (16, 32, 8, 16, 2.2, 0.1, 1.0, 3.0, 28, "metropolis", "random"),     # 2 subdomains / dir
    (48, 48, 12, 12, 2.5, 0.1, 0.5, 3.0, 28, "metropolis", "random"),    # 144 sites: last nibble partly used
    (36, 36, 12, 6, 2.0, -0.1, 1.0, 3.0, 28, "glauber", "random"),       # 72 sites, 2 / lane
    (16, 16, 2, 16, 2.5, 0.0, 1.0, 4.0, 28, "metropolis", "random"),     # 2-wide blocks
    (4, 4, 4, 4, 2.0, 0.1, 1.0, 6.0, 28, "metropolis", "random"),        # smallest lattice, wraps both ways
    (48, 48, 24, 24, 2.5, 0.1, 0.5, 2.0, 28, "metropolis", "random"),    # 576 sites: 9 of 16 nibbles used
    (36, 36, 18, 18, 2.0, 0.0, 1.0, 3.0, 28, "glauber", "random"),       # 324 sites, rows not lane-aligned
    (60, 30, 20, 6, 2.2, 0.05, 1.0, 3.0, 28, "metropolis", "random"),    # 120 sites, 2 / lane
]


@pytest.mark.parametrize("Lx,Ly,bx,by,T,h,win,hor,tb,rule,init", CASES)
def test_gpu_matches_oracle(Lx, Ly, bx, by, T, h, win, hor, tb, rule, init):
    p = W.params(Lx, Ly, bx, by, T=T, h=h, window=win, horizon=hor, seed=1234 + Lx + bx,
                 tick_bits=tb, rule=rule, init=init)
    check_against_oracle(p)


# one relaxation launch per iteration instead of graph replays (the library
# reads SR_NO_GRAPHS when a simulation is created): every kernel variant --
# 16x16 without and with wrap, 32x32, runtime shape
@pytest.mark.parametrize("case", [CASES[1], CASES[6], CASES[2], CASES[3]])
def test_plain_launches_without_graphs(monkeypatch, case):
    monkeypatch.setenv("SR_NO_GRAPHS", "1")
    Lx, Ly, bx, by, T, h, win, hor, tb, rule, init = case
    p = W.params(Lx, Ly, bx, by, T=T, h=h, window=win, horizon=hor, seed=1234 + Lx + bx,
                 tick_bits=tb, rule=rule, init=init)
    check_against_oracle(p)


def test_gpu_user_spins():
    s0 = W.random_spins(32, 32, 77, p_up=0.3)
    p = W.params(32, 32, 16, 16, T=2.0, h=0.1, window=1.0, horizon=3.0, seed=5,
                 init="user", init_spins=s0)
    check_against_oracle(p)


def test_small_workload_full_horizon():
    """64x64, h=0, T=1.5, 16 subdomains of 16x16, window 1.0, horizon 50."""
    check_against_oracle(W.small(), with_sr_g=True)


@pytest.mark.parametrize("T", W.MEDIUM_TEMPS)
def test_medium_workload_prefix(T):
    """1024x1024 with 4096 subdomains at its three temperatures, compared over
    the first time unit (the oracle's DES at full horizon takes too long)."""
    p = W.medium(T=T, horizon=1.0)
    check_against_oracle(p, with_sr_g=False)


def test_large_workload_window_sweep_prefix():
    """4096x4096, 32x32 blocks, all-up start at T=1: windows 0.25, 1, 4 give
    the same trajectory as the oracle over [0, 4)."""
    for win in W.LARGE_WINDOWS:
        p = W.large(window=win, horizon=4.0)
        check_against_oracle(p, with_sr_g=False)


def test_checkpoint_resume_bit_identical():
    sr = _sr()
    p = W.params(32, 32, 16, 16, T=2.5, h=0.1, window=0.5, horizon=6.0, seed=3,
                 log_mode="digest")
    a = sr.Sim(p)
    a.run()
    b = sr.Sim(p)
    b.run(5)
    blob = b.save()
    b.close()
    c = sr.Sim.load(blob)
    c.run()
    assert np.array_equal(a.spins(), c.spins())
    assert np.array_equal(a.digests()[0], c.digests()[0])
    assert np.array_equal(a.carry(), c.carry())


def test_overflow_regrow_keeps_result():
    sr = _sr()
    p = W.params(32, 32, 16, 16, T=3.0, h=0.0, window=2.0, horizon=4.0, seed=9,
                 log_mode="full")
    ref = sr.Sim(p)
    ref.run()
    tiny = sr.Sim(dict(p, hist_cap=1, wlog_cap=2))
    tiny.run()
    assert np.array_equal(ref.spins(), tiny.spins())
    assert np.array_equal(ref.digests()[0], tiny.digests()[0])
    for d in range(4):
        assert np.array_equal(ref.log(d)[0], tiny.log(d)[0])


def test_no_convergence_leaves_state_committed():
    sr = _sr()
    p = W.params(32, 32, 8, 8, T=3.0, h=0.0, window=1.0, horizon=3.0, seed=4,
                 max_iters=1)
    s = sr.Sim(p)
    before = s.spins().copy()
    with pytest.raises(sr.SRError) as e:
        s.run()
    assert e.value.code == sr.SR_ENOCONV
    assert np.array_equal(s.spins(), before)
    assert s.observables()["tick"] == 0
