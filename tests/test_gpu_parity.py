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


# ---- edge cases of the method
def test_zero_total_rate_subdomains():
    """T = 0.1: every uphill rate rounds to 0, so subdomains whose sites sit
    in zero-rate classes have Lambda = 0 (no pending event until a neighbour
    flip changes their halo).  A half-up / half-down start puts whole blocks
    there from time 0; the random start freezes into domains."""
    rates = oracle.rate_table(1.0, 0.05, 0.1)
    assert (rates == 0).sum() >= 4
    s0 = np.ones((64, 64), dtype=np.int8)
    s0[:, 32:] = -1
    s0[10:20, 5:9] = -1                       # a few unstable sites to start
    for init, spins in (("user", s0), ("random", None)):
        p = W.params(64, 64, 16, 16, T=0.1, h=0.05, window=0.5, horizon=6.0, seed=77,
                     init=init, init_spins=spins)
        check_against_oracle(p)


@pytest.mark.parametrize("J,h,T,rule", [(-1.0, 0.0, 1.5, "metropolis"), (-1.0, 0.3, 2.5, "glauber"),
                                        (-0.5, -0.1, 0.8, "metropolis")])
def test_antiferromagnetic_coupling(J, h, T, rule):
    p = W.params(48, 32, 16, 16, T=T, h=h, J=J, window=0.75, horizon=3.0, seed=501, rule=rule)
    check_against_oracle(p)


def _random_case(rng):
    # block sides 2..32 with bx*by <= 1024, 1..4 blocks per direction (lattice
    # sides >= 4), any tick resolution the library accepts, either rule, any
    # sign of J and h, windows from a few ticks to longer than the horizon
    while True:
        bx, by = int(rng.integers(2, 33)), int(rng.integers(2, 33))
        nbx, nby = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        Lx, Ly = bx * nbx, by * nby
        if bx * by <= 1024 and Lx >= 4 and Ly >= 4 and Lx * Ly <= 96 * 96:
            break
    tb = int(rng.choice([4, 6, 10, 16, 28]))
    horizon = float(rng.uniform(0.5, 3.0))
    window = float(rng.choice([rng.uniform(0.05, 0.5), rng.uniform(0.5, 2.0), 4.0]))
    window = max(window, 2.0 ** -tb)
    return W.params(Lx, Ly, bx, by, T=float(rng.uniform(0.7, 4.0)), h=float(rng.uniform(-0.5, 0.5)),
                    J=float(rng.choice([1.0, 1.0, 0.5, -1.0])), window=window, horizon=horizon,
                    seed=int(rng.integers(0, 2**63)), tick_bits=tb,
                    rule=["metropolis", "glauber"][int(rng.integers(0, 2))],
                    init=["random", "up"][int(rng.integers(0, 4)) == 0])


def test_randomised_small_lattices():
    """A seeded sweep over shapes, blocks, tick resolutions, windows and
    parameters; stops at the first case that differs from the oracle."""
    rng = np.random.default_rng(20260)
    for i in range(40):
        p = _random_case(rng)
        say("random case", i)
        check_against_oracle(p)


@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[8], CASES[10]])
def test_boundary_events_f_per_window(case):
    """f of Sec. 6 (most own events on boundary sites of one subdomain in one
    iteration, the largest over the window's iterations) for every window,
    against the literal CPU relaxation."""
    Lx, Ly, bx, by, T, h, win, hor, tb, rule, init = case
    p = W.params(Lx, Ly, bx, by, T=T, h=h, window=win, horizon=hor, seed=1234 + Lx + bx,
                 tick_bits=tb, rule=rule, init=init)
    srr = oracle.sr(p, log=False)
    sr = _sr()
    sim = sr.Sim(dict(p, log_mode="digest"))
    fs, gs = [], []
    while True:
        g = sim.run(1)
        if len(g) == 0:
            break
        gs.append(int(g[0]))
        fs.append(sim.observables()["last_f"])
    sim.close()
    assert gs == srr["g"].tolist()
    assert fs == srr["f"].tolist(), (fs, srr["f"].tolist())


def test_created_rate_tables_equal_oracle():
    sr = _sr()
    ps = [W.small(), *[W.medium(T=T, horizon=1.0) for T in W.MEDIUM_TEMPS]]
    ps += [W.params(32, 32, 16, 16, T=T, h=h, J=J, rule=r, window=1.0, horizon=1.0)
           for (J, h, T, r) in [(1.0, 0.1, 0.1, "metropolis"), (-1.0, 0.2, 1.3, "glauber"),
                                (0.0, 0.0, 1.0, "metropolis")]]
    for p in ps:
        s = sr.Sim(dict(p, log_mode="digest"))
        assert np.array_equal(s.rate_table(), oracle.rate_table(p["J"], p["h"], p["T"], p["rule"]))
        s.close()


def test_checkpoint_user_start_and_tuned_window():
    """A user start and a tuned step size survive sr_save / sr_load: the
    loaded simulation continues bit for bit, and reset works on it."""
    sr = _sr()
    s0 = W.random_spins(48, 48, 5, p_up=0.6)
    for p in (W.params(48, 48, 16, 16, T=2.2, h=0.1, window=0.5, horizon=5.0, seed=8, init="user",
                       init_spins=s0, log_mode="digest"),
              W.params(64, 64, 0, 0, T=2.6, h=-0.1, window=0.0, horizon=6.0, seed=9, log_mode="digest")):
        a = sr.Sim(p)
        a.run()
        b = sr.Sim(p)
        b.run(4)
        c = sr.Sim.load(b.save())
        assert c.observables()["window_ticks"] == b.observables()["window_ticks"]
        b.close()
        c.run()
        assert np.array_equal(a.spins(), c.spins())
        assert np.array_equal(a.digests()[0], c.digests()[0])
        assert np.array_equal(a.carry(), c.carry())
        c.reset()
        c.run()
        assert np.array_equal(a.spins(), c.spins())
        a.close()
        c.close()


# the wipe-the-slate step rule (Sec. 5): every window start drops the
# pending events, so the trajectory depends on the window; the oracle's DES
# and literal relaxation apply the same rule
WIPE_CASES = [
    (32, 32, 16, 16, 2.5, 0.1, 0.5, 4.0, 28, "metropolis", "random"),     # 16x16, no wrap
    (64, 64, 32, 32, 2.269, 0.05, 0.25, 2.0, 28, "metropolis", "random"),  # 32x32
    (32, 16, 8, 4, 2.5, -0.2, 1.0, 5.0, 28, "glauber", "random"),         # runtime shape
    (16, 16, 16, 16, 2.0, 0.1, 0.5, 5.0, 28, "metropolis", "random"),     # one subdomain, wraps
    (32, 32, 8, 8, 2.0, 0.0, 0.25, 3.1, 4, "metropolis", "random"),       # ties, ragged horizon
    (32, 32, 16, 16, 1.0, 0.05, 0.5, 6.0, 28, "metropolis", "up"),        # sparse
]


@pytest.mark.parametrize("Lx,Ly,bx,by,T,h,win,hor,tb,rule,init", WIPE_CASES)
def test_wipe_step_rule_matches_oracle(Lx, Ly, bx, by, T, h, win, hor, tb, rule, init):
    p = W.params(Lx, Ly, bx, by, T=T, h=h, window=win, horizon=hor, seed=4321 + Lx + bx,
                 tick_bits=tb, rule=rule, init=init, step="wipe")
    check_against_oracle(p)


def test_wipe_step_rule_one_launch_per_iteration(monkeypatch):
    monkeypatch.setenv("SR_NO_GRAPHS", "1")
    Lx, Ly, bx, by, T, h, win, hor, tb, rule, init = WIPE_CASES[0]
    p = W.params(Lx, Ly, bx, by, T=T, h=h, window=win, horizon=hor, seed=77,
                 tick_bits=tb, rule=rule, init=init, step="wipe")
    check_against_oracle(p)


def test_capacity_limit_shortens_the_step():
    # 64-wide edges at T = 3.5 over one 40-unit window collect ~1500 boundary
    # events, beyond the largest list (1024): the window is committed in
    # shorter steps, with the same events as the oracle (the continue rule's
    # trajectory does not depend on the step size); the wipe rule, whose
    # trajectory does, reports the limit
    sr = _sr()
    p = W.params(128, 32, 64, 16, T=3.5, h=0.0, window=40.0, horizon=40.0, seed=919, log_mode="digest")
    s = sr.Sim(p)
    w0 = s.observables()["window_ticks"]
    s.run()
    o = s.observables()
    ref = oracle.des(p, log=False)
    assert o["tick"] == o["horizon_ticks"]
    assert o["window_ticks"] < w0 and o["windows"] >= 2
    assert np.array_equal(s.spins(), ref["spins"])
    assert np.array_equal(s.digests()[0], ref["sub_digest"])
    assert np.array_equal(s.carry(), ref["carry"][:, :3])
    s.close()
    # the batched form: the overflowing lattice is finished by the plain path
    # with the shorter step
    s = sr.Sim(p)
    sr.batch_run([s])
    o = s.observables()
    assert o["tick"] == o["horizon_ticks"] and o["window_ticks"] < w0
    assert np.array_equal(s.spins(), ref["spins"])
    assert np.array_equal(s.digests()[0], ref["sub_digest"])
    s.close()
    s = sr.Sim(dict(p, step="wipe"))
    with pytest.raises(sr.SRError) as e:
        s.run()
    assert e.value.code == sr.SR_EOVERFLOW
    s.close()
