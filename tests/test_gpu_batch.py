"""Persistent batched form (one launch, device work queue) against the plain
form and the oracle: bit-identical committed state for every lattice, the same
iteration counts, and the same result alone as inside a mix."""
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


def mix(n=12, horizon=3.0, seed=7):
    rng = np.random.default_rng(seed)
    ps = []
    for i in range(n):
        L = int(16 * rng.integers(2, 9))
        b = int([4, 8, 16][rng.integers(0, 3)])
        b = min(b, L)
        ps.append(W.params(L, L, b, b, T=float(rng.uniform(1.0, 3.5)), h=float(rng.uniform(-0.2, 0.2)),
                           window=float([0.25, 0.5, 1.0][rng.integers(0, 3)]),
                           horizon=float(horizon * rng.uniform(0.5, 1.0)), seed=100 + i,
                           log_mode="digest", rule=["metropolis", "glauber"][i % 2]))
    return ps


def state(s):
    o = s.observables()
    return (s.spins().copy(), s.digests()[0].copy(), s.digests()[1].copy(), s.carry().copy(),
            o["tick"], o["windows"], o["iterations"], o["flips"])


def same(a, b):
    return (np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
            and np.array_equal(a[3], b[3]) and a[4:] == b[4:])


def test_batched_equals_plain_and_oracle():
    sr = _sr()
    ps = mix()
    say("plain")
    plain = []
    for p in ps:
        s = sr.Sim(p)
        s.run()
        plain.append(state(s))
        s.close()
    say("batched")
    sims = [sr.Sim(p) for p in ps]
    sr.batch_run(sims)
    for i, (p, s) in enumerate(zip(ps, sims)):
        got = state(s)
        if not same(got, plain[i]):
            names = ["spins", "digests", "flips", "carry", "tick", "windows", "iterations", "total flips"]
            bad = [n for n, a, b in zip(names, got, plain[i])
                   if not (np.array_equal(a, b) if isinstance(a, np.ndarray) else a == b)]
            pp = {k: v for k, v in p.items() if k != "init_spins"}
            raise AssertionError(f"lattice {i} differs from its plain run in {bad}: {pp}; "
                                 f"batched {got[4:]} plain {plain[i][4:]}")
    for i in (0, 3, 7):
        ref = oracle.des(ps[i], log=False)
        assert np.array_equal(sims[i].spins(), ref["spins"])
        assert np.array_equal(sims[i].digests()[0], ref["sub_digest"])
    for s in sims:
        s.close()


@pytest.mark.parametrize("L,b,win,T", [(32, 16, 1.0, 3.0), (64, 16, 0.5, 2.5), (48, 8, 0.25, 3.5),
                                       (64, 4, 1.0, 2.0), (32, 8, 0.5, 1.5)])
def test_single_lattice_batch_equals_plain(L, b, win, T):
    sr = _sr()
    p = W.params(L, L, b, b, T=T, h=0.05, window=win, horizon=2.0, seed=31, log_mode="digest")
    a = sr.Sim(p)
    a.run()
    s = sr.Sim(p)
    sr.batch_run([s])
    ga, gs = state(a), state(s)
    assert same(gs, ga), (gs[4:], ga[4:])


def test_alone_equals_in_mix():
    sr = _sr()
    ps = mix(n=8, seed=11)
    target = ps[5]
    alone = sr.Sim(target)
    sr.batch_run([alone])
    a = state(alone)
    sims = [sr.Sim(p) for p in ps]
    sr.batch_run(sims)
    assert same(state(sims[5]), a)


def test_batch_resumes_partial_runs_and_reset():
    sr = _sr()
    ps = mix(n=6, seed=3)
    sims = [sr.Sim(p) for p in ps]
    for s in sims[:3]:
        s.run(2)                 # some lattices already advanced
    sr.batch_run(sims)
    ref = [sr.Sim(p) for p in ps]
    for s in ref:
        s.run()
    for a, b in zip(sims, ref):
        assert same(state(a), state(b))
    for s in sims:
        s.reset()
    sr.batch_run(sims)
    for a, b in zip(sims, ref):
        assert same(state(a)[:5], state(b)[:5])


def test_batch_repeats_bit_identical():
    """The same batch three times gives the same bits (the queue order and
    the XCD a task lands on must not matter)."""
    sr = _sr()
    ps = mix(n=16, seed=23, horizon=2.0)
    ref = None
    for rep in range(3):
        sims = [sr.Sim(p) for p in ps]
        sr.batch_run(sims)
        got = [state(s) for s in sims]
        if ref is None:
            ref = got
        else:
            assert all(same(a, b) for a, b in zip(got, ref)), rep
        for s in sims:
            s.close()


def test_batch_overflow_falls_back_and_matches():
    sr = _sr()
    p = W.params(32, 32, 16, 16, T=3.0, h=0.0, window=2.0, horizon=4.0, seed=9, log_mode="digest")
    ref = sr.Sim(p)
    ref.run()
    tiny = sr.Sim(dict(p, hist_cap=1, wlog_cap=2))
    other = sr.Sim(W.params(32, 32, 8, 8, T=2.0, h=0.1, window=0.5, horizon=2.0, seed=2,
                            log_mode="digest"))
    sr.batch_run([tiny, other])
    assert np.array_equal(ref.spins(), tiny.spins())
    assert np.array_equal(ref.digests()[0], tiny.digests()[0])


def test_batch_rejects_full_logs():
    sr = _sr()
    s = sr.Sim(W.params(32, 32, 8, 8, T=3.0, window=1.0, horizon=1.0, seed=4, log_mode="full"))
    with pytest.raises(sr.SRError) as e:
        sr.batch_run([s])
    assert e.value.code == sr.SR_EINVAL


def test_batch_no_convergence_reports():
    sr = _sr()
    p = W.params(32, 32, 8, 8, T=3.0, h=0.0, window=1.0, horizon=3.0, seed=4, max_iters=1,
                 log_mode="digest")
    s = sr.Sim(p)
    with pytest.raises(sr.SRError) as e:
        sr.batch_run([s])
    assert e.value.code == sr.SR_ENOCONV
    assert s.observables()["tick"] == 0


def test_batched_wipe_step_rule_equals_oracle():
    # the wipe rule inside the persistent kernel (window starts by the decider)
    sr = _sr()
    ps = [dict(p, step="wipe") for p in mix(n=6, horizon=3.0, seed=11)]
    sims = [sr.Sim(p) for p in ps]
    sr.batch_run(sims)
    for p, s in zip(ps, sims):
        ref = oracle.des(p, log=False)
        assert np.array_equal(s.spins(), ref["spins"]), p
        assert np.array_equal(s.digests()[0], ref["sub_digest"]), p
        assert np.array_equal(s.carry(), ref["carry"][:, :3]), p
        s.close()


@pytest.mark.parametrize("kernel", ["16x16", "generic"])
def test_both_persistent_kernels_equal_plain_and_oracle(monkeypatch, kernel):
    # lattices that all have 16x16 blocks without self-wrap can run on the
    # compile-time 16x16 persistent kernel; both kernels must give the plain
    # result (the library reads SR_BATCH_KERNEL at each batched launch)
    sr = _sr()
    rng = np.random.default_rng(21)
    ps = [W.params(L, L, 16, 16, T=float(rng.uniform(1.0, 3.5)), h=float(rng.uniform(-0.2, 0.2)),
                   window=[0.5, 1.0][i % 2], horizon=3.0, seed=900 + i, log_mode="digest")
          for i, L in enumerate([32, 48, 64, 96, 128, 160])]
    plain = []
    for p in ps:
        s = sr.Sim(p)
        s.run()
        plain.append(state(s))
        s.close()
    monkeypatch.setenv("SR_BATCH_KERNEL", kernel)
    sims = [sr.Sim(p) for p in ps]
    sr.batch_run(sims)
    for i, (p, s) in enumerate(zip(ps, sims)):
        assert same(state(s), plain[i]), (kernel, i)
    ref = oracle.des(ps[3], log=False)
    assert np.array_equal(sims[3].spins(), ref["spins"])
    assert np.array_equal(sims[3].digests()[0], ref["sub_digest"])
    for s in sims:
        s.close()


def test_reset_repeats_the_same_work():
    # a reset simulation starts over with the step size chosen at creation:
    # the same windows, iterations and re-simulated events come back, in the
    # batched and in the plain form (a tuned step size adapts during a run)
    sr = _sr()
    ps = [dict(p, window=0.0) for p in mix(n=6, seed=21)]
    sims = [sr.Sim(p) for p in ps]

    def work():
        return [(o["windows"], o["iterations"], o["events_processed"], o["window_ticks"])
                for o in (s.observables() for s in sims)]

    sr.batch_run(sims)
    first, st1 = work(), [state(s) for s in sims]
    for s in sims:
        s.reset()
    sr.batch_run(sims)
    assert work() == first
    assert all(same(state(s), a) for s, a in zip(sims, st1))
    for s in sims:
        s.close()
    s = sr.Sim(ps[0])
    g1 = s.run()
    o1 = s.observables()
    s.reset()
    g2 = s.run()
    o2 = s.observables()
    s.close()
    assert np.array_equal(g1, g2)
    assert (o1["events_processed"], o1["window_ticks"]) == (o2["events_processed"], o2["window_ticks"])
