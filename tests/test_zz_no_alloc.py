"""The no-allocation batch step (sr_batch_step_static: the persistent
launch's queue and records in the library's fixed per-GPU array) against
sr_batch_step on the same inputs, bit for bit: two calls in a row, the second
with fewer and smaller lattices, so that it runs on the array the first call
left behind."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(s):
    o = s.observables()
    dg, fl = s.digests()
    return (s.spins().copy(), dg.copy(), fl.copy(), s.carry().copy(),
            (o["tick"], o["windows"], o["iterations"], o["flips"], o["M"], o["bond_sum"]))


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a[:4], b[:4])) and a[4] == b[4]


def _mix(n, Lmax, seed):
    rng = np.random.default_rng(seed)
    ps = []
    for i in range(n):
        L = int(16 * rng.integers(2, Lmax // 16 + 1))
        ps.append(W.params(L, L, 0, 0, T=float(rng.uniform(1.0, 3.5)), h=float(rng.uniform(-0.2, 0.2)),
                           window=float([0.0, 0.5, 1.0][i % 3]), horizon=float(rng.uniform(2.0, 4.0)),
                           seed=500 + 10 * seed + i, log_mode="digest"))
    return ps


@pytest.mark.parametrize("call,n,Lmax,budget", [(1, 8, 256, -1), (2, 3, 64, 2)])
def test_static_batch_step_equals_batch_step(call, n, Lmax, budget):
    import paper_cs_0405053_amd as sr
    ps = _mix(n, Lmax, seed=call)
    say(f"call {call}: {n} lattices, L <= {Lmax}, budget {budget}")
    ref = [sr.Sim(p) for p in ps]
    sr.batch_step(ref, budget)
    got = [sr.Sim(p) for p in ps]
    sr.batch_step_static(got, budget)
    for i, (a, b) in enumerate(zip(got, ref)):
        assert _same(_state(a), _state(b)), f"lattice {i} differs: {ps[i]}"
        assert a.observables()["windows"] >= 1
    # finish both the same way: the static step continues where it stopped
    sr.batch_step_static(got, -1)
    sr.batch_step(ref, -1)
    for i, (a, b) in enumerate(zip(got, ref)):
        assert _same(_state(a), _state(b)), f"lattice {i} differs after finishing: {ps[i]}"
        a.close()
        b.close()
