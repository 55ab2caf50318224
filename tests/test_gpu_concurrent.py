"""Several simulations driven at once from different host threads, each on
its own HIP stream (so their device work overlaps), give exactly the results
of the same simulations run one after the other, and the oracle's."""
import sys
import threading

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lattices():
    return [W.params(64, 64, 16, 16, T=T, h=0.1, window=0.5, horizon=4.0, seed=40 + i, log_mode="digest")
            for i, T in enumerate((1.5, 2.269, 3.0, 2.0))] + \
           [W.params(96, 96, 0, 0, T=2.5, h=-0.05, window=0.0, horizon=3.0, seed=50, log_mode="digest")]


def state(s):
    o = s.observables()
    return (s.spins().copy(), s.digests()[0].copy(), s.carry().copy(), o["flips"], o["windows"], o["iterations"])


def same(a, b):
    return all(np.array_equal(x, y) if isinstance(x, np.ndarray) else x == y for x, y in zip(a, b))


def test_concurrent_streams_equal_sequential_and_oracle():
    import torch
    import paper_cs_0405053_amd as sr
    ps = lattices()
    say("sequential")
    ref = []
    for p in ps:
        s = sr.Sim(p)
        s.run()
        ref.append(state(s))
        s.close()
    say("concurrent")
    streams = [torch.cuda.Stream() for _ in ps]
    sims = [sr.Sim(p, stream=st) for p, st in zip(ps, streams)]
    errors = []

    def drive(s):
        try:
            s.run()
        except Exception as e:          # reported by the main thread
            errors.append(repr(e))
    th = [threading.Thread(target=drive, args=(s,)) for s in sims]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i, (s, r) in enumerate(zip(sims, ref)):
        assert same(state(s), r), i
    o = oracle.des(dict(ps[2], window=0.5), log=False)
    assert np.array_equal(sims[2].spins(), o["spins"])
    assert np.array_equal(sims[2].digests()[0], o["sub_digest"])
    for s in sims:
        s.close()


def test_creation_errors_stay_per_thread():
    import paper_cs_0405053_amd as sr
    msgs = {}

    def bad(key, p):
        try:
            sr.Sim(p)
        except sr.SRError as e:
            msgs[key] = str(e)
    good = W.params(32, 32, 16, 16, T=2.0, window=0.5, horizon=1.0, seed=1, log_mode="digest")
    th = [threading.Thread(target=bad, args=("T", dict(good, T=-1.0))),
          threading.Thread(target=bad, args=("block", dict(good, bx=7, by=7)))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert "T > 0" in msgs["T"] and "bx" in msgs["block"], msgs
