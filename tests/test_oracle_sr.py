"""The oracle's DES against the paper's own iteration (Sec. 4 box, Sec. 5).

The literal CPU synchronous relaxation (Jacobi iterations over subdomains,
canonical empty neighbour histories first, repeat until no boundary history
changes, commit, continue with the pending random numbers) must reach the DES
trajectory bit for bit: consistency implies correctness (Sec. 4), and random
numbers are a presimulated list (Sec. 4, Sec. 5 "Subsequent steps").  Also:
the trajectory does not depend on the window length; a single subdomain
needs one iteration per window (it is the serial n-fold way); a window whose
iterations produce no boundary flip needs exactly one iteration.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _same(a, b):
    return (a["n_events"] == b["n_events"]
            and np.array_equal(a["log_tick"], b["log_tick"])
            and np.array_equal(a["log_site"], b["log_site"])
            and np.array_equal(a["log_sub"], b["log_sub"])
            and np.array_equal(a["spins"], b["spins"])
            and np.array_equal(a["carry"], b["carry"])
            and np.array_equal(a["sub_digest"], b["sub_digest"]))


SR_CASES = [
    # Lx, Ly, bx, by, T, h, window, horizon, tick_bits, rule, init
    (16, 16, 8, 8, 1.5, 0.0, 1.0, 6.0, 28, "metropolis", "random"),
    (16, 16, 4, 4, 3.0, 0.1, 0.5, 4.0, 28, "metropolis", "random"),
    (32, 16, 16, 8, 2.269, 0.05, 0.25, 3.0, 28, "metropolis", "random"),
    (12, 8, 4, 4, 2.5, -0.2, 1.0, 5.0, 28, "glauber", "random"),
    (16, 16, 16, 4, 2.0, 0.0, 1.0, 4.0, 28, "metropolis", "random"),  # wraps in x
    (16, 16, 8, 16, 2.0, 0.1, 1.0, 4.0, 28, "metropolis", "random"),  # wraps in y
    (16, 16, 8, 8, 2.0, 0.0, 1.0, 4.0, 4, "metropolis", "random"),    # coarse ticks: ties
    (16, 16, 4, 8, 3.0, 0.2, 0.5, 3.0, 6, "glauber", "random"),       # ties, 2 rows of blocks
    (32, 32, 16, 16, 1.0, 0.05, 2.0, 6.0, 28, "metropolis", "up"),
]


@pytest.mark.parametrize("Lx,Ly,bx,by,T,h,win,hor,tb,rule,init", SR_CASES)
def test_sr_reaches_des_trajectory(Lx, Ly, bx, by, T, h, win, hor, tb, rule, init):
    p = W.params(Lx, Ly, bx, by, T=T, h=h, window=win, horizon=hor, seed=21,
                 tick_bits=tb, rule=rule, init=init)
    a = oracle.des(p)
    b = oracle.sr(p)
    assert a["n_events"] > 0
    assert _same(a, b)
    assert np.array_equal(a["snap_M"], b["snap_M"])
    assert np.array_equal(a["snap_bond"], b["snap_bond"])
    # f == 0 in a window means no boundary flip: one iteration suffices
    assert np.all(b["g"][b["f"] == 0] == 1)
    assert np.all(b["g"] >= 1)
    if tb < 10:   # the coarse-tick cases must really contain simultaneous events
        assert np.any(np.diff(a["log_tick"]) == 0)


def test_trajectory_independent_of_window():
    base = W.params(32, 32, 8, 8, T=2.5, h=0.1, window=1.0, horizon=8.0, seed=5)
    ref = oracle.des(base)
    for win in (0.25, 1.0, 4.0, 3.0):
        p = dict(base, window=win)
        assert _same(ref, oracle.sr(p)), win


def test_single_subdomain_is_serial_nfold_way():
    p = W.params(16, 16, 16, 16, T=2.0, h=0.1, window=0.5, horizon=10.0, seed=3)
    b = oracle.sr(p)
    assert np.all(b["g"] == 1)
    assert _same(oracle.des(p), b)


def test_horizon_not_multiple_of_window():
    p = W.params(16, 16, 8, 8, T=2.5, h=0.0, window=0.75, horizon=5.1, seed=8)
    a, b = oracle.des(p), oracle.sr(p)
    assert _same(a, b)
    assert a["log_tick"].max() < a["horizon_ticks"]
    assert len(b["g"]) == 7


def test_event_log_invariants():
    p = W.params(32, 32, 8, 8, T=3.0, h=0.1, window=1.0, horizon=5.0, seed=2)
    a = oracle.des(p)
    # per subdomain, ticks strictly increase (one event per draw)
    for d in range(16):
        t = a["log_tick"][a["log_sub"] == d]
        assert np.all(np.diff(t) > 0)
    # log site belongs to its subdomain
    x, y = a["log_site"] % 32, a["log_site"] // 32
    assert np.array_equal((y // 8) * 4 + x // 8, a["log_sub"])
    # replaying the log from the initial state gives the final spins
    p0 = dict(p, horizon=0.0)
    s = oracle.des(p0)["spins"].reshape(-1).copy()
    for v in a["log_site"]:
        s[v] = -s[v]
    assert np.array_equal(s.reshape(32, 32), a["spins"])
    assert a["M"] == int(a["spins"].sum())
    assert int(a["sub_flips"].sum()) == a["n_events"]
