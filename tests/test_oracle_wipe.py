"""Pins of the oracle's "wipe the slate" step rule (Sec. 5, the alternate
approach to subsequent steps): at every step start t_c > 0 each subdomain
drops its pending event and draws its next random pair afresh, its hazard
counted from t_c.

* The literal CPU relaxation with the rule reaches the DES with the rule bit
  for bit (consistency implies correctness, Sec. 4, whatever the steps).
* With no step start inside (0, horizon) the rule changes nothing, and with
  step starts it does change the trajectory (it depends on the window, unlike
  continuation).
* The paper's claim that the rule is unbiased for Ising dynamics (Poisson
  memorylessness): exact Boltzmann averages of 3x3 tori, and the J = 0
  closed forms (relaxation of m(t), stationary flip rate 2ab/(a+b)), hold
  with windows much shorter than the mean time between a subdomain's events.
  A rule that reused the dropped pair, kept its integrated hazard, or kept
  its old anchor would bias the flip rate by tens of percent here.

Tolerances as in the other physics pins: 3 standard errors, Bonferroni for
families of comparisons.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_physics import _enumerate, z_limit


def _same(a, b):
    return (a["n_events"] == b["n_events"]
            and np.array_equal(a["log_tick"], b["log_tick"])
            and np.array_equal(a["log_site"], b["log_site"])
            and np.array_equal(a["log_sub"], b["log_sub"])
            and np.array_equal(a["spins"], b["spins"])
            and np.array_equal(a["carry"], b["carry"])
            and np.array_equal(a["sub_digest"], b["sub_digest"]))


WIPE_CASES = [
    # Lx, Ly, bx, by, T, h, window, horizon, tick_bits, rule
    (16, 16, 8, 8, 1.5, 0.0, 1.0, 6.0, 28, "metropolis"),
    (16, 16, 4, 4, 3.0, 0.1, 0.25, 3.0, 28, "metropolis"),
    (12, 8, 4, 4, 2.5, -0.2, 0.5, 4.1, 28, "glauber"),       # ragged last step
    (16, 16, 16, 4, 2.0, 0.0, 1.0, 4.0, 28, "metropolis"),   # wraps in x
    (16, 16, 8, 8, 2.0, 0.0, 0.5, 4.0, 4, "metropolis"),     # coarse ticks: ties, and events at step starts
]


@pytest.mark.parametrize("Lx,Ly,bx,by,T,h,win,hor,tb,rule", WIPE_CASES)
def test_wipe_sr_reaches_wipe_des(Lx, Ly, bx, by, T, h, win, hor, tb, rule):
    p = W.params(Lx, Ly, bx, by, T=T, h=h, window=win, horizon=hor, seed=31,
                 tick_bits=tb, rule=rule, step="wipe")
    a, b = oracle.des(p), oracle.sr(p)
    assert a["n_events"] > 0
    assert _same(a, b)
    assert np.array_equal(a["snap_M"], b["snap_M"])
    assert np.all(b["g"][b["f"] == 0] == 1)


def test_wipe_without_step_starts_is_continuation():
    p = W.params(16, 16, 8, 8, T=2.5, h=0.1, window=4.0, horizon=4.0, seed=5)
    assert _same(oracle.des(p), oracle.des(dict(p, step="wipe")))
    p = dict(p, window=10.0)
    assert _same(oracle.des(p), oracle.des(dict(p, step="wipe")))


def test_wipe_trajectory_depends_on_window():
    base = W.params(16, 16, 8, 8, T=2.5, h=0.1, window=1.0, horizon=4.0, seed=5, step="wipe")
    a = oracle.des(base)
    b = oracle.des(dict(base, window=0.5))
    c = oracle.des(dict(base, step="continue"))
    assert not np.array_equal(a["log_tick"], b["log_tick"])
    assert not np.array_equal(a["log_tick"], c["log_tick"])
    # the first step is the same under both rules
    first = a["log_tick"] < 2**28
    assert np.array_equal(a["log_tick"][first], c["log_tick"][c["log_tick"] < 2**28])


def test_wipe_draws_one_pair_per_step_start():
    # every step start skips exactly the pending pair: j = events + starts
    p = W.params(16, 16, 8, 8, T=2.0, h=0.0, window=0.5, horizon=3.0, seed=9, step="wipe")
    a = oracle.des(p)
    starts = 5                                   # 0.5, 1.0, ..., 2.5
    assert np.array_equal(a["carry"][:, 0], a["sub_flips"] + starts)
    # the pending event of a wiped subdomain never precedes its step start
    late = a["carry"][:, 1] >= 5 * 2**27
    assert np.all(a["carry"][late, 3] > a["carry"][late, 1])


@pytest.mark.parametrize("L,bx,by,J,h,T,rule,win", [
    (3, 3, 3, 1.0, 0.0, 2.0, "metropolis", 0.1),
    (3, 1, 3, 1.0, 0.3, 1.5, "glauber", 0.05),
])
def test_wipe_des_matches_exact_enumeration(L, bx, by, J, h, T, rule, win):
    exact = _enumerate(L, J, h, T)
    reps = []
    for rep in range(24):
        p = W.params(L, L, bx, by, T=T, h=h, J=J, window=win, horizon=1050.0,
                     seed=1000 * rep + 23, rule=rule, step="wipe")
        r = oracle.des(p, log=False, burn=50.0)
        n = r["int_ticks"]
        E = (-J * r["int_bond"] - h * r["int_M"]) / n
        reps.append((E, r["int_M"] / n, r["int_M2"] / n, r["int_absM"] / n))
    reps = np.array(reps)
    mean = reps.mean(0)
    se = reps.std(0, ddof=1) / math.sqrt(len(reps))
    from scipy.stats import f as fdist, norm
    keys = ["E", "M", "M2", "absM"]
    for i, key in enumerate(keys):
        assert abs(mean[i] - exact[key]) < 3 * se[i] + 1e-12, (key, mean[i], exact[key], se[i])
    n, q = reps.shape
    d = mean - np.array([exact[k] for k in keys])
    S = np.cov(reps, rowvar=False)
    F = n * float(d @ np.linalg.solve(S, d)) * (n - q) / (q * (n - 1))
    assert F < fdist.isf(2 * norm.sf(3.0), q, n - q), (F, d.tolist())


@pytest.mark.parametrize("h,T,rule", [(0.2, 1.0, "metropolis"), (-0.3, 2.0, "glauber")])
def test_wipe_zero_coupling_closed_forms(h, T, rule):
    L = 64
    rt = oracle.rate_table(0.0, h, T, rule) / 2.0**28
    a, b = rt[0], rt[5]
    m_eq = (b - a) / (a + b)
    N = L * L
    # 8x8 blocks: a subdomain's total rate is ~64 a..64 b per time unit, so a
    # 0.02 window holds about one of its events or fewer
    win = 0.02
    p = W.params(L, L, 8, 8, J=0.0, T=T, h=h, window=win, horizon=5.0, seed=4,
                 init="up", rule=rule, step="wipe")
    r = oracle.des(p, log=False)
    idx = np.arange(0, len(r["snap_M"]), 12)              # every 0.24 time units
    lim = z_limit(len(idx))
    for k in idx:
        t = k * win
        mt = m_eq + (1.0 - m_eq) * math.exp(-(a + b) * t)
        sig = math.sqrt(max(1 - mt * mt, 1e-12) / N)
        assert abs(r["snap_M"][k] / N - mt) < lim * sig + 1e-12, (t, r["snap_M"][k] / N, mt)
    p2 = W.params(L, L, 8, 8, J=0.0, T=T, h=h, window=win, horizon=40.0, seed=5,
                  rule=rule, step="wipe")
    r2 = oracle.des(p2)
    late = r2["log_tick"] >= 10 * 2**28
    rate = late.sum() / (N * 30.0)
    want = 2 * a * b / (a + b)
    assert abs(rate - want) < 3 * math.sqrt(want / (N * 30.0)), (rate, want)


@pytest.mark.parametrize("tb", [28, 5])
def test_wipe_event_order(tb):
    # the DES emits events in tick order, each subdomain's strictly
    # increasing, and no event falls on a step start (the wipe there drops
    # the pending event and a fresh one is at least one tick later)
    win = 0.25
    p = W.params(16, 16, 8, 8, T=2.0, h=0.1, window=win, horizon=4.0, seed=13,
                 tick_bits=tb, step="wipe")
    a = oracle.des(p)
    assert np.all(np.diff(a["log_tick"]) >= 0)
    for d in range(4):
        t = a["log_tick"][a["log_sub"] == d]
        assert np.all(np.diff(t) > 0)
    wt = oracle.to_ticks(win, tb)
    assert not np.any((a["log_tick"] % wt == 0) & (a["log_tick"] > 0))
