"""Pins of the 3D simple-cubic oracle (the generalisation to more
dimensions and neighbours the paper names in Secs. 3 and 5): six neighbours,
14 classes k = 7*[s = -1] + n_up, faces W/E/N/S/D/U.

* rate table: detailed balance of every class against its reverse, the
  Metropolis and Glauber normalisations;
* selection: over [0, Lambda) the targets fall on the subdomain's sites in
  runs of length r_k(v), in (class, local index) order, with classes computed
  independently here from the spins;
* whole DES: exact Boltzmann enumeration of 2x3x3 (2^18 states), 2x2x4 and
  3x2x2 tori on several partitions, both rules, h != 0 (3 standard errors
  per observable, Hotelling T^2 for the four together); J = 0 closed forms;
  J = h = 0 Poisson counts and uniform sites;
* relaxation: the literal 3D synchronous relaxation (six face histories)
  reaches the DES bit for bit, with either step rule; continuation does not
  depend on the window; one subdomain needs one iteration per window.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_physics import z_limit


def p3(L, b, T, h=0.0, J=1.0, **kw):
    Lx, Ly, Lz = L
    bx, by, bz = b
    p = W.params(Lx, Ly, bx, by, T=T, h=h, J=J, **kw)
    p.update(Lz=Lz, bz=bz)
    return p


def _same(a, b):
    return (a["n_events"] == b["n_events"]
            and np.array_equal(a["log_tick"], b["log_tick"])
            and np.array_equal(a["log_site"], b["log_site"])
            and np.array_equal(a["log_sub"], b["log_sub"])
            and np.array_equal(a["spins"], b["spins"])
            and np.array_equal(a["carry"], b["carry"])
            and np.array_equal(a["sub_digest"], b["sub_digest"]))


# ------------------------------------------------------------------ rates
@pytest.mark.parametrize("J,h,T,rule", [(1.0, 0.0, 4.5, "metropolis"), (1.0, 0.2, 3.0, "glauber"),
                                        (0.5, -0.3, 2.0, "metropolis"), (-1.0, 0.1, 5.0, "glauber")])
def test_rate_table3_detailed_balance(J, h, T, rule):
    r = oracle.rate_table3(J, h, T, rule).astype(np.float64)
    one = 2.0**28
    assert len(r) == 14 and r.max() <= one
    for k in range(7):
        kb = k + 7
        dE = 2.0 * (J * (2 * k - 6) + h)
        ratio = math.exp(-dE / T)
        if r[k] >= 64 and r[kb] >= 64:
            assert abs(r[k] / r[kb] - ratio) / ratio < 2.0 / min(r[k], r[kb]), k
        if rule == "metropolis":
            assert max(r[k], r[kb]) == one
        else:
            assert abs(r[k] + r[kb] - one) <= 1.0


def test_rate_table3_printed_case():
    # all six neighbours aligned, J = 1, h = 0: p = exp(-12/T); three up
    # neighbours cost nothing
    r = oracle.rate_table3(1.0, 0.0, 4.0)
    assert r[6] == r[7] == round(math.exp(-12 / 4.0) * 2**28)
    assert r[3] == r[10] == 2**28


# ------------------------------------------------------------------ selection
def _classes3(s):
    up = sum((np.roll(s, sh, ax) > 0).astype(int) for ax in range(3) for sh in (1, -1))
    return 7 * (s < 0) + up


@pytest.mark.parametrize("seed,T,h", [(1, 4.5, 0.0), (2, 3.0, 0.1)])
def test_selection3_partitions_target_range(seed, T, h):
    L, b = (4, 6, 4), (2, 3, 2)
    p = p3(L, b, T=T, h=h, window=1.0, horizon=1.0, seed=seed)
    rng = np.random.default_rng(seed)
    spins = np.where(rng.random((L[2], L[1], L[0])) < 0.5, 1, -1).astype(np.int8)
    rates = oracle.rate_table3(1.0, h, T).astype(np.int64)
    cls = _classes3(spins)
    nbx, nby = L[0] // b[0], L[1] // b[1]
    for d in range((L[0] // b[0]) * (L[1] // b[1]) * (L[2] // b[2])):
        x0, y0, z0 = (d % nbx) * b[0], ((d // nbx) % nby) * b[1], (d // (nbx * nby)) * b[2]
        loc = [(cls[z0 + lz, y0 + ly, x0 + lx], (lz * b[1] + ly) * b[0] + lx,
                ((z0 + lz) * L[1] + y0 + ly) * L[0] + x0 + lx)
               for lz in range(b[2]) for ly in range(b[1]) for lx in range(b[0])]
        lam = sum(int(rates[k]) for k, _, _ in loc)
        assert oracle.subdomain_lambda(p, spins, d) == lam

        def pick(target):
            V = -(-(target << 64) // lam)
            return oracle.select_site(p, spins, d, V)

        start = 0
        for k, li, g in sorted((k, li, g) for k, li, g in loc if rates[k] > 0):
            assert pick(start) == g and pick(start + int(rates[k]) - 1) == g
            start += int(rates[k])
        assert start == lam


# ------------------------------------------------------------------ physics
def _enumerate3(L, J, h, T):
    Lx, Ly, Lz = L
    n = Lx * Ly * Lz
    states = np.arange(2**n, dtype=np.int64)
    bits = ((states[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int8)
    s = (2 * bits - 1).reshape(-1, Lz, Ly, Lx).astype(np.int64)
    M = s.sum(axis=(1, 2, 3)).astype(np.float64)
    # every bond once: +x, +y, +z of every site (a direction of length 2
    # links the pair twice)
    bond = sum((s * np.roll(s, -1, ax)).sum(axis=(1, 2, 3)) for ax in (1, 2, 3)).astype(np.float64)
    E = -J * bond - h * M
    w = np.exp(-(E - E.min()) / T)
    Z = w.sum()
    return {"E": (w * E).sum() / Z, "M": (w * M).sum() / Z,
            "M2": (w * M * M).sum() / Z, "absM": (w * np.abs(M)).sum() / Z}


ENUM3 = [
    # L, block, J, h, T, rule
    ((2, 3, 3), (2, 3, 1), 1.0, 0.2, 4.0, "metropolis"),
    ((2, 2, 4), (2, 2, 2), 1.0, -0.3, 3.0, "glauber"),
    ((3, 2, 2), (1, 2, 2), 0.5, 0.4, 2.0, "metropolis"),
    ((2, 3, 3), (2, 3, 3), 1.0, 0.0, 5.0, "glauber"),
]


@pytest.mark.parametrize("L,b,J,h,T,rule", ENUM3)
def test_des3_matches_exact_enumeration(L, b, J, h, T, rule):
    exact = _enumerate3(L, J, h, T)
    reps = []
    for rep in range(64):
        p = p3(L, b, T=T, h=h, J=J, window=25.0, horizon=1025.0, seed=3000 * rep + 29, rule=rule)
        r = oracle.des(p, log=False, burn=25.0)
        n = r["int_ticks"]
        E = (-J * r["int_bond"] - h * r["int_M"]) / n
        reps.append((E, r["int_M"] / n, r["int_M2"] / n, r["int_absM"] / n))
    reps = np.array(reps)
    mean = reps.mean(0)
    se = reps.std(0, ddof=1) / math.sqrt(len(reps))
    keys = ["E", "M", "M2", "absM"]
    for i, key in enumerate(keys):
        assert abs(mean[i] - exact[key]) < 3 * se[i] + 1e-12, (key, mean[i], exact[key], se[i])
    from scipy.stats import f as fdist, norm
    n, q = reps.shape
    d = mean - np.array([exact[k] for k in keys])
    S = np.cov(reps, rowvar=False)
    F = n * float(d @ np.linalg.solve(S, d)) * (n - q) / (q * (n - 1))
    assert F < fdist.isf(2 * norm.sf(3.0), q, n - q), (F, d.tolist())


def test_enumeration3_reduces_to_independent_spins():
    # J = 0: each spin independently up with probability e^{h/T}/(2 cosh(h/T))
    L, h, T = (2, 2, 3), 0.3, 1.5
    ex = _enumerate3(L, 0.0, h, T)
    n = 12
    m = math.tanh(h / T)
    assert abs(ex["M"] - n * m) < 1e-9
    assert abs(ex["M2"] - (n + n * (n - 1) * m * m)) < 1e-9


@pytest.mark.parametrize("h,T,rule", [(0.2, 1.0, "metropolis"), (-0.3, 2.0, "glauber")])
def test_zero_coupling3_closed_forms(h, T, rule):
    L = (16, 16, 16)
    N = 16**3
    rt = oracle.rate_table3(0.0, h, T, rule) / 2.0**28
    assert np.all(rt[:7] == rt[0]) and np.all(rt[7:] == rt[7])
    a, b = rt[0], rt[7]
    m_eq = (b - a) / (a + b)
    p = p3(L, (8, 8, 8), T=T, h=h, J=0.0, window=0.25, horizon=5.0, seed=4, init="up", rule=rule)
    r = oracle.des(p, log=False)
    lim = z_limit(len(r["snap_M"]))
    for k, M in enumerate(r["snap_M"]):
        mt = m_eq + (1.0 - m_eq) * math.exp(-(a + b) * k * 0.25)
        sig = math.sqrt(max(1 - mt * mt, 1e-12) / N)
        assert abs(M / N - mt) < lim * sig + 1e-12, (k, M / N, mt)
    p2 = p3(L, (8, 8, 8), T=T, h=h, J=0.0, window=1.0, horizon=25.0, seed=5, rule=rule)
    r2 = oracle.des(p2)
    late = r2["log_tick"] >= 5 * 2**28
    rate = late.sum() / (N * 20.0)
    want = 2 * a * b / (a + b)
    assert abs(rate - want) < 3 * math.sqrt(want / (N * 20.0)), (rate, want)


def test_free_spins3_poisson_counts_and_uniform_sites():
    L, H = (8, 8, 8), 20.0
    p = p3(L, (4, 4, 4), T=1.0, J=0.0, window=1.0, horizon=H, seed=8)
    r = oracle.des(p)
    N = 512
    n = r["n_events"]
    assert abs(n - N * H) < 3 * math.sqrt(N * H)
    counts = np.bincount(r["log_site"], minlength=N)
    chi2 = ((counts - n / N) ** 2 / (n / N)).sum()
    assert abs(chi2 - (N - 1)) < 3 * math.sqrt(2 * (N - 1))


# ------------------------------------------------------------------ relaxation
SR3 = [
    # L, block, T, h, window, horizon, tick_bits, rule, init, step
    ((8, 8, 8), (4, 4, 4), 4.5, 0.1, 0.5, 3.0, 28, "metropolis", "random", "continue"),
    ((8, 8, 4), (4, 4, 2), 3.0, 0.0, 1.0, 4.0, 28, "glauber", "random", "continue"),
    ((8, 4, 8), (8, 2, 4), 4.0, 0.2, 0.5, 3.0, 28, "metropolis", "random", "continue"),  # wraps in x
    ((4, 8, 8), (2, 8, 4), 4.0, -0.1, 0.5, 3.0, 28, "metropolis", "random", "continue"), # wraps in y
    ((8, 8, 4), (4, 4, 4), 4.0, 0.1, 1.0, 3.0, 28, "metropolis", "random", "continue"),  # wraps in z
    ((8, 8, 8), (4, 4, 4), 4.0, 0.0, 0.5, 3.0, 5, "metropolis", "random", "continue"),   # ties
    ((8, 8, 8), (4, 4, 4), 3.0, 0.05, 1.0, 4.0, 28, "metropolis", "up", "continue"),     # low T, sparse
    ((8, 8, 8), (4, 4, 4), 4.5, 0.1, 0.5, 3.1, 28, "glauber", "random", "wipe"),
    ((8, 8, 8), (4, 4, 4), 4.0, 0.0, 0.25, 2.0, 5, "metropolis", "random", "wipe"),      # ties at step starts
]


@pytest.mark.parametrize("L,b,T,h,win,hor,tb,rule,init,step", SR3)
def test_sr3_reaches_des_trajectory(L, b, T, h, win, hor, tb, rule, init, step):
    p = p3(L, b, T=T, h=h, window=win, horizon=hor, seed=41, tick_bits=tb, rule=rule, init=init, step=step)
    a, s = oracle.des(p), oracle.sr(p)
    assert a["n_events"] > 0
    assert _same(a, s)
    assert np.array_equal(a["snap_M"], s["snap_M"]) and np.array_equal(a["snap_bond"], s["snap_bond"])
    assert np.all(s["g"][s["f"] == 0] == 1)
    if tb < 10:
        assert np.any(np.diff(a["log_tick"]) == 0)


def test_trajectory3_independent_of_window():
    base = p3((8, 8, 8), (4, 4, 4), T=4.0, h=0.1, window=1.0, horizon=4.0, seed=5)
    ref = oracle.des(base)
    for win in (0.25, 1.0, 3.0):
        assert _same(ref, oracle.sr(dict(base, window=win))), win


def test_single_subdomain3_is_serial():
    p = p3((4, 4, 4), (4, 4, 4), T=4.0, h=0.1, window=0.5, horizon=5.0, seed=3)
    s = oracle.sr(p)
    assert np.all(s["g"] == 1)
    assert _same(oracle.des(p), s)


def test_event_log3_invariants():
    p = p3((8, 8, 8), (4, 4, 4), T=4.5, h=0.1, window=1.0, horizon=3.0, seed=2)
    a = oracle.des(p)
    for d in range(8):
        t = a["log_tick"][a["log_sub"] == d]
        assert np.all(np.diff(t) > 0)
    v = a["log_site"]
    x, y, z = v % 8, (v // 8) % 8, v // 64
    assert np.array_equal(((z // 4) * 2 + y // 4) * 2 + x // 4, a["log_sub"])
    s = oracle.des(dict(p, horizon=0.0))["spins"].reshape(-1).copy()
    for q in v:
        s[q] = -s[q]
    assert np.array_equal(s.reshape(8, 8, 8), a["spins"])
    assert a["M"] == int(a["spins"].sum())
