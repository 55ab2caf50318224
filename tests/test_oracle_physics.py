"""Pins of the oracle's whole simulation against exact physics.

The DES must be the continuous-time Markov chain of Sec. 3 (every site tries
to flip at rate lambda = 1 and succeeds with p of eq. pMin or eq. pglauber),
whose stationary law is the Boltzmann distribution of eq. hamil.  Checked by:

* exact enumeration of all 2^9 / 2^16 states of 3x3 / 4x4 tori (time averages
  of E, M, M^2, |M| each within 3 standard errors over independent replicas,
  and the four together by one Hotelling T^2 test at the same false-alarm
  level), on several partitions into subdomains, both acceptance rules,
  h != 0;
* Onsager's exact energy per site and Yang's spontaneous magnetisation on a
  128x128 torus at h = 0 (batch-means standard errors);
* J = 0 closed forms: independent two-state spins relax as
  m(t) = m_eq + (m_0 - m_eq) exp(-(a+b) t) and flip at stationary rate
  2ab/(a+b); J = h = 0: all rates 1, so the event count is Poisson(N t) and
  the flipped sites are uniform.

Tolerances: 3 standard errors for a single comparison.  A test that makes k
comparisons at once uses the Bonferroni threshold that keeps the chance of a
false alarm anywhere in the family at that of one 3-SE comparison (two-sided
0.27%).  Seeds are fixed, so every test is deterministic.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def z_limit(k=1, sigmas=3.0):
    """Two-sided z threshold for k simultaneous comparisons whose family-wise
    false-alarm probability equals that of one `sigmas`-SE comparison."""
    from scipy.stats import norm
    return float(norm.isf(norm.sf(sigmas) / k))


def _enumerate(L, J, h, T):
    n = L * L
    states = np.arange(2**n, dtype=np.int64)
    bits = ((states[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)
    s = (2 * bits - 1).reshape(-1, L, L)
    M = s.sum(axis=(1, 2)).astype(np.float64)
    bond = (s * np.roll(s, -1, 1) + s * np.roll(s, -1, 2)).sum(axis=(1, 2)).astype(np.float64)
    E = -J * bond - h * M
    w = np.exp(-(E - E.min()) / T)
    Z = w.sum()
    return {"E": (w * E).sum() / Z, "M": (w * M).sum() / Z,
            "M2": (w * M * M).sum() / Z, "absM": (w * np.abs(M)).sum() / Z}


ENUM_CASES = [
    # L, bx, by, J, h, T, rule
    (3, 3, 3, 1.0, 0.0, 2.0, "metropolis"),
    (3, 1, 3, 1.0, 0.3, 1.5, "glauber"),
    (4, 2, 2, 1.0, 0.1, 2.5, "metropolis"),
    (4, 4, 2, 1.0, -0.2, 1.8, "metropolis"),
    (4, 2, 2, 0.5, 0.4, 1.0, "glauber"),
]


@pytest.mark.parametrize("L,bx,by,J,h,T,rule", ENUM_CASES)
def test_des_matches_exact_enumeration(L, bx, by, J, h, T, rule):
    exact = _enumerate(L, J, h, T)
    reps = []
    for rep in range(24):
        p = W.params(L, L, bx, by, T=T, h=h, J=J, window=50.0, horizon=1550.0,
                     seed=1000 * rep + 17, rule=rule)
        r = oracle.des(p, log=False, burn=50.0)
        n = r["int_ticks"]
        E = (-J * r["int_bond"] - h * r["int_M"]) / n
        reps.append((E, r["int_M"] / n, r["int_M2"] / n, r["int_absM"] / n))
    reps = np.array(reps)
    mean = reps.mean(0)
    se = reps.std(0, ddof=1) / math.sqrt(len(reps))
    keys = ["E", "M", "M2", "absM"]
    for i, key in enumerate(keys):
        assert abs(mean[i] - exact[key]) < 3 * se[i] + 1e-12, (key, mean[i], exact[key], se[i])
    # the four observables together: Hotelling's T^2 over the replicas,
    # n (n - p) / (p (n - 1)) d' S^-1 d ~ F(p, n - p)
    from scipy.stats import f as fdist, norm
    n, q = reps.shape
    d = mean - np.array([exact[k] for k in keys])
    S = np.cov(reps, rowvar=False)
    F = n * float(d @ np.linalg.solve(S, d)) * (n - q) / (q * (n - 1))
    assert F < fdist.isf(2 * norm.sf(3.0), q, n - q), (F, d.tolist())


def _onsager(T, J=1.0):
    from scipy.special import ellipk
    b = 1.0 / T
    k = 2 * math.sinh(2 * b * J) / math.cosh(2 * b * J) ** 2
    u = -J / math.tanh(2 * b * J) * (1 + 2 / math.pi * (2 * math.tanh(2 * b * J) ** 2 - 1)
                                     * ellipk(k * k))
    Tc = 2 * J / math.log(1 + math.sqrt(2))
    m0 = (1 - math.sinh(2 * b * J) ** -4) ** 0.125 if T < Tc else 0.0
    return u, m0


def test_onsager_closed_form_values():
    # the closed forms themselves, at points where they are known exactly
    Tc = 2 / math.log(1 + math.sqrt(2))
    u, m0 = _onsager(Tc * (1 + 1e-6))        # u(Tc) = -sqrt(2) J, m0(Tc) = 0
    assert abs(u + math.sqrt(2)) < 1e-4 and m0 == 0.0
    u, m0 = _onsager(0.05)
    assert abs(u + 2.0) < 1e-9 and abs(m0 - 1.0) < 1e-9


@pytest.mark.parametrize("T,burn,horizon", [(1.0, 20.0, 220.0), (1.5, 30.0, 330.0),
                                            (3.0, 20.0, 120.0)])
def test_des_matches_onsager(T, burn, horizon):
    L = 128
    p = W.params(L, L, 8, 8, T=T, h=0.0, window=1.0, horizon=horizon, seed=99,
                 init="up")
    r = oracle.des(p, log=False)
    nb = int(burn)
    e = -r["snap_bond"][nb:] / (L * L)          # energy per site at unit times
    m = r["snap_M"][nb:] / (L * L)
    u, m0 = _onsager(T)

    def batch_se(x, nbatch=10):
        xs = np.array_split(x, nbatch)
        bm = np.array([b.mean() for b in xs])
        return bm.mean(), bm.std(ddof=1) / math.sqrt(nbatch)

    em, ese = batch_se(e)
    lim = z_limit(2 if m0 > 0 else 1)
    assert abs(em - u) < lim * ese, (em, u, ese)
    if m0 > 0:
        mm, mse = batch_se(m)
        assert abs(mm - m0) < lim * mse, (mm, m0, mse)


@pytest.mark.parametrize("h,T,rule", [(0.2, 1.0, "metropolis"), (-0.3, 2.0, "glauber")])
def test_zero_coupling_relaxation(h, T, rule):
    L = 64
    p = W.params(L, L, 16, 16, J=0.0, T=T, h=h, window=0.25, horizon=5.0, seed=4,
                 init="up", rule=rule)
    r = oracle.des(p, log=False)
    rt = oracle.rate_table(0.0, h, T, rule) / 2.0**28
    a, b = rt[0], rt[5]                  # + -> - and - -> + (no neighbour effect)
    m_eq = (b - a) / (a + b)
    N = L * L
    lim = z_limit(len(r["snap_M"]))
    for k, M in enumerate(r["snap_M"]):
        t = k * 0.25
        mt = m_eq + (1.0 - m_eq) * math.exp(-(a + b) * t)
        sig = math.sqrt(max(1 - mt * mt, 1e-12) / N)   # independent spins: exact sd
        assert abs(M / N - mt) < lim * sig + 1e-12, (t, M / N, mt)
    # stationary flip rate per site, 2ab/(a+b), measured after relaxation
    p2 = W.params(L, L, 16, 16, J=0.0, T=T, h=h, window=1.0, horizon=40.0, seed=5,
                  rule=rule)
    r2 = oracle.des(p2)
    late = r2["log_tick"] >= 10 * 2**28
    rate = late.sum() / (N * 30.0)
    want = 2 * a * b / (a + b)
    assert abs(rate - want) < 3 * math.sqrt(want / (N * 30.0)), (rate, want)


def test_free_spins_poisson_counts_and_uniform_sites():
    L, H = 32, 20.0
    p = W.params(L, L, 8, 8, J=0.0, T=1.0, h=0.0, window=1.0, horizon=H, seed=8)
    r = oracle.des(p)
    assert np.all(oracle.rate_table(0.0, 0.0, 1.0) == 2**28)
    N = L * L
    n = r["n_events"]
    assert abs(n - N * H) < 3 * math.sqrt(N * H)
    counts = np.bincount(r["log_site"], minlength=N)
    chi2 = ((counts - n / N) ** 2 / (n / N)).sum()
    # chi-square with N-1 dof: mean N-1, sd sqrt(2(N-1))
    assert abs(chi2 - (N - 1)) < 3 * math.sqrt(2 * (N - 1))
    # per-window counts of one 8x8 block are Poisson(64 * 1)
    per = np.zeros(int(H), dtype=np.int64)
    sel = r["log_sub"] == 0
    np.add.at(per, (r["log_tick"][sel] >> 28), 1)
    assert abs(per.mean() - 64) < 3 * math.sqrt(64 / H)
