"""Pins of the oracle's primitives against things other than itself.

* Philox-4x32-10: against rocRAND's independent implementation (its device
  API compiled for the host), over keys/counters that exercise every word.
* fixed-point -ln U: against mpmath at 50 digits (closed form), exact special
  values, monotonicity, and the Exp(1) law (KS test).
* rate table (eqs. pMin / pglauber of Sec. 2): detailed balance between a
  flip and its reverse, Metropolis' max-rate property, Glauber's p + p' = 1.
* class / site choice (eqs. Wsum, Wstop, nores, vindex of Sec. 3): the map
  from the integer target to a site partitions [0, Lambda) into consecutive
  runs of length r_k(v), one per site, ordered by (class, local index).
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W

MASK64 = 2**64 - 1


# ----------------------------------------------------------------- Philox
@pytest.fixture(scope="module")
def rocrand_bin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    out = tmp_path_factory.mktemp("rr") / "rocrand_philox"
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox.cpp")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", src,
                           "-o", str(out)], stdout=subprocess.DEVNULL)
    return str(out)


def test_philox_matches_rocrand(rocrand_bin):
    # rocrand_init(seed, subsequence, offset) uses key = (seed lo, seed hi)
    # and counter = (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi).
    rng = np.random.default_rng(11)
    cases = [(0, 0, 0), (MASK64, MASK64, 0), (0x5EED0001, 3, 4 * 17)]
    for _ in range(200):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        c01 = int(rng.integers(0, 2**62))
        c23 = int(rng.integers(0, 2**63))
        cases.append((seed, c23, 4 * c01))
    inp = "".join(f"{s} {q} {o}\n" for s, q, o in cases)
    res = subprocess.run([rocrand_bin], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for (seed, sub, off), line in zip(cases, res):
        want = tuple(int(x) for x in line.split())
        c = off // 4
        got = oracle.philox((seed & 0xFFFFFFFF, seed >> 32),
                            (c & 0xFFFFFFFF, c >> 32, sub & 0xFFFFFFFF, sub >> 32))
        assert got == want, (seed, sub, off)


def test_philox_uniform_bits():
    # 4096 blocks of one stream: every output bit is set about half the time.
    words = np.array([oracle.philox((5, 0), (j, 0, 3, 0)) for j in range(4096)],
                     dtype=np.uint64)
    for b in range(32):
        frac = ((words >> np.uint64(b)) & np.uint64(1)).mean()
        assert abs(frac - 0.5) < 5 * 0.5 / math.sqrt(words.size)


# ----------------------------------------------------------------- digest mixer
GAMMA = 0x9E3779B97F4A7C15          # SplitMix64's Weyl increment


def test_digest_mixer_known_answers():
    # SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) seeded with 0 returns
    # mix(k * GAMMA) for k = 1, 2, 3, ...; its published first outputs:
    assert oracle.mix64(GAMMA) == 0xE220A8397B1DCDAF
    assert oracle.mix64((2 * GAMMA) & MASK64) == 0x6E789E6AA1B965F4
    assert oracle.mix64((3 * GAMMA) & MASK64) == 0x06C45D188009454F
    # one committed event (tick, global site) is folded as mix(mix(tick) + site)
    rng = np.random.default_rng(4)
    for t, v in [(0, 0), (1, 2), (2**40 + 3, 1 << 24)] + \
            [(int(a), int(b)) for a, b in zip(rng.integers(0, 2**46, 50), rng.integers(0, 2**26, 50))]:
        assert oracle.event_digest(t, v) == oracle.mix64((oracle.mix64(t) + v) & MASK64)


def test_digest_mixer_avalanche():
    # a digest compared in place of a full event list is only as good as the
    # mixer: flipping any one input bit must flip about half the output bits
    rng = np.random.default_rng(8)
    xs = [int(x) for x in rng.integers(0, 2**63, size=300)] + [0, 1, MASK64]
    flips = np.zeros(64)
    for x in xs:
        y = oracle.mix64(x)
        for b in range(64):
            flips[b] += bin(y ^ oracle.mix64(x ^ (1 << b))).count("1")
    flips /= len(xs)
    # binomial(64, 1/2): mean 32, sd 4 per pair; mean over ~300 pairs
    assert np.all(np.abs(flips - 32.0) < 1.5), flips.round(2)
    # distinct event pairs map to distinct digests (no collisions in a sample)
    ds = {oracle.event_digest(t, v) for t in range(300) for v in range(40)}
    assert len(ds) == 300 * 40


# ----------------------------------------------------------------- -ln U
mpmath = pytest.importorskip("mpmath")
mpmath.mp.dps = 50


def _exact_neglog(u):
    m = (u | 1)
    return -mpmath.log(mpmath.mpf(m) / mpmath.mpf(2) ** 64)


def test_ln2_constant():
    assert int(mpmath.floor(mpmath.log(2) * mpmath.mpf(2) ** 64)) == 0xB17217F7D1CF79AB


def test_expq_error_bound_and_special_values():
    rng = np.random.default_rng(5)
    us = [0, 1, 2, 3, 2**63, 2**63 + 1, MASK64, MASK64 - 1, 2**32, 2**40 + 12345]
    us += [1 << k for k in range(64)] + [(1 << k) - 1 for k in range(1, 65)]
    us += [int(x) for x in rng.integers(0, 2**63, size=3000)] + \
          [int(x) * 2 + 1 for x in rng.integers(0, 2**63, size=3000)]
    worst = 0.0
    for u in us:
        u &= MASK64
        E = oracle.expq(u, 28)
        err = abs(float(mpmath.mpf(E) / mpmath.mpf(2) ** 56 - _exact_neglog(u)))
        worst = max(worst, err)
    # 32 truncated squarings plus the final floor: well inside 2^-28 of -ln U
    assert worst < 2.0 ** -28, worst
    # m = 1 and m = 2^63 + 1 have mantissa exactly 1: frac = 0 exactly
    L = 0xB17217F7D1CF79AB
    assert oracle.expq(0, 28) == L >> 2              # 64 ln 2 in Q56
    assert oracle.expq(2**63, 28) == L >> 8          # 1 ln 2 in Q56 (m = 2^63+1)


def test_expq_monotone_and_tick_scaling():
    rng = np.random.default_rng(9)
    us = sorted(set(int(x) for x in rng.integers(0, 2**63, size=4000)) |
                {0, 1, 2, 2**62, 2**63 - 1, 2**63, MASK64})
    Es = [oracle.expq(u, 28) for u in us]
    assert all(a >= b for a, b in zip(Es, Es[1:]))
    for u in us[::97]:
        for tb in (4, 10, 20, 27):
            assert oracle.expq(u, tb) == oracle.expq(u, 28) >> (28 - tb)


def test_expq_is_exponential():
    scipy_stats = pytest.importorskip("scipy.stats")
    x = np.array([oracle.expq(oracle.philox((1, 2), (j, 0, 0, 0))[0] |
                              (oracle.philox((1, 2), (j, 0, 0, 0))[1] << 32), 28)
                  for j in range(20000)], dtype=np.float64) / 2.0**56
    st = scipy_stats.kstest(x, "expon")
    assert st.pvalue > 1e-3
    assert abs(x.mean() - 1.0) < 5 / math.sqrt(x.size)


# ----------------------------------------------------------------- rates
@pytest.mark.parametrize("J,h,T", [(1, 0, 1.5), (1, 0.1, 2.269), (1, 0.05, 1.0),
                                   (1, -0.2, 3.5), (0.5, 0.3, 0.7), (1, 0.0, 20.0)])
@pytest.mark.parametrize("rule", ["metropolis", "glauber"])
def test_rate_table_detailed_balance(J, h, T, rule):
    r = oracle.rate_table(J, h, T, rule).astype(np.float64)
    one = 2.0**28
    assert r.max() <= one
    for k in range(5):          # class (+, n_up) and its reverse (-, n_up)
        kb = k + 5
        dE = 2.0 * (J * (2 * k - 4) + h)          # energy change of + -> -
        ratio_exact = math.exp(-dE / T)
        if r[k] >= 64 and r[kb] >= 64:           # both resolvable in Q28
            rel = abs(r[k] / r[kb] - ratio_exact) / ratio_exact
            assert rel < 2.0 / min(r[k], r[kb]), (k, r[k], r[kb])
        if rule == "metropolis":
            assert max(r[k], r[kb]) == one        # the downhill flip always succeeds
        else:
            assert abs(r[k] + r[kb] - one) <= 1.0  # theta/(1+theta) + 1/(1+theta)


def test_rate_table_printed_cases():
    # Metropolis with J=1, h=0, T=1.5: the least likely flip (all four
    # neighbours aligned) has p = exp(-8/1.5); reverse classes of zero-cost
    # flips (n_up = 2, h = 0) have p = 1.
    r = oracle.rate_table(1.0, 0.0, 1.5)
    assert r[4] == r[5] == round(math.exp(-8 / 1.5) * 2**28)
    assert r[2] == r[7] == 2**28
    with pytest.raises(ValueError):
        oracle.rate_table(1.0, 0.0, 0.0)


# ----------------------------------------------------------------- selection
def _classes(spins):
    s = spins
    up = ((np.roll(s, 1, 0) > 0).astype(int) + (np.roll(s, -1, 0) > 0) +
          (np.roll(s, 1, 1) > 0) + (np.roll(s, -1, 1) > 0))
    return 5 * (s < 0) + up


@pytest.mark.parametrize("seed,T,h", [(1, 1.5, 0.0), (2, 3.0, 0.1), (3, 2.0, -0.2)])
def test_selection_partitions_target_range(seed, T, h):
    p = W.params(8, 8, 4, 4, T=T, h=h, window=1.0, horizon=1.0, seed=seed)
    spins = W.random_spins(8, 8, seed)
    rates = oracle.rate_table(1.0, h, T).astype(np.int64)
    cls = _classes(spins)
    for d in range(4):
        y0, x0 = (d // 2) * 4, (d % 2) * 4
        loc = [(cls[y0 + ly, x0 + lx], ly * 4 + lx, (y0 + ly) * 8 + x0 + lx)
               for ly in range(4) for lx in range(4)]
        lam = sum(int(rates[k]) for k, _, _ in loc)
        assert oracle.subdomain_lambda(p, spins, d) == lam

        def pick(target):   # V with floor(V * lam / 2^64) == target
            V = -(-(target << 64) // lam)
            assert (V * lam) >> 64 == target
            return oracle.select_site(p, spins, d, V)

        order = sorted((k, li, g) for k, li, g in loc if rates[k] > 0)
        start = 0
        for k, li, g in order:
            # site g owns exactly the targets [start, start + r_k)
            assert pick(start) == g
            assert pick(start + int(rates[k]) - 1) == g
            if start > 0:
                assert pick(start - 1) != g
            start += int(rates[k])
        assert start == lam
