"""The rate table is the one place where floating point decides an integer
(eqs. hamil, pMin / pglauber: r_k = round(2^28 p_k) computed in IEEE double).
The library and the oracle compute it independently; both must give the same
ten integers for every parameter set any workload or test uses, so that the
integer trajectories can agree bit for bit.  Host-only (no GPU)."""
import numpy as np
import pytest

import oracle
import workloads as W


def _sr():
    import paper_cs_0405053_amd as sr
    return sr


def _check(ps):
    sr = _sr()
    for p in ps:
        got = sr.rate_table(p)
        want = oracle.rate_table(p["J"], p["h"], p["T"], p.get("rule", "metropolis"))
        assert np.array_equal(got, want), (p["J"], p["h"], p["T"], p.get("rule"), got, want)


def test_every_workload_family():
    ps = [W.small(), *[W.medium(T=T) for T in W.MEDIUM_TEMPS], W.large()]
    ps += W.batch()                    # all 512 lattices (random T, h)
    ps += W.serve_stream()             # every request the benchmark replays
    _check(ps)


def test_random_sweep_both_rules_any_sign():
    rng = np.random.default_rng(17)
    ps = []
    for i in range(4000):
        ps.append(dict(J=float(rng.uniform(-2.0, 2.0)), h=float(rng.uniform(-1.0, 1.0)),
                       T=float(np.exp(rng.uniform(np.log(0.05), np.log(50.0)))),
                       rule=["metropolis", "glauber"][i % 2], Lx=16, Ly=16, horizon=1.0))
    _check(ps)


@pytest.mark.parametrize("J,h,T", [(1.0, 0.0, 0.02), (1.0, 0.05, 0.1), (-1.0, 0.3, 0.05),
                                   (0.0, 0.0, 1.0), (1.0, 1e-12, 1.5), (3.0, -2.0, 0.3)])
def test_edge_parameters(J, h, T):
    # tiny T underflows the uphill rates to 0 (Lambda can be 0); J < 0; J = 0
    ps = [dict(J=J, h=h, T=T, rule=r, Lx=16, Ly=16, horizon=1.0) for r in ("metropolis", "glauber")]
    _check(ps)
    if T <= 0.05:
        assert (oracle.rate_table(J, h, T) == 0).any()


def test_rejects_bad_temperature():
    sr = _sr()
    for T in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(sr.SRError):
            sr.rate_table(dict(J=1.0, h=0.0, T=T, Lx=16, Ly=16, horizon=1.0))
