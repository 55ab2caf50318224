"""3D simple-cubic lattice on the GPU (six neighbours, 14 classes, six face
histories) against the CPU oracle's 3D DES, bit for bit: final spins, the
(tick, site) of every committed flip of every subdomain, digests, flip
counts, carry, M and the bond sum; and g of every window against the oracle's
literal 3D relaxation."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import check_against_oracle, say

pytestmark = pytest.mark.gpu


def p3(L, b, T, h=0.0, J=1.0, **kw):
    p = W.params(L[0], L[1], b[0], b[1], T=T, h=h, J=J, **kw)
    p.update(Lz=L[2], bz=b[2])
    return p


CASES3 = [
    # L, block, T, h, window, horizon, tick_bits, rule, init, step
    ((8, 8, 8), (4, 4, 4), 4.5, 0.1, 0.5, 3.0, 28, "metropolis", "random", "continue"),   # 64 sites: 1 per lane
    ((16, 16, 16), (8, 8, 8), 4.0, 0.05, 0.25, 1.5, 28, "metropolis", "random", "continue"),  # 512: 8 per lane
    ((16, 8, 8), (8, 4, 4), 4.5, -0.1, 0.5, 2.0, 28, "glauber", "random", "continue"),   # 128 sites, 2 per lane
    ((8, 8, 8), (8, 4, 4), 4.0, 0.1, 0.5, 2.0, 28, "metropolis", "random", "continue"),  # wraps in x
    ((8, 8, 8), (4, 8, 4), 4.0, 0.1, 0.5, 2.0, 28, "metropolis", "random", "continue"),  # wraps in y
    ((8, 8, 4), (4, 4, 4), 4.0, 0.0, 0.5, 2.0, 28, "metropolis", "random", "continue"),  # wraps in z
    ((8, 8, 8), (8, 8, 8), 4.0, 0.1, 0.5, 3.0, 28, "metropolis", "random", "continue"),  # one subdomain
    ((12, 12, 12), (6, 6, 6), 4.5, 0.0, 0.5, 2.0, 28, "metropolis", "random", "continue"),  # 216: partial nibbles
    ((8, 8, 8), (4, 4, 4), 4.0, 0.0, 0.5, 3.0, 5, "metropolis", "random", "continue"),   # coarse ticks: ties
    ((16, 16, 16), (8, 8, 8), 3.0, 0.05, 1.0, 5.0, 28, "metropolis", "up", "continue"),  # low T, sparse
    ((8, 8, 8), (4, 4, 4), 4.5, 0.1, 0.25, 2.1, 28, "glauber", "random", "wipe"),        # wipe rule
    ((8, 16, 8), (4, 4, 4), 5.0, 0.2, 0.5, 2.0, 28, "metropolis", "random", "continue"),  # 4 blocks along y
]


@pytest.mark.parametrize("L,b,T,h,win,hor,tb,rule,init,step", CASES3)
def test_gpu3d_matches_oracle(L, b, T, h, win, hor, tb, rule, init, step):
    p = p3(L, b, T=T, h=h, window=win, horizon=hor, seed=777 + L[0] + b[2], tick_bits=tb, rule=rule,
           init=init, step=step)
    check_against_oracle(p)


def test_gpu3d_one_launch_per_iteration(monkeypatch):
    monkeypatch.setenv("SR_NO_GRAPHS", "1")
    p = p3((8, 8, 8), (4, 4, 4), T=4.5, h=0.1, window=0.5, horizon=2.0, seed=5)
    check_against_oracle(p)


def test_gpu3d_user_spins_and_rate_table():
    import oracle
    rng = np.random.default_rng(3)
    s0 = np.where(rng.random((8, 8, 8)) < 0.7, 1, -1).astype(np.int8)
    p = p3((8, 8, 8), (4, 4, 4), T=3.5, h=-0.1, window=0.5, horizon=2.0, seed=9, init="user", init_spins=s0)
    check_against_oracle(p)
    import paper_cs_0405053_amd as sr
    s = sr.Sim(p)
    assert np.array_equal(s.rate_table(), oracle.rate_table3(1.0, -0.1, 3.5))
    s.close()


def test_gpu3d_tuned_block_and_window():
    # the tuner picks a cubic block; the continued trajectory does not depend
    # on the adapted window
    import paper_cs_0405053_amd as sr
    import oracle
    p = p3((16, 16, 16), (0, 0, 0), T=4.5, h=0.1, window=0.0, horizon=2.0, seed=12)
    s = sr.Sim(dict(p, log_mode="digest"))
    s.run()
    o = s.observables()
    assert (o["bx"], o["by"], o["bz"]) == (8, 8, 8)
    ref = oracle.des(dict(p, bx=8, by=8, bz=8, window=1.0), log=False)
    assert np.array_equal(s.spins(), ref["spins"])
    assert np.array_equal(s.digests()[0], ref["sub_digest"])
    s.close()


def test_gpu3d_checkpoint_resume():
    import paper_cs_0405053_amd as sr
    p = p3((8, 8, 8), (4, 4, 4), T=4.0, h=0.1, window=0.5, horizon=3.0, seed=21, log_mode="digest")
    a = sr.Sim(p)
    a.run(2)
    b = sr.Sim.load(a.save())
    a.run()
    b.run()
    assert np.array_equal(a.spins(), b.spins())
    assert np.array_equal(a.digests()[0], b.digests()[0])
    a.close()
    b.close()


def test_gpu3d_batch_rejected():
    import paper_cs_0405053_amd as sr
    s = sr.Sim(p3((8, 8, 8), (4, 4, 4), T=4.0, window=0.5, horizon=1.0, seed=1, log_mode="digest"))
    with pytest.raises(sr.SRError) as e:
        sr.batch_run([s])
    assert e.value.code == sr.SR_EINVAL
    s.close()
