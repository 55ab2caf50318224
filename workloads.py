"""Seeded synthetic workloads for synchronous-relaxation Ising runs.

This module holds only *inputs*: lattice sizes, couplings, temperatures,
fields, window lengths, horizons, seeds, and the seeded draws that generate
batches of lattices and request streams.  It holds none of the method's
arithmetic (no rates, no random streams of the method, no tick conversion),
so that both the GPU library's tests and the CPU oracle can take their inputs
from here without sharing any computation.

Workload families (2D square periodic lattice, J = 1, Metropolis rates):

* ``small``    64x64, h=0, T=1.5, random +-1 start, 16 subdomains of 16x16,
               window 1.0, horizon 50.
* ``medium``   1024x1024, h=0.1, T in {1.5, 2.269, 3.0}, random start,
               4096 subdomains of 16x16, window 0.5, horizon 100.
* ``large``    4096x4096, h=0.05, T=1.0, all spins up, 16384 subdomains of
               32x32, window in {0.25, 1, 4}, horizon 200.
* ``batch``    512 independent lattices, L uniform on multiples of 16 in
               [32, 512], T ~ U[1, 3.5], h ~ U[-0.2, 0.2], random start,
               horizon 50 each.
* ``serve``    Poisson request stream at 200 req/s, L log-uniform in
               [64, 2048] rounded to a multiple of 16, T ~ U[1, 3.5],
               h ~ U[-0.2, 0.2], horizon ~ U[10, 100], own seed per request.

The paper has no datasets or benchmark inputs; these synthetic families are
the measured workloads.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

SEED_BASE = 0x5EED0000


def params(Lx, Ly, bx, by, T, h=0.0, J=1.0, window=1.0, horizon=1.0, seed=1,
           init="random", rule="metropolis", tick_bits=28, init_spins=None,
           max_iters=0, log_mode="full", step="continue") -> Dict:
    """One lattice run description (plain dict, shared vocabulary).  `step`:
    "continue" (pending random pairs carry over between steps) or "wipe"
    (every step starts afresh)."""
    return dict(Lx=int(Lx), Ly=int(Ly), bx=int(bx), by=int(by), J=float(J),
                h=float(h), T=float(T), rule=rule, window=float(window),
                horizon=float(horizon), seed=int(seed), init=init,
                tick_bits=int(tick_bits), init_spins=init_spins,
                max_iters=int(max_iters), log_mode=log_mode, step=step)


def small() -> Dict:
    return params(64, 64, 16, 16, T=1.5, h=0.0, window=1.0, horizon=50.0,
                  seed=SEED_BASE + 1)


MEDIUM_TEMPS = (1.5, 2.269, 3.0)


def medium(T: float = 3.0, horizon: float = 100.0) -> Dict:
    i = MEDIUM_TEMPS.index(T) if T in MEDIUM_TEMPS else 0
    return params(1024, 1024, 16, 16, T=T, h=0.1, window=0.5, horizon=horizon,
                  seed=SEED_BASE + 2 + (i << 8))


LARGE_WINDOWS = (0.25, 1.0, 4.0)


def large(window: float = 1.0, horizon: float = 200.0) -> Dict:
    return params(4096, 4096, 32, 32, T=1.0, h=0.05, window=window,
                  horizon=horizon, seed=SEED_BASE + 3, init="up")


def batch(n: int = 512, horizon: float = 50.0, seed: int = SEED_BASE + 4) -> List[Dict]:
    """Uneven lattices for the persistent batched form.  Block and window
    are left to the tuner (bx = by = 0, window = 0)."""
    rng = np.random.default_rng(seed)
    Ls = 16 * rng.integers(2, 33, size=n)          # 32, 48, ..., 512
    Ts = rng.uniform(1.0, 3.5, size=n)
    hs = rng.uniform(-0.2, 0.2, size=n)
    out = []
    for i in range(n):
        out.append(params(int(Ls[i]), int(Ls[i]), 0, 0, T=float(Ts[i]),
                          h=float(hs[i]), window=0.0, horizon=horizon,
                          seed=seed * 1000 + i, log_mode="digest"))
    return out


def serve_stream(n: int = 2000, rate: float = 200.0, seed: int = SEED_BASE + 5,
                 Lmin: int = 64, Lmax: int = 2048, hmin: float = 10.0,
                 hmax: float = 100.0) -> List[Dict]:
    """Poisson arrivals (exponential gaps at `rate` per second)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrive = np.cumsum(gaps) - gaps[0]
    logL = rng.uniform(math.log(Lmin), math.log(Lmax), size=n)
    Ls = np.clip(16 * np.rint(np.exp(logL) / 16.0).astype(np.int64), Lmin, Lmax)
    Ts = rng.uniform(1.0, 3.5, size=n)
    hs = rng.uniform(-0.2, 0.2, size=n)
    hor = rng.uniform(hmin, hmax, size=n)
    out = []
    for i in range(n):
        p = params(int(Ls[i]), int(Ls[i]), 0, 0, T=float(Ts[i]), h=float(hs[i]),
                   window=0.0, horizon=float(hor[i]), seed=seed * 1000 + i,
                   log_mode="digest")
        p["t_arrive"] = float(arrive[i])
        p["req_id"] = i
        out.append(p)
    return out


def tuned_block(Lx: int, Ly: int, T: float):
    """The subdomain block the library's tuner assigns to a lattice (a fixed
    table, so that the block, which keys the random streams, depends on the
    request alone): 16x16, or 32x32 for lattices of side >= 2048 at T <= 1.25
    (sparse flips), halved until it divides both sides.  Stated here so that
    stored oracle results of tuned workloads are computed from inputs alone;
    the GPU tests check that the tuner agrees."""
    b = 16
    if min(Lx, Ly) >= 2048 and T <= 1.25:
        b = 32
    while b > 2 and (Lx % b or Ly % b):
        b >>= 1
    return b, b


def random_spins(Lx: int, Ly: int, seed: int, p_up: float = 0.5) -> np.ndarray:
    """User-supplied start configuration (int8 +-1), independent of the
    method's own initial-spin stream."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random((Ly, Lx)) < p_up, 1, -1).astype(np.int8)
