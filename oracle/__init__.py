"""CPU oracle for synchronous relaxation of the n-fold way Ising simulation.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The GPU library never imports it and it
never imports the GPU library.  The C source (`sr_oracle.c`) is plain,
single-threaded and unoptimised; this module is a ctypes wrapper around it.

Entry points:

* ``philox(key, ctr)``          Philox-4x32-10 block (published definition).
* ``expq(u, tick_bits)``        fixed-point -ln(U) in hazard units.
* ``rate_table(J, h, T, rule)`` the 10 class rates (Q28), eqs. pMin/pglauber.
* ``des(p)``                    the plain discrete-event simulation that the
                                converged synchronous relaxation reproduces.
* ``sr(p)``                     literal Jacobi synchronous relaxation (Sec. 4
                                box) on the CPU, with iteration counts g.

A lattice description with ``Lz`` > 1 is a 3D simple-cubic lattice (six
neighbours, 14 classes, blocks bx x by x bz; ``sr_oracle3d.c``): ``des`` and
``sr`` dispatch on it, and ``rate_table3`` gives its 14 class rates.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sr_oracle.c")
_SRC3 = os.path.join(_HERE, "sr_oracle3d.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

METROPOLIS, GLAUBER = 0, 1
INIT = {"random": 0, "up": 1, "user": 2}
RULE = {"metropolis": 0, "glauber": 1, 0: 0, 1: 1}
STEP = {"continue": 0, "wipe": 1, 0: 0, 1: 1}


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-fPIC", "-shared",
           "-ffp-contract=off", "-o", _LIB, _SRC, _SRC3, "-lm"]
    subprocess.check_call(cmd)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("bx", C.c_int32),
                ("by", C.c_int32), ("J", C.c_double), ("h", C.c_double),
                ("T", C.c_double), ("rule", C.c_int32), ("tick_bits", C.c_int32),
                ("init", C.c_int32), ("window_ticks", C.c_int64),
                ("horizon_ticks", C.c_int64), ("burn_ticks", C.c_int64),
                ("seed", C.c_uint64), ("init_spins", C.c_void_p),
                ("step_rule", C.c_int32)]


class _Params3(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("Lz", C.c_int32),
                ("bx", C.c_int32), ("by", C.c_int32), ("bz", C.c_int32),
                ("J", C.c_double), ("h", C.c_double), ("T", C.c_double),
                ("rule", C.c_int32), ("tick_bits", C.c_int32), ("init", C.c_int32),
                ("window_ticks", C.c_int64), ("horizon_ticks", C.c_int64),
                ("burn_ticks", C.c_int64), ("seed", C.c_uint64),
                ("init_spins", C.c_void_p), ("step_rule", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("spins", C.c_void_p), ("log_tick", C.c_void_p),
                ("log_site", C.c_void_p), ("log_sub", C.c_void_p),
                ("log_cap", C.c_int64), ("sub_flips", C.c_void_p),
                ("sub_digest", C.c_void_p), ("snap_M", C.c_void_p),
                ("snap_bond", C.c_void_p), ("carry", C.c_void_p),
                ("n_events", C.c_int64), ("M", C.c_int64), ("bond", C.c_int64),
                ("int_M", C.c_double), ("int_M2", C.c_double),
                ("int_absM", C.c_double), ("int_bond", C.c_double),
                ("int_E2", C.c_double), ("int_M4", C.c_double),
                ("int_ticks", C.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_expq.argtypes = [C.c_uint64, C.c_int]
        L.orc_expq.restype = C.c_uint64
        L.orc_rate_table.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int,
                                     C.POINTER(C.c_uint32)]
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_mix64.restype = C.c_uint64
        L.orc_event_digest.argtypes = [C.c_int64, C.c_int64]
        L.orc_event_digest.restype = C.c_uint64
        L.orc_select_site.argtypes = [C.POINTER(_Params), C.c_void_p, C.c_int,
                                      C.c_uint64, C.POINTER(C.c_int64)]
        L.orc_subdomain_lambda.argtypes = [C.POINTER(_Params), C.c_void_p, C.c_int,
                                           C.POINTER(C.c_uint64)]
        L.orc_des_run.argtypes = [C.POINTER(_Params), C.POINTER(_Result)]
        L.orc_sr_run.argtypes = [C.POINTER(_Params), C.POINTER(_Result),
                                 C.c_void_p, C.c_void_p, C.c_int32]
        L.orc3_rate_table.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int,
                                      C.POINTER(C.c_uint32)]
        L.orc3_select_site.argtypes = [C.POINTER(_Params3), C.c_void_p, C.c_int,
                                       C.c_uint64, C.POINTER(C.c_int64)]
        L.orc3_subdomain_lambda.argtypes = [C.POINTER(_Params3), C.c_void_p, C.c_int,
                                            C.POINTER(C.c_uint64)]
        L.orc3_des_run.argtypes = [C.POINTER(_Params3), C.POINTER(_Result)]
        L.orc3_sr_run.argtypes = [C.POINTER(_Params3), C.POINTER(_Result),
                                  C.c_void_p, C.c_void_p, C.c_int32]
        _lib = L
    return _lib


def is3d(p) -> bool:
    return int(p.get("Lz", 1) or 1) > 1


# ---------------------------------------------------------------- primitives
def philox(key, ctr):
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(k, c, o)
    return tuple(int(x) for x in o)


def expq(u: int, tick_bits: int = 28) -> int:
    return int(lib().orc_expq(C.c_uint64(u & (2**64 - 1)), tick_bits))


def rate_table(J, h, T, rule="metropolis"):
    out = (C.c_uint32 * 10)()
    rc = lib().orc_rate_table(J, h, T, RULE[rule], out)
    if rc != 0:
        raise ValueError("bad rate-table parameters")
    return np.array(list(out), dtype=np.uint32)


def rate_table3(J, h, T, rule="metropolis"):
    """The 14 class rates (Q28) of the 3D lattice, class 7*[s=-1] + n_up."""
    out = (C.c_uint32 * 14)()
    rc = lib().orc3_rate_table(J, h, T, RULE[rule], out)
    if rc != 0:
        raise ValueError("bad rate-table parameters")
    return np.array(list(out), dtype=np.uint32)


def mix64(z: int) -> int:
    """SplitMix64 finaliser (the 64-bit mixer of the event digests)."""
    return int(lib().orc_mix64(C.c_uint64(z & (2**64 - 1))))


def event_digest(tick: int, site: int) -> int:
    return int(lib().orc_event_digest(tick, site))


def to_ticks(x: float, tick_bits: int) -> int:
    """Round-half-away-from-zero of x * 2^tick_bits (x >= 0)."""
    y = float(x) * (1 << tick_bits)         # exact: power-of-two scaling
    f = math.floor(y)
    return int(f) + (1 if y - f >= 0.5 else 0)


def _cparams(p, burn=0.0, window=None):
    tb = int(p.get("tick_bits", 28))
    w = p["window"] if window is None else window
    if is3d(p):
        cp = _Params3()
        cp.Lz, cp.bz = int(p["Lz"]), int(p["bz"])
    else:
        cp = _Params()
    cp.Lx, cp.Ly, cp.bx, cp.by = p["Lx"], p["Ly"], p["bx"], p["by"]
    cp.J, cp.h, cp.T = p["J"], p["h"], p["T"]
    cp.rule = RULE[p.get("rule", "metropolis")]
    cp.tick_bits = tb
    cp.init = INIT[p.get("init", "random")]
    cp.window_ticks = max(1, to_ticks(w, tb)) if w > 0 else to_ticks(p["horizon"], tb) or 1
    cp.horizon_ticks = to_ticks(p["horizon"], tb)
    cp.burn_ticks = to_ticks(burn, tb)
    cp.seed = p["seed"] & (2**64 - 1)
    cp.step_rule = STEP[p.get("step", "continue")]
    keep = None
    if cp.init == 2:
        keep = np.ascontiguousarray(p["init_spins"], dtype=np.int8).reshape(-1)
        cp.init_spins = keep.ctypes.data
    return cp, keep


def select_site(p, spins, d, V):
    cp, _keep = _cparams(p)
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    out = C.c_int64()
    fn = lib().orc3_select_site if is3d(p) else lib().orc_select_site
    rc = fn(C.byref(cp), s.ctypes.data, d, C.c_uint64(V), C.byref(out))
    if rc != 0:
        raise ValueError(f"select_site failed ({rc})")
    return int(out.value)


def subdomain_lambda(p, spins, d):
    cp, _keep = _cparams(p)
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    out = C.c_uint64()
    fn = lib().orc3_subdomain_lambda if is3d(p) else lib().orc_subdomain_lambda
    rc = fn(C.byref(cp), s.ctypes.data, d, C.byref(out))
    if rc != 0:
        raise ValueError("subdomain_lambda failed")
    return int(out.value)


# ---------------------------------------------------------------- full runs
def _run(p, kind, log=True, burn=0.0, log_cap=None, max_iters=0):
    cp, keep = _cparams(p, burn=burn)
    three = is3d(p)
    Lz = int(p["Lz"]) if three else 1
    nsub = (p["Lx"] // p["bx"]) * (p["Ly"] // p["by"]) * (Lz // int(p["bz"]) if three else 1)
    nsite = p["Lx"] * p["Ly"] * Lz
    nwin = 0 if cp.horizon_ticks == 0 else -(-cp.horizon_ticks // cp.window_ticks)
    if log_cap is None:
        log_cap = int(1.25 * nsite * p["horizon"]) + 4096 if log else 0
    while True:
        spins = np.zeros(nsite, dtype=np.int8)
        lt = np.zeros(max(log_cap, 1), dtype=np.int64)
        ls = np.zeros(max(log_cap, 1), dtype=np.int64)
        lsub = np.zeros(max(log_cap, 1), dtype=np.int32)
        flips = np.zeros(nsub, dtype=np.int64)
        dig = np.zeros(nsub, dtype=np.uint64)
        sM = np.zeros(nwin + 1, dtype=np.int64)
        sB = np.zeros(nwin + 1, dtype=np.int64)
        carry = np.zeros(4 * nsub, dtype=np.int64)
        g = np.zeros(max(nwin, 1), dtype=np.int32)
        f = np.zeros(max(nwin, 1), dtype=np.int32)
        r = _Result()
        r.spins = spins.ctypes.data
        r.log_tick, r.log_site, r.log_sub = lt.ctypes.data, ls.ctypes.data, lsub.ctypes.data
        r.log_cap = log_cap
        r.sub_flips, r.sub_digest = flips.ctypes.data, dig.ctypes.data
        r.snap_M, r.snap_bond = sM.ctypes.data, sB.ctypes.data
        r.carry = carry.ctypes.data
        if kind == "des":
            fn = lib().orc3_des_run if three else lib().orc_des_run
            rc = fn(C.byref(cp), C.byref(r))
        else:
            fn = lib().orc3_sr_run if three else lib().orc_sr_run
            rc = fn(C.byref(cp), C.byref(r), g.ctypes.data, f.ctypes.data, max_iters)
        if rc != 0:
            raise RuntimeError(f"oracle {kind} failed with code {rc}")
        if not log or r.n_events <= log_cap:
            break
        log_cap = int(r.n_events)
    n = int(r.n_events)
    shape = (Lz, p["Ly"], p["Lx"]) if three else (p["Ly"], p["Lx"])
    out = dict(spins=spins.reshape(shape), n_events=n,
               sub_flips=flips, sub_digest=dig, snap_M=sM, snap_bond=sB,
               carry=carry.reshape(nsub, 4), M=int(r.M), bond=int(r.bond),
               int_M=r.int_M, int_M2=r.int_M2, int_absM=r.int_absM,
               int_bond=r.int_bond, int_E2=r.int_E2, int_M4=r.int_M4,
               int_ticks=int(r.int_ticks), window_ticks=int(cp.window_ticks),
               horizon_ticks=int(cp.horizon_ticks))
    if log:
        out.update(log_tick=lt[:n].copy(), log_site=ls[:n].copy(), log_sub=lsub[:n].copy())
    if kind == "sr":
        out.update(g=g[:nwin].copy(), f=f[:nwin].copy())
    out["digest"] = int(np.sum(dig, dtype=np.uint64))
    return out


def des(p, log=True, burn=0.0):
    """Plain DES over [0, horizon).  Returns final spins, the event log in
    (tick, subdomain) order, per-subdomain flips and digests, M and bond sum
    at every committed time k*window, per-subdomain carry (j, anchor, acc,
    next) and tick-weighted sums of M, M^2, |M|, bond, E^2, M^4 over
    [burn, horizon)."""
    return _run(p, "des", log=log, burn=burn)


def sr(p, log=True, max_iters=0):
    """Literal synchronous relaxation on the CPU; adds g (iterations per
    window, including the confirming one) and f (most boundary-site events of
    one subdomain in one iteration) per window."""
    return _run(p, "sr", log=log, max_iters=max_iters)
