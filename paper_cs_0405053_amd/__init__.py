"""Python binding of the MI355X synchronous-relaxation library (libsr.so).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI declared in ``include/sr.h``.  The library must have
been built (``python -m paper_cs_0405053_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.

Typical use::

    import paper_cs_0405053_amd as sr
    sim = sr.Sim(dict(Lx=64, Ly=64, bx=16, by=16, J=1.0, h=0.0, T=1.5,
                      window=1.0, horizon=50.0, seed=1))
    g = sim.run()                 # iterations per committed window
    obs = sim.observables()
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsr.so")

SR_OK, SR_EINVAL, SR_ENOMEM, SR_EOVERFLOW, SR_ENOCONV, SR_EDEVICE, SR_EDONE = 0, -1, -2, -3, -4, -5, -6
_RULE = {"metropolis": 0, "glauber": 1, 0: 0, 1: 1}
_INIT = {"random": 0, "up": 1, "user": 2, 0: 0, 1: 1, 2: 2}
_LOG = {"digest": 0, "full": 1, 0: 0, 1: 1}
_STEP = {"continue": 0, "wipe": 1, 0: 0, 1: 1}

# every function the C ABI exports (include/sr.h)
EXPORTS = ["sr_create", "sr_run_window", "sr_observables", "sr_destroy", "sr_get_spins",
           "sr_get_log", "sr_get_digests", "sr_get_carry", "sr_get_rate_table", "sr_rate_table",
           "sr_save",
           "sr_load", "sr_last_error", "sr_batch_run", "sr_tune", "sr_reset",
           "sr_batch_step", "sr_batch_step_static", "sr_server_create", "sr_server_submit", "sr_server_pump",
           "sr_server_poll", "sr_server_stats", "sr_server_destroy"]


class SRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("bx", C.c_int32), ("by", C.c_int32),
                ("J", C.c_double), ("h", C.c_double), ("T", C.c_double), ("rule", C.c_int32),
                ("window", C.c_double), ("horizon", C.c_double), ("seed", C.c_uint64),
                ("init", C.c_int32), ("init_spins", C.c_void_p), ("log_mode", C.c_int32),
                ("max_iters", C.c_int32), ("tick_bits", C.c_int32), ("hist_cap", C.c_int32),
                ("wlog_cap", C.c_int32), ("step_rule", C.c_int32), ("Lz", C.c_int32),
                ("bz", C.c_int32)]


class Obs(C.Structure):
    _fields_ = [("tick", C.c_int64), ("M", C.c_int64), ("bond_sum", C.c_int64),
                ("flips", C.c_int64), ("events_processed", C.c_int64), ("windows", C.c_int64),
                ("iterations", C.c_int64), ("last_g", C.c_int32), ("last_f", C.c_int32),
                ("tick_bits", C.c_int32), ("n_sub", C.c_int32), ("bx", C.c_int32),
                ("by", C.c_int32), ("Lx", C.c_int32), ("Ly", C.c_int32),
                ("window_ticks", C.c_int64), ("horizon_ticks", C.c_int64),
                ("relax_launches", C.c_int64), ("relax_ms", C.c_double),
                ("subdomain_runs", C.c_int64), ("Lz", C.c_int32), ("bz", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("digest", C.c_uint64), ("M", C.c_int64),
                ("bond_sum", C.c_int64), ("flips", C.c_int64), ("events_processed", C.c_int64),
                ("windows", C.c_int64), ("iterations", C.c_int64), ("t_arrive", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double), ("status", C.c_int32),
                ("bx", C.c_int32), ("by", C.c_int32)]


class ServerInfo(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("queued", C.c_int64), ("rounds", C.c_int64), ("bytes_in_use", C.c_int64),
                ("peak_bytes", C.c_int64), ("peak_active", C.c_int32), ("restarts", C.c_int32),
                ("busy_s", C.c_double), ("uptime_s", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load libsr.so; raises if it was never built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_cs_0405053_amd.build`")
        # One HIP runtime per process: PyTorch ships its own copy, and loaded
        # before libsr.so it also serves libsr.so; loaded after, it would be a
        # second runtime in the process, and whichever of the two initialises
        # last finds no device.  So torch (when installed) comes first, and
        # torch streams passed to the library belong to the same runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.sr_create.argtypes = [C.POINTER(Params), P, C.POINTER(P)]
        L.sr_run_window.argtypes = [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.sr_observables.argtypes = [P, C.POINTER(Obs)]
        L.sr_destroy.argtypes = [P]
        L.sr_destroy.restype = None
        L.sr_get_spins.argtypes = [P, P]
        L.sr_get_log.argtypes = [P, C.c_int32, P, P, C.c_int64, C.POINTER(C.c_int64)]
        L.sr_get_digests.argtypes = [P, P, P]
        L.sr_get_carry.argtypes = [P, P]
        L.sr_get_rate_table.argtypes = [P, P]
        L.sr_rate_table.argtypes = [C.POINTER(Params), P]
        L.sr_save.argtypes = [P, P, C.c_size_t, C.POINTER(C.c_size_t)]
        L.sr_load.argtypes = [P, C.c_size_t, P, C.POINTER(P)]
        L.sr_last_error.argtypes = [P]
        L.sr_last_error.restype = C.c_char_p
        L.sr_batch_run.argtypes = [P, C.c_int32, P]
        L.sr_reset.argtypes = [P]
        L.sr_batch_step.argtypes = [P, C.c_int32, C.c_int32, P]
        L.sr_batch_step_static.argtypes = [P, C.c_int32, C.c_int32, P]
        L.sr_server_create.argtypes = [C.c_size_t, C.c_int32, P, C.POINTER(P)]
        L.sr_server_submit.argtypes = [P, C.POINTER(Params), C.POINTER(C.c_uint64)]
        L.sr_server_pump.argtypes = [P, C.POINTER(C.c_int32)]
        L.sr_server_poll.argtypes = [P, P, C.c_int32, C.POINTER(C.c_int32)]
        L.sr_server_stats.argtypes = [P, C.POINTER(ServerInfo)]
        L.sr_server_destroy.argtypes = [P]
        L.sr_server_destroy.restype = None
        L.sr_tune.argtypes = [C.POINTER(Params), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                              C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)           # a torch.cuda.Stream


def to_params(p: Dict) -> (Params, Optional[np.ndarray]):
    cp = Params()
    cp.Lx, cp.Ly = int(p["Lx"]), int(p["Ly"])
    cp.bx, cp.by = int(p.get("bx", 0)), int(p.get("by", 0))
    cp.J, cp.h, cp.T = float(p.get("J", 1.0)), float(p.get("h", 0.0)), float(p["T"])
    cp.rule = _RULE[p.get("rule", "metropolis")]
    cp.window, cp.horizon = float(p.get("window", 0.0)), float(p["horizon"])
    cp.seed = int(p.get("seed", 0)) & (2**64 - 1)
    cp.init = _INIT[p.get("init", "random")]
    keep = None
    if cp.init == 2 and p.get("init_spins") is not None:
        keep = np.ascontiguousarray(p["init_spins"], dtype=np.int8).reshape(-1)
        nz = int(p.get("Lz", 0) or 0)
        if keep.size != cp.Lx * cp.Ly * max(nz, 1):
            raise SRError(SR_EINVAL, "init_spins must hold Lx*Ly (3D: Lx*Ly*Lz) values")
        cp.init_spins = keep.ctypes.data
    cp.log_mode = _LOG[p.get("log_mode", "digest")]
    cp.max_iters = int(p.get("max_iters", 0))
    cp.tick_bits = int(p.get("tick_bits", 0))
    cp.hist_cap = int(p.get("hist_cap", 0))
    cp.wlog_cap = int(p.get("wlog_cap", 0))
    cp.step_rule = _STEP[p.get("step", "continue")]
    cp.Lz = int(p.get("Lz", 0) or 0)
    cp.bz = int(p.get("bz", 0) or 0)
    return cp, keep


def last_error(handle=None) -> str:
    m = lib().sr_last_error(handle)
    return m.decode() if m else ""


def tune(p: Dict):
    """(bx, by, window) the tuner would choose."""
    cp, _ = to_params(p)
    bx, by, w = C.c_int32(), C.c_int32(), C.c_double()
    rc = lib().sr_tune(C.byref(cp), C.byref(bx), C.byref(by), C.byref(w))
    if rc != SR_OK:
        raise SRError(rc, "tuner rejected the lattice")
    return bx.value, by.value, w.value


def rate_table(p: Dict) -> np.ndarray:
    """The class rates the library computes for these parameters (host only,
    no device work): 10 in 2D, 14 for a 3D lattice (Lz > 1)."""
    cp, _ = to_params(p)
    r = np.zeros(14, dtype=np.uint32)
    rc = lib().sr_rate_table(C.byref(cp), r.ctypes.data)
    if rc != SR_OK:
        raise SRError(rc, "sr_rate_table rejected the parameters")
    return r[:14 if cp.Lz > 1 else 10].copy()


class Sim:
    """One lattice simulation (owns its device state)."""

    def __init__(self, p: Dict = None, stream=None, _handle=None):
        self._h = None
        if _handle is not None:
            self._h = _handle
            return
        cp, keep = to_params(p)
        h = C.c_void_p()
        rc = lib().sr_create(C.byref(cp), _stream_ptr(stream), C.byref(h))
        del keep
        if rc != SR_OK:
            raise SRError(rc, last_error(None))
        self._h = h

    # -- lifetime
    def close(self):
        if self._h is not None:
            lib().sr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, what):
        if rc != SR_OK:
            raise SRError(rc, f"{what}: {last_error(self._h)}")

    @property
    def handle(self):
        return self._h

    # -- the method
    def run(self, n_windows: int = -1) -> np.ndarray:
        """Commit up to n_windows windows (all remaining if < 0); returns the
        iterations g of each committed window."""
        # The step size may change after every window (tuned windows), so the
        # number of windows is not known ahead: fetch g in bounded chunks.
        out = []
        want = n_windows
        while want != 0:
            o = self.observables()
            if o["tick"] >= o["horizon_ticks"]:
                break
            chunk = 256 if want < 0 else min(want, 256)
            g = np.zeros(chunk, dtype=np.int32)
            done = C.c_int32()
            rc = lib().sr_run_window(self._h, chunk, g.ctypes.data_as(C.POINTER(C.c_int32)),
                                     C.byref(done))
            out.append(g[:done.value].copy())
            self._check(rc, "sr_run_window")
            if want > 0:
                want -= done.value
        return np.concatenate(out) if out else np.zeros(0, dtype=np.int32)

    def reset(self) -> None:
        """Back to time 0 with the initial spins; keeps all allocations."""
        self._check(lib().sr_reset(self._h), "sr_reset")

    def observables(self) -> Dict:
        o = Obs()
        self._check(lib().sr_observables(self._h, C.byref(o)), "sr_observables")
        return {k: getattr(o, k) for k, _ in Obs._fields_}

    def spins(self) -> np.ndarray:
        o = self.observables()
        nz = o["Lz"] if o["Lz"] > 1 else 1
        buf = np.zeros(nz * o["Ly"] * o["Lx"], dtype=np.int8)
        self._check(lib().sr_get_spins(self._h, buf.ctypes.data), "sr_get_spins")
        return buf.reshape(nz, o["Ly"], o["Lx"]) if o["Lz"] > 1 else buf.reshape(o["Ly"], o["Lx"])

    def log(self, d: int):
        n = C.c_int64()
        self._check(lib().sr_get_log(self._h, d, None, None, 0, C.byref(n)), "sr_get_log")
        t = np.zeros(max(n.value, 1), dtype=np.int64)
        v = np.zeros(max(n.value, 1), dtype=np.int64)
        self._check(lib().sr_get_log(self._h, d, t.ctypes.data, v.ctypes.data, n.value,
                                     C.byref(n)), "sr_get_log")
        return t[:n.value], v[:n.value]

    def digests(self):
        n = self.observables()["n_sub"]
        dg = np.zeros(n, dtype=np.uint64)
        fl = np.zeros(n, dtype=np.int64)
        self._check(lib().sr_get_digests(self._h, dg.ctypes.data, fl.ctypes.data),
                    "sr_get_digests")
        return dg, fl

    def carry(self) -> np.ndarray:
        n = self.observables()["n_sub"]
        c = np.zeros(3 * n, dtype=np.int64)
        self._check(lib().sr_get_carry(self._h, c.ctypes.data), "sr_get_carry")
        return c.reshape(n, 3)

    def rate_table(self) -> np.ndarray:
        r = np.zeros(14, dtype=np.uint32)
        self._check(lib().sr_get_rate_table(self._h, r.ctypes.data), "sr_get_rate_table")
        return r[:14 if self.observables()["Lz"] > 1 else 10].copy()

    def save(self) -> bytes:
        n = C.c_size_t()
        self._check(lib().sr_save(self._h, None, 0, C.byref(n)), "sr_save")
        buf = C.create_string_buffer(n.value)
        self._check(lib().sr_save(self._h, buf, n.value, C.byref(n)), "sr_save")
        return buf.raw

    @classmethod
    def load(cls, blob: bytes, stream=None) -> "Sim":
        h = C.c_void_p()
        b = C.create_string_buffer(blob, len(blob))
        rc = lib().sr_load(b, len(blob), _stream_ptr(stream), C.byref(h))
        if rc != SR_OK:
            raise SRError(rc, last_error(None))
        return cls(_handle=h)


def batch_step(sims: Sequence[Sim], max_windows: int, stream=None) -> None:
    """Every simulation commits at most max_windows more windows, in one
    persistent launch (continuous-batching scheduling step)."""
    arr = (C.c_void_p * len(sims))(*[s.handle for s in sims])
    rc = lib().sr_batch_step(arr, len(sims), max_windows, _stream_ptr(stream))
    if rc != SR_OK:
        raise SRError(rc, "sr_batch_step: " + last_error(sims[0].handle if sims else None))


def batch_step_static(sims: Sequence[Sim], max_windows: int, stream=None) -> None:
    """batch_step without any device allocation: the launch's queue and
    records live in the library's fixed per-GPU array (sr_batch_step_static)."""
    arr = (C.c_void_p * len(sims))(*[s.handle for s in sims])
    rc = lib().sr_batch_step_static(arr, len(sims), max_windows, _stream_ptr(stream))
    if rc != SR_OK:
        raise SRError(rc, "sr_batch_step_static: " + last_error(sims[0].handle if sims else None))


def batch_run(sims: Sequence[Sim], stream=None) -> None:
    """Run every simulation to its horizon in one persistent launch."""
    arr = (C.c_void_p * len(sims))(*[s.handle for s in sims])
    rc = lib().sr_batch_run(arr, len(sims), _stream_ptr(stream))
    if rc != SR_OK:
        raise SRError(rc, "sr_batch_run: " + last_error(sims[0].handle if sims else None))


class Server:
    """Continuous-batching request loop, driven by the caller: `submit`
    queues a request; `pump` keeps one persistent launch running over the
    admitted lattices, ends it at the next window boundaries when a request
    can be admitted or a lattice finished, then retires, admits by HBM
    footprint and relaunches; `poll` returns retired results."""

    def __init__(self, hbm_budget: int, windows_per_round: int = 0, stream=None):
        h = C.c_void_p()
        rc = lib().sr_server_create(int(hbm_budget), int(windows_per_round), _stream_ptr(stream),
                                    C.byref(h))
        if rc != SR_OK:
            raise SRError(rc, last_error(None))
        self._h = h

    def submit(self, p: Dict) -> int:
        cp, keep = to_params(dict(p, log_mode="digest"))
        rid = C.c_uint64()
        rc = lib().sr_server_submit(self._h, C.byref(cp), C.byref(rid))
        del keep
        if rc != SR_OK:
            raise SRError(rc, last_error(None))
        return int(rid.value)

    def pump(self) -> int:
        """One scheduling step (retire, admit, (re)launch, or ask the running
        launch to end at the next window boundaries); waits at most about a
        millisecond.  Returns the requests not yet retired."""
        n = C.c_int32()
        rc = lib().sr_server_pump(self._h, C.byref(n))
        if rc != SR_OK:
            raise SRError(rc, "sr_server_pump: " + last_error(None))
        return int(n.value)

    def poll(self, cap: int = 1024) -> List[Dict]:
        buf = (Result * cap)()
        n = C.c_int32()
        rc = lib().sr_server_poll(self._h, buf, cap, C.byref(n))
        if rc != SR_OK:
            raise SRError(rc, "sr_server_poll")
        return [{k: getattr(buf[i], k) for k, _ in Result._fields_} for i in range(n.value)]

    def stats(self) -> Dict:
        o = ServerInfo()
        lib().sr_server_stats(self._h, C.byref(o))
        return {k: getattr(o, k) for k, _ in ServerInfo._fields_}

    def close(self):
        if self._h is not None:
            lib().sr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
