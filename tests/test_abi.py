"""The C ABI library loads and exports every symbol include/sr.h declares;
parameter validation runs on the host (no device work, no GPU needed)."""
import re
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sr_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_cs_0405053_amd as sr
    lib = sr.lib()
    declared = _declared()
    assert "sr_create" in declared and "sr_run_window" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(sr.EXPORTS) == declared


def test_one_hip_runtime_per_process():
    # PyTorch ships its own HIP runtime; the binding loads it before libsr.so
    # so that both use one runtime (with two, whichever initialises last
    # finds no device).  A fresh process, loading the library first.
    code = ("import paper_cs_0405053_amd as sr; sr.lib(); "
            "print(sorted(set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l)))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    runtimes = eval(r.stdout.strip().splitlines()[-1])
    assert len(runtimes) == 1, runtimes


@pytest.mark.parametrize("bad", [
    dict(bx=7),                  # does not divide Lx
    dict(bx=1, by=1),            # blocks too small
    dict(T=0.0),
    dict(tick_bits=40),
    dict(horizon=-1.0),
    dict(rule=5),
    dict(window=-1.0),
    dict(Lx=2, Ly=2, bx=2, by=2),
    dict(bx=32, by=48, Ly=96),   # bx*by > 1024
    dict(Lx=128, bx=128, by=4),  # bx > 64
    dict(init="user"),           # no spins given
    dict(step="wipe", window=0.0),   # wipe rule with a tuned window
    dict(step=7),                # unknown step rule
    dict(Lz=2, bz=2),            # 3D needs Lz >= 4
    dict(Lz=16, bz=16),          # 3D face 16x16 > 64 sites
    dict(Lz=16, bz=3),           # does not divide Lz
    dict(Lz=16, bx=8, by=8, bz=1),   # block side 1
])
def test_invalid_parameters_rejected(bad):
    import paper_cs_0405053_amd as sr
    p = dict(Lx=64, Ly=64, bx=16, by=16, T=1.5, h=0.0, window=1.0, horizon=5.0, seed=1)
    p.update(bad)
    if p.get("step") == 7:
        import ctypes
        cp, _ = sr.to_params(dict(p, step="continue"))
        cp.step_rule = 7
        h = ctypes.c_void_p()
        assert sr.lib().sr_create(ctypes.byref(cp), None, ctypes.byref(h)) == sr.SR_EINVAL
        return
    if p.get("rule") == 5:
        p["rule"] = 1
        p["T"] = -1.0
    with pytest.raises(sr.SRError) as e:
        sr.Sim(p)
    assert e.value.code == sr.SR_EINVAL


def test_tuner_block_is_deterministic_and_valid():
    import paper_cs_0405053_amd as sr
    for L in (32, 48, 64, 96, 512, 1024, 2048, 4096):
        for T in (1.0, 2.0, 3.5):
            bx, by, w = sr.tune(dict(Lx=L, Ly=L, T=T, horizon=10.0))
            assert L % bx == 0 and L % by == 0 and w > 0
            assert (bx, by, w) == sr.tune(dict(Lx=L, Ly=L, T=T, horizon=10.0))


def test_tuner_block_matches_stated_workload_block():
    # stored oracle results of tuned workloads use workloads.tuned_block
    import paper_cs_0405053_amd as sr
    import workloads as W
    ps = W.batch() + W.serve_stream(n=256)
    for p in ps:
        bx, by, _ = sr.tune(p)
        assert (bx, by) == W.tuned_block(p["Lx"], p["Ly"], p["T"]), p
    for L in (32, 48, 64, 80, 96, 1000, 2048, 4096):
        for T in (1.0, 1.25, 1.3, 3.0):
            bx, by, _ = sr.tune(dict(Lx=L, Ly=L, T=T, horizon=1.0))
            assert (bx, by) == W.tuned_block(L, L, T), (L, T)


def test_rate_table3_host_entry_equals_oracle():
    import numpy as np
    import oracle
    import paper_cs_0405053_amd as sr
    rng = np.random.default_rng(5)
    for _ in range(500):
        J, h, T = float(rng.uniform(-2, 2)), float(rng.uniform(-1, 1)), float(rng.uniform(0.2, 8))
        rule = ["metropolis", "glauber"][int(rng.integers(0, 2))]
        p = dict(Lx=8, Ly=8, Lz=8, J=J, h=h, T=T, rule=rule, horizon=1.0)
        assert np.array_equal(sr.rate_table(p), oracle.rate_table3(J, h, T, rule)), (J, h, T, rule)


def test_tuner3_cubic_block():
    import paper_cs_0405053_amd as sr
    for L, want in ((8, 8), (16, 8), (12, 4), (20, 4), (6, 2), (64, 8)):
        bx, by, w = sr.tune(dict(Lx=L, Ly=L, Lz=L, T=4.0, horizon=1.0))
        assert (bx, by) == (want, want) and 0.125 <= w <= 2.0


def test_binding_structures_match_the_header(tmp_path):
    """Every structure the binding mirrors has the header's size and field
    offsets (compiled from include/sr.h with the host C compiler)."""
    import ctypes
    import shutil
    import paper_cs_0405053_amd as sr
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    mirrors = {"sr_params": sr.Params, "sr_obs": sr.Obs, "sr_result": sr.Result,
               "sr_server_info": sr.ServerInfo}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "sr.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, timeout=60).stdout.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
