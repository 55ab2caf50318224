"""Host runtime of the library (window loop, tuner, batched form, serving,
checkpoints) under AddressSanitizer and UBSan, without a GPU.

sr_api.hip is compiled with g++ against a host-only stand-in for the HIP
runtime and the kernel launchers (tests/host_mock): device memory is host
memory and the stand-in "kernels" only drive convergence and window
bookkeeping.  This checks memory safety and bookkeeping of the host code
(buffer sizes, lifetimes, budgets), not the physics, which the GPU parity
tests cover."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MOCK = os.path.join(ROOT, "tests", "host_mock")


def _build(tmp_path_factory, name, sanitize):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("host_rt") / name)
    cmd = [gxx, "-std=c++17", "-g", "-O1", *sanitize, "-fno-omit-frame-pointer", "-pthread", f"-I{MOCK}",
           "-x", "c++", os.path.join(ROOT, "paper_cs_0405053_amd", "csrc", "sr_api.hip"),
           "-x", "c++", os.path.join(MOCK, "mock_runtime.cpp"),
           "-x", "c++", os.path.join(MOCK, "drive.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.fixture(scope="module")
def drive(tmp_path_factory):
    return _build(tmp_path_factory, "drive", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])


@pytest.fixture(scope="module")
def drive_tsan(tmp_path_factory):
    return _build(tmp_path_factory, "drive_tsan", ["-fsanitize=thread"])


def run(exe, scenario, **env):
    e = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", SR_MOCK_G="1")
    e.update({k: str(v) for k, v in env.items()})
    r = subprocess.run([exe, scenario], capture_output=True, text=True, timeout=120, env=e)
    assert r.returncode == 0 and f"ok {scenario}" in r.stdout, (r.stdout + r.stderr)[-4000:]
    return r.stdout


def test_tuned_window_count_exceeds_first_estimate(drive):
    # windows needing 40 iterations shrink the tuned step size, so far more
    # windows are committed than the first window predicts; the iteration
    # counts must still land only in caller-bounded buffers
    out = run(drive, "tuned", SR_MOCK_G=40)
    assert "windows" in out


@pytest.mark.parametrize("graphs", ["0", "1"])
def test_tuned_window_plain_and_graph_paths(drive, graphs):
    run(drive, "tuned", SR_MOCK_G=48, SR_NO_GRAPHS=graphs)


@pytest.mark.parametrize("g", [1, 7])
def test_server_rounds_then_plain_sims(drive, g):
    run(drive, "server", SR_MOCK_G=g)


def test_server_with_overflow_fallback(drive):
    run(drive, "server", SR_MOCK_G=3, SR_MOCK_OVERFLOW=1)


@pytest.mark.parametrize("give_ups", [1, 3, 100])
def test_server_continues_lattices_a_launch_gave_up_on(drive, give_ups):
    out = run(drive, "server_give_up", SR_MOCK_GIVE_UP=give_ups)
    assert ("gave up waiting" in out) == (give_ups > 3)


@pytest.mark.parametrize("give_ups", [2, 100])
def test_batch_run_continues_lattices_a_launch_gave_up_on(drive, give_ups):
    run(drive, "batch_give_up", SR_MOCK_GIVE_UP=give_ups)


@pytest.mark.parametrize("overflow", [0, 1])
def test_batch_budget_resume_reset(drive, overflow):
    run(drive, "batch", SR_MOCK_G=4, SR_MOCK_OVERFLOW=overflow)


def test_batch_log_overflow_at_list_capacity_limit(drive):
    # only the window log overflowed, on a lattice whose lists are already at
    # their largest capacity: the fallback grows the log and completes
    run(drive, "batch", SR_MOCK_G=4, SR_MOCK_OVERFLOW=2)


@pytest.mark.parametrize("overflow", [0, 1])
def test_static_batch_step_allocates_nothing(drive, overflow):
    run(drive, "static", SR_MOCK_G=3, SR_MOCK_OVERFLOW=overflow)


def test_checkpoint_and_argument_errors(drive):
    run(drive, "errors")


def test_threads_drive_separate_simulations(drive):
    run(drive, "threads", SR_MOCK_G=3)


def test_batched_runs_from_threads_with_give_ups(drive):
    run(drive, "batch_threads", SR_MOCK_G=2, SR_MOCK_GIVE_UP=3)


def test_batched_runs_from_threads_without_data_races(drive_tsan):
    r = subprocess.run([drive_tsan, "batch_threads"], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, SR_MOCK_G="2", SR_MOCK_GIVE_UP="3", TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0 and "ok batch_threads" in r.stdout, (r.stdout + r.stderr)[-4000:]


def test_threads_without_data_races(drive_tsan):
    # ThreadSanitizer: the only state shared between handles is the
    # per-thread creation error
    r = subprocess.run([drive_tsan, "threads"], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, SR_MOCK_G="3", TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0 and "ok threads" in r.stdout, (r.stdout + r.stderr)[-4000:]


@pytest.mark.parametrize("regrow", [0, 1])
def test_window_graphs_from_eight_threads(drive, regrow):
    # the library's own graph building (kernel nodes whose arguments live on
    # the builder's stack, graphs dropped and rebuilt when lists grow) under
    # AddressSanitizer, from eight threads at once
    run(drive, "graph_threads", SR_MOCK_G=5, SR_MOCK_REGROW=regrow)


def test_window_graphs_from_eight_threads_without_races(drive_tsan):
    r = subprocess.run([drive_tsan, "graph_threads"], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, SR_MOCK_G="5", SR_MOCK_REGROW="1", TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0 and "ok graph_threads" in r.stdout, (r.stdout + r.stderr)[-4000:]
