"""PA_LOG, the library's diagnostic log on stderr (CPU, no GPU).

Each case runs in a fresh process, since the level is read once per
process: off by default; "error" (or 1) reports every failing call with its
status and message; "info" (2) adds server set-up; "debug" (3) adds
spectrum builds and evictions of the serving scheduler.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import ctypes
import paper_1809_07592_amd as pa
u64p = ctypes.POINTER(ctypes.c_uint64)
p = lambda a: ctypes.cast(a, u64p)
assert pa.lib().pa_toeplitz_hash(p(0x1000), 100, p(0x2000), 101, p(0x3000), None) == pa.PA_ERR_INVALID_ARG
n, m = 200_000, 50_000
budget = 2 * 4 * pa.transform_len(n, m) + 4096
with pa.Server(budget, max_inflight=2, executor=pa.EXEC_SIMULATED, sim_bits_per_us=1e6) as s:
    a = s.register_seed(0x100000, n + m)
    b = s.register_seed(0x200000, n + m)
    s.wait(s.submit(a, 0x300000, n, m, 0x400000))
    s.wait(s.submit(b, 0x300000, n, m, 0x400000))
print("done")
"""


def run(level):
    env = dict(os.environ, PYTHONPATH=ROOT)
    env.pop("PA_LOG", None)
    if level is not None:
        env["PA_LOG"] = level
    r = subprocess.run([sys.executable, "-c", CODE], env=env, capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0 and "done" in r.stdout, r.stderr[-3000:]
    return [ln for ln in r.stderr.splitlines() if ln.startswith("[pa] ")]


def test_off_by_default():
    assert run(None) == []
    assert run("off") == [] and run("0") == []


def test_error_level_reports_failing_calls():
    for level in ("error", "1"):
        lines = run(level)
        assert any("error: PA_ERR_INVALID_ARG" in ln and "m > n" in ln for ln in lines), lines
        assert not any(ln.startswith("[pa] info") or ln.startswith("[pa] debug") for ln in lines)


def test_info_and_debug_levels():
    info = run("info")
    assert any("info: server: budget" in ln and "simulated executor" in ln for ln in info), info
    assert not any(ln.startswith("[pa] debug") for ln in info)
    debug = run("3")
    assert any("debug: server: building the spectrum of seed 0" in ln for ln in debug), debug
    # the pool holds one spectrum and one workspace: seed 1 evicts seed 0's
    assert any("debug: server: evicting the spectrum of seed 0" in ln for ln in debug), debug
