"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer.

  * libretina's host-side argument checks (csrc/validate.h, the code every
    entry point runs before any device work) compiled into a CPU driver
    (tests/sanitize/host_checks.cpp) with valid, invalid and edge inputs;
  * the FP64 oracle (oracle.c) built with the sanitizers and driven from
    Python with the ASan runtime preloaded, on small cases of every routine
    the tests use (meas_dim 1 and 2, empty events, explicit seeds, the grid
    search, the merge, BFGS);
  * both harnesses first shown to catch a planted out-of-bounds read, so that
    a clean run means something.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc / g++")


def _libasan():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _env(extra):
    env = dict(os.environ)
    env.update({"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1",
                "PYTHONPATH": ROOT, "OMP_NUM_THREADS": "4"})
    env.update(extra)
    return env


def _sanitizer_report(text):
    return "AddressSanitizer" in text or "runtime error:" in text


def test_host_check_harness_catches_a_planted_read(tmp_path):
    src = tmp_path / "oob.cpp"
    src.write_text("#include <vector>\nint main(int c, char**) { std::vector<int> v(4); return v.data()[3 + c]; }\n")
    exe = tmp_path / "oob"
    subprocess.check_call(["g++", "-std=c++17"] + SAN + ["-o", str(exe), str(src)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=_env({}))
    assert r.returncode != 0 and _sanitizer_report(r.stderr)


def test_host_checks_under_sanitizers(tmp_path):
    exe = tmp_path / "host_checks"
    subprocess.check_call(["g++", "-std=c++17", "-Wall"] + SAN + ["-I", os.path.join(ROOT, "include"), "-o",
                          str(exe), os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp")])
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=_env({}))
    assert r.returncode == 0, r.stdout + r.stderr
    assert not _sanitizer_report(r.stderr), r.stderr
    assert "all cases passed" in r.stdout


def _run_python_with_asan(lib, code):
    asan = _libasan()
    if asan is None:
        pytest.skip("gcc's libasan.so not found")
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                          env=_env({"LD_PRELOAD": asan, "ORACLE_LIB": str(lib)}), timeout=600)


def test_preload_harness_catches_a_planted_read(tmp_path):
    src = tmp_path / "oob.c"
    src.write_text("int oob(int k) { int a[4] = {1, 2, 3, 4}; volatile int* p = a; return p[k]; }\n")
    lib = tmp_path / "liboob.so"
    subprocess.check_call(["gcc", "-shared", "-fPIC"] + SAN + ["-o", str(lib), str(src)])
    code = "import ctypes; print(ctypes.CDLL(%r).oob(5))" % str(lib)
    r = _run_python_with_asan(lib, code)
    assert r.returncode != 0 and _sanitizer_report(r.stderr)


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    code = textwrap.dedent("""
        import numpy as np, oracle
        from paper_1709_08610_amd import events
        assert oracle._LIB_OVERRIDE, "the sanitizer build is not the one loaded"
        c1 = events.load_config("c1"); b1 = events.make_batch(c1, 1); ev = b1.event(0)
        r = oracle.find_tracks(b1, c1["params"]); assert len(r["theta"]) > 0
        R, G, H = oracle.response(1, b1.plane_z, ev.x, None, ev.plane, oracle.lattice(1, c1["params"]), 0.02)
        oracle.grid_search(1, b1.plane_z, ev.x, None, ev.plane,
                           dict(n=[100, 100], lo=[-1, -0.5], hi=[1, 0.5], sigma=0.02, R0=4.0))
        oracle.polish(1, b1.plane_z, ev.x, None, ev.plane, r["theta"][:, :2], 0.02, 2)
        c3 = events.load_config("c3")
        evs = [events.make_event(c3, i) for i in range(2)]
        empty = events.Event(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.int32),
                             np.zeros(0, np.int32), np.zeros((0, 4)), np.zeros(0, np.int32))
        b3 = events.batch_from_events(2, events.plane_z(c3), [evs[0], empty, evs[1]])
        P = dict(c3["params"], lattice_n=[10, 10])
        r3 = oracle.find_tracks(b3, P)
        seeds = np.concatenate([evs[0].truth[:20], evs[1].truth[:3]])
        r4 = oracle.find_tracks(b3, P, seeds, np.array([0, 20, 20, 23], np.int64))
        for rule in ("gradient", "bfgs"):
            oracle.find_tracks(b3, dict(P, update=rule), seeds, np.array([0, 20, 20, 23], np.int64))
        e0 = b3.event(0)
        R, G, H = oracle.response(2, b3.plane_z, e0.x, e0.y, e0.plane, evs[0].truth[:50], 0.03)
        oracle.merge(2, r4["theta"], r4["R"], np.ones(len(r4["R"]), np.int32), 8.0, 0.03, 20.0, 750.0)
        B = np.eye(4); oracle.bfgs_update(B, np.ones(4), np.arange(4.0) + 1)
        print("oracle under sanitizers: ok")
    """)
    r = _run_python_with_asan(lib, code)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert not _sanitizer_report(r.stderr), r.stderr[-4000:]
    assert "ok" in r.stdout
