"""The oracle's C kernels (oracle/oracle.c) built with AddressSanitizer and UndefinedBehaviorSanitizer
and driven through representative steps: 2D original MPM (Terzaghi), 2D GIMP Newmark with Kelvin
damping, the 3D footing, consistent-mass mapping with point tractions, self-weight consolidation
(gravity, Hencky, Kozeny-Carman, drained free surface) and the two-body impact (point pressure
conditions).  Any out-of-bounds access or undefined operation aborts the child process."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import sys
sys.path.insert(0, sys.argv[2])
from oracle import oracle as O
O.build = lambda force=False: sys.argv[1]
from paper_1905_00671_amd import workloads as W

def run(w, n):
    pr = O.from_workload(w)
    for k in range(1, n + 1):
        pr.step(w.dt, w.bc(k))

run(W.config(1, nsteps=2), 2)
w = W.config(2, nx=12, ny=12, width=2.0, empty_rows=2, nsteps=2)
w.material.alpha_vis = 0.04
run(w, 2)
run(W.footing3d(n=4, size=1.0, half_b=0.25, nsteps=1), 1)
w = W.config(3, nx=32, ny=16, width=2.0, empty_rows=2, nsteps=1)
w.options.consistent_mass = 1
run(w, 1)
run(W.harmonic_footing(h=1.0, width=4.0, depth=4.0), 1)
run(W.self_weight(h=0.25, ppa=2), 2)
run(W.two_body_impact(h=0.05, ppa=2), 2)
print("sanitized oracle ok", flush=True)
'''


def _libasan():
    if shutil.which("gcc") is None:
        return None
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return os.path.realpath(p) if p and os.path.exists(p) else None


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    asan = _libasan()
    if asan is None:
        pytest.skip("gcc with libasan is not available")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    script = tmp_path / "run.py"
    script.write_text(SCRIPT)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(script), lib, ROOT], capture_output=True, text=True, env=env,
                       timeout=600, cwd=str(tmp_path))
    report = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, report
    assert "sanitized oracle ok" in r.stdout, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
