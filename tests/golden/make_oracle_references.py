"""Writes the oracle's reference states for the GPU parity tests of the benchmark configurations
whose oracle runs take minutes to hours on one core (config 2: 100 dynamic steps; config 3:
several seeds; config 4: a 24^3 replica over all 20 steps; the harmonic strip footing over its
400 steps; the two-body impact on a coarse grid through contact).

TEST INFRASTRUCTURE: calls only the CPU oracle (oracle/) and the seeded input generators
(paper_1905_00671_amd/workloads.py, no method arithmetic).  Nothing here runs the HIP library.
The GPU tests (tests/test_gpu_configs.py) step the same workloads through the C ABI and compare
the sampled material points element by element with the files written here.

Usage (single-threaded, as the oracle is specified):
    OMP_NUM_THREADS=1 OPENBLAS_NUM_THREADS=1 python tests/golden/make_oracle_references.py [case ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1905_00671_amd import workloads as W  # noqa: E402

# Newton is driven to 1e-10 per residual block in the references, so that the comparison with the
# GPU path measures the implementation, not the stopping point of the nonlinear iteration.
NEWTON_RTOL = 1e-10


def _config2(tau_kind):
    return W.config(2, tau_kind=tau_kind)


def _config3(seed):
    return W.config(3, nx=128, ny=64, width=8.0, empty_rows=4, nsteps=4, seed=seed)


def _config4_replica():
    return W.footing3d(n=24, size=3.0, half_b=0.25, nsteps=20)


# name -> (workload factory, steps, snapshot steps, sample stride over the points)
CASES = {
    "config2_tauW": (lambda: _config2(W.TAU_WHITE), 100, (10, 50, 90), 16),
    "config2_tau0": (lambda: _config2(W.TAU_OFF), 100, (10, 50, 100), 16),
    "config4_r24": (_config4_replica, 20, (1, 10, 20), 64),
    # Sec. 5.2: harmonic strip footing, consistent mass, point tractions, all 400 steps
    "harmonic_footing": (lambda: W.harmonic_footing(), 400, (100, 200, 300, 400), 8),
    # Sec. 5.4: two-body impact on a coarse grid (h = 0.05 m, 2 x 2 points per cell), through the
    # contact at t ~ 1.5 s and the rebound
    "impact_coarse": (lambda: W.two_body_impact(h=0.05, ppa=2), 2200, (1000, 1600, 2000, 2200), 1),
}
for _s in range(5):
    CASES[f"config3_seed{_s}_128x64"] = ((lambda s=_s: _config3(s)), 4, (1, 4), 32)


def path(name):
    return os.path.join(HERE, f"oracle_{name}.npz")


def snapshot(pr, idx):
    """Material-point state of the sampled points (caller order)."""
    out = dict(u=pr.u[idx], p=pr.p[idx], x=pr.x[idx], F=pr.F[idx], vol=pr.V[idx], sig=pr.sig[idx],
               lp=pr.lp[idx])
    if pr.opt.dynamic:
        out.update(v=pr.v[idx], a=pr.a[idx], pd=pr.pd[idx], pdd=pr.pdd[idx])
    return out


def run(name):
    make, nsteps, snaps, stride = CASES[name]
    w = make()
    w.options.newton_rtol = NEWTON_RTOL
    pr = O.from_workload(w)
    idx = np.arange(0, w.particles.n, stride)
    data = dict(sample=idx, newton=np.zeros(nsteps, np.int64), u_norm=np.zeros(nsteps), p_norm=np.zeros(nsteps),
                p_max=np.zeros(nsteps), sig_max=np.zeros(nsteps))
    t0 = time.perf_counter()
    data["last_step"] = np.array(nsteps)
    for n in range(1, nsteps + 1):
        try:
            st = pr.step(w.dt, w.bc(n))
        except O.NewtonFailure as e:
            # the run ends where the oracle's own Newton iteration no longer converges
            data["last_step"] = np.array(n - 1)
            print(f"[{name}] step {n}: {e}; the reference ends at step {n - 1}", flush=True)
            break
        data["newton"][n - 1] = st["newton_iters"]
        data["u_norm"][n - 1] = np.linalg.norm(pr.u)
        data["p_norm"][n - 1] = np.linalg.norm(pr.p)
        data["p_max"][n - 1] = np.abs(pr.p).max()
        data["sig_max"][n - 1] = np.abs(pr.sig).max()
        if n in snaps:
            for k, v in snapshot(pr, idx).items():
                data[f"s{n}_{k}"] = v
        print(f"[{name}] step {n}/{nsteps}: newton={st['newton_iters']} {time.perf_counter() - t0:.1f} s",
              flush=True)
    data["snaps"] = np.array([k for k in snaps if k <= int(data["last_step"])])
    np.savez_compressed(path(name), **data)
    print(f"[{name}] wrote {path(name)}", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        run(name)
