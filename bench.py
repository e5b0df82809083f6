#!/usr/bin/env python
"""Benchmark of the stabilized implicit MPM hot path on one MI355X.

Workload: the large 2D quasi-static footing -- GIMP basis, 512 x 256 material cells of
h = 0.0625 m plus 16 empty rows, 4 points per cell (524,288 points), neo-Hookean skeleton,
permeability drawn once from seed 0, rigid footing pushed 5 mm per step, dt = 0.1 s.
One "step" is one full implicit time step (sort, P2G, Newton iterations with assembly and the
block-preconditioned BiCGStab, G2P) with Newton driven to 1e-8 relative residual per block.

Reported: particle-updates/s per Newton step (points x Newton iterations / s) for the FP64 path
(the headline value) and for the mixed path (FP32 Jacobian, SpMV, preconditioner; FP64 residual
and update) at the same 1e-8 residual; particle-steps/s; p50/p99 step latency; the SpMV roofline
from HIP events recorded inside the library; the CPU oracle on a bounded sample; a small parity
check against the oracle.
"""
import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-updates/s per Newton step, p50/p99 latency; FP32-mixed vs FP64 at 1e-8 resid"


WORKLOAD = "footing2d_large"
DESCR = {
    "footing2d_large": "footing2d_large: 2D GIMP quasi-static rigid-footing half-model, 512x256 cells (h=0.0625 m) "
                       "+16 empty rows, 524,288 points, neo-Hookean E=10 MPa nu=0.3, k from seed 0, "
                       "dt=0.1 s, 5 mm/step, Newton 1e-8 per residual block",
    "footing3d": "footing3d: 3D trilinear quasi-static rigid square-footing quarter-model, 96^3 cells (h=0.125 m) "
                 "+2 empty layers, 7,077,888 points, neo-Hookean E=10 MPa nu=0.3, k=1e-12, dt=0.1 s, "
                 "5 mm/step, Newton 1e-8 per residual block",
}


def workload(scale: int = 1):
    from paper_1905_00671_amd import workloads as W
    if WORKLOAD == "footing3d":
        n = 96 // scale
        return W.footing3d(n=n, size=12.0 * n / 96, half_b=max(0.25, 1.0 * n / 96))
    return W.config(3, nx=512 // scale, ny=256 // scale, width=32.0 / scale, empty_rows=max(2, 16 // scale))


def device_bcs(w, steps):
    import torch
    out = {}
    for n in steps:
        b = w.bc(n)
        out[n] = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in b.items()}
    torch.cuda.synchronize()
    return out


def run_path(w, precision, warmup, steps, bcs):
    import torch
    from paper_1905_00671_amd import binding as B
    p = B.Problem.from_workload(w, precision=precision)
    try:
        for n in range(1, warmup + 1):
            ts = time.perf_counter()
            st = p.step(w.dt, bcs[n])
            torch.cuda.synchronize()
            print(f"[bench] precision={precision} warm-up step {n}: {(time.perf_counter() - ts) * 1e3:.1f} ms "
                  f"newton={st['newton_iters']} krylov={st['krylov_iters']}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        B.timing_reset()
        B.timing_enable(True)
        lat, stats = [], []
        t0 = time.perf_counter()
        for n in range(warmup + 1, warmup + steps + 1):
            ts = time.perf_counter()
            st = p.step(w.dt, bcs[n])
            lat.append(time.perf_counter() - ts)
            stats.append(st)
            print(f"[bench] precision={precision} step {n}: {lat[-1] * 1e3:.1f} ms newton={st['newton_iters']} "
                  f"krylov={st['krylov_iters']}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        B.timing_enable(False)
        kt = B.timing_get()
    finally:
        p.close()
    npt = w.particles.n
    newton = sum(s["newton_iters"] for s in stats)
    krylov = sum(s["krylov_total"] for s in stats)
    lat_ms = np.array(lat) * 1e3
    return dict(
        particle_updates_per_s=npt * newton / T,
        particle_steps_per_s=npt * steps / T,
        seconds=T,
        ms_per_step=T / steps * 1e3,
        latency_ms=dict(p50=float(np.percentile(lat_ms, 50)), p99=float(np.percentile(lat_ms, 99))),
        newton_iters=newton,
        krylov_iters=krylov,
        newton_per_step=[s["newton_iters"] for s in stats],
        krylov_per_newton=[s["krylov_iters"] for s in stats],
        final_rel_residual=[max(s["res_u"][-1] / max(s["res_u"][0], 1e-300), s["res_p"][-1] / max(s["res_p"][0], 1e-300))
                            for s in stats],
        phase_s=dict(assemble=sum(s["t_assemble"] for s in stats), precond=sum(s["t_precond"] for s in stats),
                     krylov=sum(s["t_krylov"] for s in stats), sort=sum(s["t_sort"] for s in stats),
                     g2p=sum(s["t_g2p"] for s in stats)),
        kernels=kt,
    )


def spmv_roofline(w, kt, precision):
    """Algorithmic bytes of one SpMV launch: every stored block of the fixed-stencil rows once
    (S b^2 words per grid node), the input vector once, the output and the dot-product vector."""
    g = w.grid
    nnode = g.nnode
    b = g.dim + 1
    S = 25 if w.options.shape == 1 else (9 if g.dim == 2 else 27)
    word = 8 if precision == 0 else 4
    bytes_per_launch = nnode * (S * b * b + 3 * b) * word
    k = kt["spmv"]
    if k["launches"] == 0:
        return None
    avg_s = k["total_ms"] / k["launches"] * 1e-3
    achieved = bytes_per_launch / avg_s / 1e9
    return dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=None, kernel="k_spmv (stencil block-CSR SpMV)", bytes_per_launch=bytes_per_launch,
                avg_launch_us=avg_s * 1e6, launches=k["launches"])


def spmv_source_digest():
    """sha256 of the SpMV kernel's source text (template line to closing brace)."""
    src = open(os.path.join(ROOT, "paper_1905_00671_amd", "csrc", "kern_solver.hip")).read()
    a = src.index("template <int DIM, int R, typename T>\n__global__ void __launch_bounds__(TPB) k_spmv(")
    b = src.index("\n}\n", a) + 3
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def pmc_traffic(roof, precision):
    """HBM bytes per SpMV launch from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by the copy-kernel calibration), if it was taken on the current kernel
    source; None otherwise."""
    path = os.path.join(ROOT, "profiles", "spmv_footing2d_large_pmc.txt")
    if roof is None or not os.path.exists(path):
        return None
    try:
        digest, per = None, {}
        for line in open(path):
            if line.startswith("kernel_source_sha256:"):
                digest = line.split(":", 1)[1].strip()
            m = re.match(r"^(fp64|mixed):.*hbm_bytes_per_launch=([0-9.eE+]+)", line)
            if m:
                per[m.group(1)] = float(m.group(2))
        if digest != spmv_source_digest():
            return None
        return per.get("fp64" if precision == 0 else "mixed")
    except Exception:
        return None


CPU_SAMPLE = r"""
import os, sys, time, json
sys.path.insert(0, {root!r})
from oracle import oracle as O
from paper_1905_00671_amd import workloads as W
w = W.config(3, nx=128, ny=64, width=8.0, empty_rows=4)
pr = O.from_workload(w)
t0 = time.perf_counter(); newton = 0
for n in (1, 2):
    st = pr.step(w.dt, w.bc(n)); newton += st["newton_iters"]
T = time.perf_counter() - t0
print(json.dumps(dict(seconds=T, newton=newton, np=pr.np)))
"""


def cpu_baseline():
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", CPU_SAMPLE.format(root=ROOT)], capture_output=True, text=True,
                       env=env, timeout=600)
    if r.returncode != 0:
        return dict(error=r.stderr[-400:])
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return dict(value=d["np"] * d["newton"] / d["seconds"], unit="particle-updates/s", cores=1, kind="oracle",
                sample=f"2 full time steps ({d['newton']} Newton iterations, SuperLU direct solve) of a 128x64-cell "
                       f"replica of the footing workload ({d['np']} points), single thread, {d['seconds']:.1f} s",
                seconds=d["seconds"])


def parity_check():
    """GPU (both precisions) vs the oracle on a 64x32 replica, 2 steps, default tolerances."""
    from oracle import oracle as O
    from paper_1905_00671_amd import binding as B
    out = {}
    w = workload(scale=8)
    pr = O.from_workload(w)
    probs = {0: B.Problem.from_workload(w, precision=0), 1: B.Problem.from_workload(w, precision=1)}
    try:
        worst = {0: [0.0, 0.0], 1: [0.0, 0.0]}
        for n in (1, 2):
            pr.step(w.dt, w.bc(n))
            for prec, p in probs.items():
                p.step(w.dt, w.bc(n))
                eu = np.linalg.norm(p.get("u") - pr.u) / np.linalg.norm(pr.u)
                ep = np.linalg.norm(p.get("p") - pr.p) / max(np.linalg.norm(pr.p), 1e-300)
                worst[prec][0] = max(worst[prec][0], eu)
                worst[prec][1] = max(worst[prec][1], ep)
        for prec, name in ((0, "fp64"), (1, "mixed")):
            out[name] = dict(rel_err_u=worst[prec][0], rel_err_p=worst[prec][1])
        out["case"] = f"1/8-scale replica of the workload ({w.particles.n} points), 2 steps, Newton 1e-8, vs FP64 oracle"
    finally:
        for p in probs.values():
            p.close()
    return out


def serve_bench(nreq, realtime):
    """The serving stream (Poisson arrivals of 2D consolidation / footing problems) through the
    continuous-batching loop, FP64 then mixed, on the same trace."""
    import torch
    from paper_1905_00671_amd import serving as S
    from paper_1905_00671_amd import workloads as W
    trace = W.serving_trace(nreq=nreq)
    out = {}
    for name, prec in (("fp64", 0), ("mixed", 1)):
        free, _ = torch.cuda.mem_get_info()
        budget = int(0.8 * free)
        rep = S.serve(trace, budget, realtime=realtime, **S.gpu_backend(prec))
        torch.cuda.synchronize()
        out[name] = rep.summary()
        out[name]["budget_bytes"] = budget
        print(f"[serve] {name}: {out[name]}", file=sys.stderr, flush=True)
    line = {
        "metric": "serving: particle-steps/s with continuous batching; p50/p99 step and request latency",
        "value": out["fp64"]["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serving stream: {nreq} requests, Poisson arrivals at 20/s, 2D n=16..256 "
                               f"(log-uniform), k=1e-16..1e-10, 20-50 steps, 50/50 consolidation (linear) / "
                               f"footing (GIMP), dt=0.1 s, {'real-time arrivals' if realtime else 'idle gaps skipped'}"},
        "fp64": out["fp64"],
        "mixed": out["mixed"],
        "mixed_vs_fp64": out["mixed"]["particle_steps_per_s"] / max(out["fp64"]["particle_steps_per_s"], 1e-300),
    }
    print(json.dumps(line))


def main():
    global WORKLOAD
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--workload", choices=sorted(DESCR), default=WORKLOAD)
    ap.add_argument("--serve", action="store_true",
                    help="run the serving stream (continuous batching) instead of the footing step benchmark")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-no-wait", action="store_true", help="skip idle gaps between arrivals")
    ap.add_argument("--calibrate-mb", type=int, default=0,
                    help="before the run, stream a float32 tensor of this many MiB through one elementwise "
                         "kernel (read once, write once): the reference for hardware byte counters")
    args = ap.parse_args()
    WORKLOAD = args.workload
    if args.gpus != 1:
        print(f"bench.py measures one MI355X: --gpus {args.gpus} is not supported (the library runs the hot path "
              f"on a single GPU; the multi-GPU decomposition is a design only).", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    from paper_1905_00671_amd import binding as B
    B.lib()
    if args.serve:
        serve_bench(args.serve_requests, not args.serve_no_wait)
        return
    if args.calibrate_mb > 0:
        a = torch.ones(args.calibrate_mb * 262144, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        b = a.mul(2.0)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {a.numel() * 4} bytes read, {b.numel() * 4} bytes written",
              file=sys.stderr, flush=True)
        del a, b
    w = workload()
    bcs = device_bcs(w, range(1, args.warmup + args.steps + 1))
    res = {}
    if args.precision in ("both", "fp64"):
        res["fp64"] = run_path(w, 0, args.warmup, args.steps, bcs)
    if args.precision in ("both", "mixed"):
        res["mixed"] = run_path(w, 1, args.warmup, args.steps, bcs)
    head = res.get("fp64") or res.get("mixed")
    head_prec = 0 if "fp64" in res else 1
    roof = spmv_roofline(w, head["kernels"], head_prec)
    if roof is not None:
        roof["traffic"] = pmc_traffic(roof, head_prec)
    line = {
        "metric": METRIC,
        "value": head["particle_updates_per_s"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_prec == 0 else "mixed-f32/f64",
        "data": "synthetic",
        "config": {
            "workload": DESCR[WORKLOAD],
            "points": w.particles.n,
            "grid_nodes": w.grid.nnode,
            "dofs": w.grid.nnode * (w.grid.dim + 1),
            "k_m2": w.meta["k"],
        },
        "latency_ms": head["latency_ms"],
        "particle_steps_per_s": head["particle_steps_per_s"],
        "newton_iters": head["newton_iters"],
        "krylov_iters": head["krylov_iters"],
        "roofline": roof,
    }
    for name in ("fp64", "mixed"):
        if name in res:
            r = res[name]
            line[name] = {k: r[k] for k in ("particle_updates_per_s", "particle_steps_per_s", "ms_per_step",
                                            "latency_ms", "newton_iters", "krylov_iters", "newton_per_step",
                                            "krylov_per_newton", "final_rel_residual", "phase_s")}
            line[name]["kernels_ms"] = {k: v for k, v in r["kernels"].items() if v["launches"]}
    if "fp64" in res and "mixed" in res:
        line["mixed_vs_fp64"] = dict(
            particle_steps_ratio=res["mixed"]["particle_steps_per_s"] / res["fp64"]["particle_steps_per_s"],
            particle_updates_ratio=res["mixed"]["particle_updates_per_s"] / res["fp64"]["particle_updates_per_s"])
        roof32 = spmv_roofline(w, res["mixed"]["kernels"], 1)
        if roof32 is not None:
            roof32["traffic"] = pmc_traffic(roof32, 1)
        line["mixed"]["roofline"] = roof32
    if not args.no_parity:
        line["parity"] = parity_check()
    if not args.no_cpu_baseline and WORKLOAD == "footing2d_large":
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
