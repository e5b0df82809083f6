#!/usr/bin/env python
"""Benchmark of the stabilized implicit MPM hot path on one MI355X.

Headline workload (default): the 3D rigid-footing quarter-model -- trilinear original MPM,
96^3 material cells of h = 0.125 m plus 2 empty layers, 8 points per cell (7,077,888 points,
931,491 grid nodes, 3,725,964 u-p unknowns in 4x4 blocks), neo-Hookean skeleton, k = 1e-12 m^2,
footing pushed 5 mm per step, dt = 0.1 s, quasi-static.  One "step" is one full implicit time
step: sort, P2G, Newton iterations (material-point residual and exact Jacobian with the PPP term,
block-preconditioned BiCGStab), G2P, with Newton driven to 1e-8 relative residual per block.

Reported on the JSON line:
  value        particle-updates/s per Newton step (points x Newton iterations / s) of the FP64 path
  fp64, mixed  both precisions at the same 1e-8 Newton residual (mixed: FP32 Jacobian, SpMV and
               preconditioner, FP64 residual and update), particle-steps/s, p50/p99 step latency,
               Newton/Krylov counts, per-kernel times; an FP64 control at the mixed path's Krylov
               tolerance separates the precision effect from the looser inner solve
  roofline     the SpMV of the Krylov solver (HIP-event launch times inside the library; HBM
               traffic from the committed rocprofv3 counter summary of the same workload and
               precision, if it was taken on the current kernel source); `assembly` the same for
               the Jacobian assembly kernels
  footing2d_large  the 512 x 256-cell 2D GIMP footing (524,288 points), both precisions
  serving      the Poisson stream of 256 independent 2D problems through the continuous-batching
               loop, both precisions on the same trace: throughput and p50/p99 latencies
  cpu_baseline the CPU oracle (single core, pinned) on a bounded sample, run before the GPU is used
  parity       GPU vs the oracle on a 1/8-scale replica of the headline workload, 2 steps
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

DESCR = {
    "footing3d": "footing3d: 3D trilinear quasi-static rigid square-footing quarter-model, 96^3 cells (h=0.125 m) "
                 "+2 empty layers, 7,077,888 points, 931,491 nodes, neo-Hookean E=10 MPa nu=0.3, k=1e-12, "
                 "dt=0.1 s, 5 mm/step, Newton 1e-8 per residual block",
    "footing2d_large": "footing2d_large: 2D GIMP quasi-static rigid-footing half-model, 512x256 cells (h=0.0625 m) "
                       "+16 empty rows, 524,288 points, neo-Hookean E=10 MPa nu=0.3, k from seed 0, "
                       "dt=0.1 s, 5 mm/step, Newton 1e-8 per residual block",
}


def workload(name, scale: int = 1):
    from paper_1905_00671_amd import workloads as W
    if name == "footing3d":
        n = 96 // scale
        return W.footing3d(n=n, size=12.0 * n / 96, half_b=max(0.25, 1.0 * n / 96))
    return W.config(3, nx=512 // scale, ny=256 // scale, width=32.0 / scale, empty_rows=max(2, 16 // scale))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------------------------
# CPU oracle baseline (a child process pinned to one core, run before this process touches the GPU)
# ---------------------------------------------------------------------------------------------
CPU_SAMPLE = r"""
import os, sys, time, json
os.sched_setaffinity(0, {{{core}}})
sys.path.insert(0, {root!r})
import numpy as np
from oracle import oracle as O
from paper_1905_00671_amd import workloads as W
out = {{}}
# (1) two full time steps of a replica of the workload (SuperLU direct solve)
if {name!r} == "footing3d":
    w = W.footing3d(n=12, size=1.5, half_b=0.25)
else:
    w = W.config(3, nx=128, ny=64, width=8.0, empty_rows=4)
pr = O.from_workload(w)
t0 = time.perf_counter(); newton = 0; t_asm = 0.0
for n in (1, 2):
    st = pr.step(w.dt, w.bc(n)); newton += st["newton_iters"]; t_asm += st["t_assemble"]
out["replica"] = dict(seconds=time.perf_counter() - t0, newton=newton, np=pr.np, t_assemble=t_asm)
# (2) the residual of the full-size workload at its first Newton iterate (the residual alone: the
#     oracle's local Jacobians would take about a minute more at 7M points)
if {full}:
    if {name!r} == "footing3d":
        w = W.footing3d()
    else:
        w = W.config(3)
    pr = O.from_workload(w)
    nodal = pr.p2g()
    g, d = w.grid, w.grid.dim
    U = np.zeros((g.nnode, d)); P = nodal["Pn"].copy()
    t0 = time.perf_counter()
    pr.assemble(U, P, nodal, w.dt, want_J=False)
    out["fullsize_assembly"] = dict(seconds=time.perf_counter() - t0, np=pr.np)
print(json.dumps(out))
"""


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, full=True):
    core = sorted(os.sched_getaffinity(0))[0]
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    src = CPU_SAMPLE.format(root=ROOT, name=name, core=core, full=full)
    t0 = time.perf_counter()
    r = subprocess.run([sys.executable, "-c", src], capture_output=True, text=True, env=env, timeout=900)
    if r.returncode != 0:
        return dict(error=r.stderr[-400:])
    d = json.loads(r.stdout.strip().splitlines()[-1])
    rep = d["replica"]
    out = dict(value=rep["np"] * rep["newton"] / rep["seconds"], unit="particle-updates/s", cores=1, kind="oracle",
               sample=(f"2 full time steps ({rep['newton']} Newton iterations, exact Jacobian, SuperLU direct solve) "
                       f"of a {'12^3-cell' if name == 'footing3d' else '128x64-cell'} replica of the workload "
                       f"({rep['np']} points) in {rep['seconds']:.1f} s, of which assembly {rep['t_assemble']:.1f} s"),
               core=core, nproc=os.cpu_count(), cpu_model=cpu_model(), wall_s=time.perf_counter() - t0)
    if "fullsize_assembly" in d:
        fa = d["fullsize_assembly"]
        out["fullsize_assembly"] = dict(seconds=fa["seconds"], points=fa["np"],
                                        what="residual of the full-size workload at its first Newton iterate, one core")
    return out


# ---------------------------------------------------------------------------------------------
# GPU runs
# ---------------------------------------------------------------------------------------------
def device_bcs(w, steps):
    import torch
    out = {}
    for n in steps:
        b = w.bc(n)
        out[n] = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in b.items()}
    torch.cuda.synchronize()
    return out


def run_path(w, precision, warmup, steps, bcs, tag="", **over):
    import torch
    from paper_1905_00671_amd import binding as B
    p = B.Problem.from_workload(w, precision=precision, **over)
    try:
        for n in range(1, warmup + 1):
            ts = time.perf_counter()
            st = p.step(w.dt, bcs[n])
            torch.cuda.synchronize()
            log(f"{tag} precision={precision} warm-up step {n}: {(time.perf_counter() - ts) * 1e3:.1f} ms "
                f"newton={st['newton_iters']} krylov={st['krylov_iters']}")
        # the timed region, as a caller runs it (the Krylov chunks replayed from captured graphs)
        torch.cuda.synchronize()
        lat, stats = [], []
        t0 = time.perf_counter()
        for n in range(warmup + 1, warmup + steps + 1):
            ts = time.perf_counter()
            st = p.step(w.dt, bcs[n])
            lat.append(time.perf_counter() - ts)
            stats.append(st)
            log(f"{tag} precision={precision} step {n}: {lat[-1] * 1e3:.1f} ms newton={st['newton_iters']} "
                f"krylov={st['krylov_iters']}")
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        # kernel-timing pass: the next `steps` steps with HIP events around every launch (direct
        # launches; the events would not fit in a captured graph) for the per-kernel averages
        B.timing_reset()
        B.timing_enable(True)
        kstats = []
        tk = time.perf_counter()
        for n in range(warmup + steps + 1, warmup + 2 * steps + 1):
            kstats.append(p.step(w.dt, bcs[n]))
        torch.cuda.synchronize()
        Tk = time.perf_counter() - tk
        B.timing_enable(False)
        kt = B.timing_get()
        log(f"{tag} precision={precision} kernel-timing pass: {Tk / steps * 1e3:.1f} ms per step")
        ws_bytes = p.workspace_bytes
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
        phase_s=dict(assemble=sum(s["t_assemble"] for s in kstats), precond=sum(s["t_precond"] for s in kstats),
                     krylov=sum(s["t_krylov"] for s in kstats), sort=sum(s["t_sort"] for s in kstats),
                     g2p=sum(s["t_g2p"] for s in kstats)),
        kernels=kt,
        kernel_timing_pass=dict(steps=steps, ms_per_step=Tk / steps * 1e3,
                                newton_per_step=[s["newton_iters"] for s in kstats]),
        hbm_footprint_bytes=ws_bytes,
    )


def stencil(w):
    return 25 if w.options.shape == 1 else (9 if w.grid.dim == 2 else 27)


def spmv_roofline(w, kt, precision):
    """Algorithmic bytes of one SpMV launch: every stored block of the fixed-stencil rows once
    (S b^2 words per grid node), the input vector once, the output and the dot-product vector."""
    g = w.grid
    b = g.dim + 1
    word = 8 if precision == 0 else 4
    bytes_per_launch = g.nnode * (stencil(w) * b * b + 3 * b) * word
    k = kt["spmv"]
    if k["launches"] == 0:
        return None
    avg_s = k["total_ms"] / k["launches"] * 1e-3
    achieved = bytes_per_launch / avg_s / 1e9
    return dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=None, kernel="k_spmv (fixed-stencil block-row SpMV)", bytes_per_launch=bytes_per_launch,
                avg_launch_us=avg_s * 1e6, launches=k["launches"])


def mg0_roofline(w, kt, precision):
    """Finest-level sweeps of the displacement-block multigrid, the launches that stream the
    operator: 3D the row kernels r = b - A x (reads the node's dim x dim blocks over the stencil,
    b, x; writes r) and out = x + omega Dinv (b - A x) (also the inverse diagonal block), so
    S dim^2 + dim^2 / 2 + 3 dim words per node and launch on average; 2D the halo-tiled down and up
    kernels, S dim^2 + dim^2 + 3 dim words (operator, inverse diagonal, b, x, r or out)."""
    g = w.grid
    k = kt["mg0_resid"]
    if k["launches"] == 0:
        return None
    D = g.dim
    word = 8 if precision == 0 else 4
    dd = D * D / 2 if D == 3 else D * D
    bytes_per_launch = g.nnode * (stencil(w) * D * D + dd + 3 * D) * word
    avg_s = k["total_ms"] / k["launches"] * 1e-3
    achieved = bytes_per_launch / avg_s / 1e9
    name = ("k_mg_resid / k_mg_post on the finest level (displacement block)" if D == 3 else
            "k_mg_down / k_mg_up on the finest level (displacement block)")
    return dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=None, kernel=name, bytes_per_launch=bytes_per_launch, avg_launch_us=avg_s * 1e6,
                launches=k["launches"])


# Assembly bytes per material point that the method must move (read x, F_n, V_n[, lp]; its share
# of the Jacobian written once; residual and state): 2D original MPM / 2D GIMP / 3D trilinear,
# FP64 and FP32 Jacobian.
ASM_BYTES_PER_POINT = {(2, 0): (230, 150), (2, 1): (534, 310), (3, 0): (544, 330)}
# Floating-point operations per (point, node pair) of the closed-form pair blocks (basis and
# spatial gradients of both nodes, the b (b+1) x (b+1) entries, the accumulation), counted from the
# formulas the Jacobian kernels evaluate (quasi-static, constant permeability): 3D 4 x 4 blocks
# about 166, 2D 3 x 3 blocks about 95.
JAC_FLOPS_PER_PAIR = {2: 95, 3: 166}
VALU_PEAK_TFLOPS = {0: 78.6, 1: 157.3}     # MI355X vector FP64 / FP32


def assembly_roofline(w, kt, precision):
    """One assembly with the Jacobian (records + residual + Jacobian kernels, average launch
    times): HBM fraction of the per-point algorithmic bytes, and the Jacobian kernels' ALU
    fraction of the pair-block flops against the vector peak of the Jacobian's precision."""
    g = w.grid
    shape = w.options.shape
    if kt["jacobian"]["launches"] == 0:
        return None

    def avg_us(name):
        k = kt[name]
        return k["total_ms"] / k["launches"] * 1e3 if k["launches"] else 0.0

    t_jac = avg_us("jacobian") + avg_us("cellmat")
    t_asm = avg_us("records") + avg_us("residual") + t_jac
    bpp = ASM_BYTES_PER_POINT[(g.dim, shape)][0 if precision == 0 else 1]
    np_ = w.particles.n
    bytes_ = np_ * bpp
    achieved = bytes_ / (t_asm * 1e-6) / 1e9
    nb = (2 if shape == 0 else 3) ** g.dim
    flops = np_ * nb * nb * JAC_FLOPS_PER_PAIR[g.dim]
    tflops = flops / (t_jac * 1e-6) / 1e12
    peak = VALU_PEAK_TFLOPS[0 if precision == 0 else 1]
    return dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=None, kernel="assembly with Jacobian (records + residual + Jacobian kernels)",
                bytes_per_launch=bytes_, bytes_per_point=bpp, avg_launch_us=t_asm,
                records_avg_us=avg_us("records"), residual_avg_us=avg_us("residual"),
                jacobian_avg_us=t_jac, cellmat_avg_us=avg_us("cellmat"),
                alu=dict(bound="alu", kernel="Jacobian kernels", achieved=tflops, peak=peak, unit="TFLOP/s",
                         frac=tflops / peak, flops_per_launch=flops, pairs_per_point=nb * nb,
                         flops_per_pair=JAC_FLOPS_PER_PAIR[g.dim]))


def kernel_digest(fname, signature):
    """sha256 of a kernel's source text (signature line to closing brace)."""
    src = open(os.path.join(ROOT, "paper_1905_00671_amd", "csrc", fname)).read()
    a = src.index(signature)
    b = src.index("\n}\n", a) + 3
    return hashlib.sha256(src[a:b].encode()).hexdigest()


SPMV_SIG = "template <int DIM, int R, typename T>\n__global__ void __launch_bounds__(TPB) k_spmv("
MG_DOWN_SIG = "__global__ void __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(1, FULL ? 2 : 8))) k_mg_down("
MG_UP_SIG = "__global__ void __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(1, FULL ? 2 : 8))) k_mg_up("
MG_ROW_SIG = "__device__ __forceinline__ void row_resid("
MG_LV_SIG = "__device__ __forceinline__ Lv<T> lv_of("
# source digest a counter summary must carry to be used for a kernel (family)
KERNEL_DIGEST = {
    "spmv": lambda: kernel_digest("kern_solver.hip", SPMV_SIG),
    "mg0": lambda: hashlib.sha256((kernel_digest("kern_mg.hip", MG_DOWN_SIG) +
                                   kernel_digest("kern_mg.hip", MG_UP_SIG) +
                                   kernel_digest("kern_mg.hip", MG_ROW_SIG) +
                                   kernel_digest("kern_mg.hip", MG_LV_SIG)).encode()).hexdigest(),
}


def pmc_traffic(name, precision, kernel="spmv"):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this workload and
    kernel (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration), if the summary names
    this workload and precision and was taken on the current kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{name}_pmc.txt")
    if not os.path.exists(path):
        return None
    try:
        digest, per, wl = None, {}, None
        for line in open(path):
            if line.startswith("kernel_source_sha256:"):
                digest = line.split(":", 1)[1].strip()
            if line.startswith("workload:"):
                wl = line.split(":", 1)[1].strip().split()[0]
            m = re.match(r"^(fp64|mixed):.*hbm_bytes_per_launch=([0-9.eE+]+)", line)
            if m:
                per[m.group(1)] = float(m.group(2))
        if wl != name or digest != KERNEL_DIGEST[kernel]():
            return None
        return per.get("fp64" if precision == 0 else "mixed")
    except Exception:
        return None


def bench_workload(name, warmup, steps, control=True):
    """FP64 and mixed paths (and the FP64 control at the mixed Krylov tolerance) on one workload."""
    w = workload(name)
    t = time.perf_counter()
    bcs = device_bcs(w, range(1, warmup + 2 * steps + 1))
    log(f"{name}: {w.particles.n} points, {w.grid.nnode} nodes, inputs on the device in {time.perf_counter() - t:.1f} s")
    res = {"fp64": run_path(w, 0, warmup, steps, bcs, name), "mixed": run_path(w, 1, warmup, steps, bcs, name)}
    if control:
        res["fp64_krylov_1e-6"] = run_path(w, 0, warmup, steps, bcs, name + " control", krylov_rtol=1e-6)
    out = {}
    for key, r in res.items():
        prec = 1 if key == "mixed" else 0
        out[key] = {k: r[k] for k in ("particle_updates_per_s", "particle_steps_per_s", "ms_per_step", "latency_ms",
                                      "newton_iters", "krylov_iters", "newton_per_step", "krylov_per_newton",
                                      "final_rel_residual", "phase_s", "hbm_footprint_bytes", "kernel_timing_pass")}
        out[key]["kernels_ms"] = {k: v for k, v in r["kernels"].items() if v["launches"]}
        spmv = spmv_roofline(w, r["kernels"], prec)
        if spmv is not None:
            spmv["traffic"] = pmc_traffic(name, prec, "spmv")
        mg0 = mg0_roofline(w, r["kernels"], prec)
        if mg0 is not None:
            mg0["traffic"] = pmc_traffic(name, prec, "mg0")
        out[key]["spmv_roofline"] = spmv
        out[key]["mg0_roofline"] = mg0
        # the headline roofline: the kernel (family) with the most device time in the run
        kt = r["kernels"]
        out[key]["roofline"] = (mg0 if mg0 is not None and spmv is not None
                                and kt["mg0_resid"]["total_ms"] > kt["spmv"]["total_ms"] else spmv)
        out[key]["assembly_roofline"] = assembly_roofline(w, r["kernels"], prec)
    out["mixed_vs_fp64"] = dict(
        particle_steps_ratio=res["mixed"]["particle_steps_per_s"] / res["fp64"]["particle_steps_per_s"],
        particle_updates_ratio=res["mixed"]["particle_updates_per_s"] / res["fp64"]["particle_updates_per_s"])
    if control:
        out["mixed_vs_fp64"]["particle_steps_ratio_vs_fp64_krylov_1e-6"] = (
            res["mixed"]["particle_steps_per_s"] / res["fp64_krylov_1e-6"]["particle_steps_per_s"])
    return w, res, out


def parity_check(name):
    """GPU (both precisions) vs the oracle on a 1/8-scale replica, 2 steps, default tolerances;
    element-wise errors of u and p over all points."""
    from oracle import oracle as O
    from paper_1905_00671_amd import binding as B
    out = {}
    w = workload(name, scale=8)
    pr = O.from_workload(w)
    probs = {0: B.Problem.from_workload(w, precision=0), 1: B.Problem.from_workload(w, precision=1)}
    try:
        worst = {0: [0.0, 0.0], 1: [0.0, 0.0]}
        for n in (1, 2):
            pr.step(w.dt, w.bc(n))
            for prec, p in probs.items():
                p.step(w.dt, w.bc(n))
                eu = np.abs(p.get("u") - pr.u).max() / np.abs(pr.u).max()
                ep = np.abs(p.get("p") - pr.p).max() / max(np.abs(pr.p).max(), 1e-3 * np.abs(pr.sig).max())
                worst[prec][0] = max(worst[prec][0], eu)
                worst[prec][1] = max(worst[prec][1], ep)
        for prec, key in ((0, "fp64"), (1, "mixed")):
            out[key] = dict(max_rel_err_u=worst[prec][0], max_rel_err_p=worst[prec][1])
        out["case"] = (f"1/8-scale replica of the workload ({w.particles.n} points), 2 steps, Newton 1e-8, "
                       f"element-wise vs the FP64 oracle")
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
    for key, prec in (("fp64", 0), ("mixed", 1)):
        free, _ = torch.cuda.mem_get_info()
        budget = int(0.8 * free)
        rep = S.serve(trace, budget, realtime=realtime, **S.gpu_backend(prec))
        torch.cuda.synchronize()
        out[key] = rep.summary()
        out[key]["budget_bytes"] = budget
        log(f"serve {key}: {json.dumps(out[key])}")
    return {
        "workload": (f"serving stream: {nreq} requests, Poisson arrivals at 20/s, 2D n=16..256 (log-uniform), "
                     f"k=1e-16..1e-10, 20-50 steps, 50/50 consolidation (original MPM) / footing (GIMP), dt=0.1 s, "
                     f"Newton 1e-8 per block, {'real-time arrivals' if realtime else 'idle gaps skipped'}, "
                     f"admission by workspace bytes within 80% of free HBM"),
        "fp64": out["fp64"],
        "mixed": out["mixed"],
        "mixed_vs_fp64": dict(
            particle_steps_ratio=out["mixed"]["particle_steps_per_s"] / max(out["fp64"]["particle_steps_per_s"], 1e-300),
            particle_updates_ratio=out["mixed"]["particle_updates_per_s"] / max(out["fp64"]["particle_updates_per_s"],
                                                                                 1e-300)),
    }


def dynamic_bench():
    """The undrained dynamic GIMP footing (config 2: 64 x 64 cells, 16,384 points, k = 1e-16,
    Newmark 1/4, 1/2) over 10 steps and the harmonic strip footing of Sec. 5.2 over its first 100
    steps, FP64 then mixed, both with the diagonal-inverse Schur block their workloads select: time
    per step and the Newton / Krylov counts (Table 1: three Newton iterations and 12-17 Krylov
    iterations per Newton iteration at step 100)."""
    import torch
    from paper_1905_00671_amd import binding as B
    from paper_1905_00671_amd import workloads as W
    out = {}
    for key, make, nst in (("footing2d_undrained", lambda: W.config(2), 10),
                           ("harmonic_footing", W.harmonic_footing, 100)):
        o = {}
        for pk, prec in (("fp64", 0), ("mixed", 1)):
            w = make()
            bcs = [w.bc(n) for n in range(1, nst + 1)]
            p = B.Problem.from_workload(w, precision=prec)
            try:
                torch.cuda.synchronize()
                t = time.perf_counter()
                sts = [p.step(w.dt, bcs[n]) for n in range(nst)]
                torch.cuda.synchronize()
                el = time.perf_counter() - t
            finally:
                p.close()
            o[pk] = dict(ms_per_step=1e3 * el / nst, newton_iters=sum(x["newton_iters"] for x in sts),
                         krylov_iters=sum(x["krylov_total"] for x in sts),
                         max_krylov_per_newton=max(max(x["krylov_iters"]) for x in sts),
                         last_step=dict(step=nst, newton=sts[-1]["newton_iters"], krylov=sts[-1]["krylov_iters"]))
            log(f"{key} {pk}: {json.dumps(o[pk])}")
        o["workload"] = f"{w.name}: {w.particles.n} points, {nst} steps, dt={w.dt} s, schur={w.options.schur}"
        o["mixed_vs_fp64"] = o["fp64"]["ms_per_step"] / o["mixed"]["ms_per_step"]
        out[key] = o
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(DESCR), default="footing3d")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline workload only (no 2D footing, serving stream or FP64 Krylov control)")
    ap.add_argument("--serve-only", action="store_true", help="only the serving stream")
    ap.add_argument("--dynamic-only", action="store_true",
                    help="only the dynamic workloads (undrained footing, harmonic footing)")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-no-wait", action="store_true", help="skip idle gaps between arrivals")
    ap.add_argument("--calibrate-mb", type=int, default=0,
                    help="before the run, stream a float32 tensor of this many MiB through one elementwise "
                         "kernel (read once, write once): the reference for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one MI355X: --gpus {args.gpus} is not supported (the library runs the hot path "
              f"on a single GPU; the multi-GPU decomposition is a design only).", file=sys.stderr)
        sys.exit(2)
    name = args.workload
    cpu = None
    if not args.no_cpu_baseline and not args.serve_only and not args.dynamic_only:
        log("CPU oracle baseline (one pinned core) before the GPU is used")
        cpu = cpu_baseline(name)
        log(f"cpu_baseline: {json.dumps(cpu)}")
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    from paper_1905_00671_amd import binding as B
    B.lib()
    if args.serve_only:
        line = serve_bench(args.serve_requests, not args.serve_no_wait)
        line.update(metric="serving: particle-steps/s with continuous batching; p50/p99 step and request latency",
                    value=line["fp64"]["particle_steps_per_s"], unit="particle-steps/s", n_gpus=1,
                    higher_is_better=True, dtype="f64", data="synthetic")
        print(json.dumps(line))
        return
    if args.dynamic_only:
        line = dynamic_bench()
        h = line["harmonic_footing"]
        line.update(metric="harmonic footing (Sec. 5.2): ms per time step", value=h["fp64"]["ms_per_step"],
                    unit="ms/step", n_gpus=1, higher_is_better=False, dtype="f64", data="synthetic")
        print(json.dumps(line))
        return
    if args.calibrate_mb > 0:
        a = torch.ones(args.calibrate_mb * 262144, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        b = a.mul(2.0)
        torch.cuda.synchronize()
        log(f"calibration copy: {a.numel() * 4} bytes read, {b.numel() * 4} bytes written")
        del a, b
    w, res, head = bench_workload(name, args.warmup, args.steps, control=not args.no_extra)
    fp = res["fp64"]
    line = {
        "metric": METRIC,
        "value": fp["particle_updates_per_s"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": DESCR[name],
            "points": w.particles.n,
            "grid_nodes": w.grid.nnode,
            "dofs": w.grid.nnode * (w.grid.dim + 1),
            "k_m2": w.meta["k"],
        },
        "latency_ms": fp["latency_ms"],
        "particle_steps_per_s": fp["particle_steps_per_s"],
        "newton_iters": fp["newton_iters"],
        "krylov_iters": fp["krylov_iters"],
        "hbm_footprint_bytes": {"fp64": res["fp64"]["hbm_footprint_bytes"], "mixed": res["mixed"]["hbm_footprint_bytes"]},
        "roofline": head["fp64"]["roofline"],
        "fp64": head["fp64"],
        "mixed": head["mixed"],
        "mixed_vs_fp64": head["mixed_vs_fp64"],
    }
    if "fp64_krylov_1e-6" in head:
        line["fp64_krylov_1e-6"] = head["fp64_krylov_1e-6"]
    if not args.no_extra:
        other = "footing2d_large" if name == "footing3d" else "footing3d"
        _, _, sub = bench_workload(other, 2 if other == "footing2d_large" else 1,
                                   6 if other == "footing2d_large" else 2, control=False)
        sub["workload"] = DESCR[other]
        line[other] = sub
        line["serving"] = serve_bench(args.serve_requests, not args.serve_no_wait)
        line["dynamic"] = dynamic_bench()
    if not args.no_parity:
        line["parity"] = parity_check(name)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()
