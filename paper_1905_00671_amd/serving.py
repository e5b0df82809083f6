"""Serving loop: a stream of independent poromechanics problems stepped with continuous batching.

Requests arrive over time (``workloads.serving_trace``).  A request is admitted, in arrival order,
as soon as it has arrived and its device workspace (``ppmpm_workspace_bytes``) fits into what is
left of the memory budget; admitted problems are advanced together, one time step each per
scheduling round, through ``ppmpm_step_batched`` (one launch per kernel phase for all problems of
a kernel variant); a problem leaves the batch when its last step is done (or a step fails) and its
workspace is returned to the budget before the next admission.  Every problem's kernels are
independent of the others in its batch, so a request's results do not depend on what it was
batched with.

The scheduler is written against four callables so that its bookkeeping runs without a GPU:
``bytes_of(req)``, ``open_problem(req)``, ``step_many(handles, reqs, step_indices)`` and
``close_problem(handle, req)``; ``gpu_backend()`` supplies the real ones.
"""
from __future__ import annotations

import json
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Job:
    req: object
    nbytes: int
    handle: object = None
    steps_done: int = 0
    t_admit: float = 0.0
    t_done: float = -1.0
    failed: bool = False
    newton: int = 0
    krylov: int = 0


@dataclass
class Report:
    completed: int = 0
    failed: int = 0
    rejected: int = 0
    rounds: int = 0
    wall_s: float = 0.0
    particle_steps: int = 0
    particle_updates: int = 0                                        # points x Newton iterations
    step_latency_ms: List[float] = field(default_factory=list)       # one entry per request step
    request_latency_s: List[float] = field(default_factory=list)     # arrival -> last step done
    batch_sizes: List[int] = field(default_factory=list)
    peak_bytes: int = 0
    newton_iters: int = 0
    krylov_iters: int = 0

    def summary(self) -> Dict:
        sl = np.array(self.step_latency_ms) if self.step_latency_ms else np.zeros(1)
        rl = np.array(self.request_latency_s) if self.request_latency_s else np.zeros(1)
        return dict(
            completed=self.completed, failed=self.failed, rejected=self.rejected, rounds=self.rounds,
            wall_s=self.wall_s,
            particle_steps_per_s=self.particle_steps / self.wall_s if self.wall_s > 0 else 0.0,
            particle_updates_per_s=self.particle_updates / self.wall_s if self.wall_s > 0 else 0.0,
            step_latency_ms=dict(p50=float(np.percentile(sl, 50)), p99=float(np.percentile(sl, 99))),
            request_latency_s=dict(p50=float(np.percentile(rl, 50)), p99=float(np.percentile(rl, 99))),
            mean_batch=float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            max_batch=int(max(self.batch_sizes)) if self.batch_sizes else 0,
            peak_bytes=self.peak_bytes, newton_iters=self.newton_iters, krylov_iters=self.krylov_iters)


def serve(requests: Sequence, budget_bytes: int, *, bytes_of: Callable, open_problem: Callable,
          step_many: Callable, close_problem: Callable, points_of: Callable = lambda r: 0,
          realtime: bool = True, clock: Callable[[], float] = time.perf_counter,
          sleep: Callable[[float], None] = time.sleep, max_active: int = 256,
          on_finish: Optional[Callable] = None, on_step: Optional[Callable] = None) -> Report:
    """Runs the request stream to completion and returns the report.

    realtime: arrivals are honoured on the wall clock (the loop sleeps while nothing is active);
    otherwise the clock skips idle gaps, so arrival order and admission still follow the trace
    but no time is spent waiting.  ``on_finish(job)`` is called before a finished problem is closed;
    ``on_step(job, step, stats, latency_ms)`` after every request step (``jsonl_step_log``).
    """
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    active: List[Job] = []
    used = 0
    rep = Report()
    t0 = clock()
    skipped = 0.0      # idle time skipped when not in real time

    def now() -> float:
        return clock() - t0 + skipped

    while pending or active:
        # admission, strictly in arrival order
        while pending and pending[0].arrival <= now() and len(active) < max_active:
            r = pending[0]
            nb = int(bytes_of(r))
            if nb <= 0 or nb > budget_bytes:
                pending.popleft()
                rep.rejected += 1
                continue
            if used + nb > budget_bytes:
                break
            pending.popleft()
            job = Job(req=r, nbytes=nb, t_admit=now())
            job.handle = open_problem(r)
            used += nb
            rep.peak_bytes = max(rep.peak_bytes, used)
            active.append(job)
        if not active:
            if pending:
                gap = pending[0].arrival - now()
                if gap > 0:
                    if realtime:
                        sleep(gap)
                    else:
                        skipped += gap
            continue
        ts = clock()
        stats = step_many([j.handle for j in active], [j.req for j in active],
                          [j.steps_done + 1 for j in active])
        te = clock()
        rep.rounds += 1
        rep.batch_sizes.append(len(active))
        keep = []
        for j, st in zip(active, stats):
            rep.step_latency_ms.append((te - ts) * 1e3)
            if on_step is not None:
                on_step(j, j.steps_done + 1, st, (te - ts) * 1e3)
            j.newton += int(st.get("newton_iters", 0))
            rep.particle_updates += int(points_of(j.req)) * int(st.get("newton_iters", 0))
            j.krylov += int(st.get("krylov_total", 0))
            if int(st.get("status", 0)) != 0:
                j.failed = True
            else:
                j.steps_done += 1
                rep.particle_steps += int(points_of(j.req))
            if j.failed or j.steps_done >= j.req.nsteps:
                j.t_done = now()
                if j.failed:
                    rep.failed += 1
                else:
                    rep.completed += 1
                    rep.request_latency_s.append(j.t_done - j.req.arrival)
                rep.newton_iters += j.newton
                rep.krylov_iters += j.krylov
                if on_finish is not None:
                    on_finish(j)
                close_problem(j.handle, j.req)
                used -= j.nbytes
            else:
                keep.append(j)
        active = keep
    rep.wall_s = clock() - t0
    return rep


def jsonl_step_log(fh) -> Callable:
    """An ``on_step`` callback that writes one JSON line per request step to the text stream fh:
    the request id, step index, status, batch latency, and what the runtime reports for the step
    (Newton iterations and their block-wise residual history, Krylov iterations per Newton
    iteration, phase times)."""
    def log(job, step, st, latency_ms):
        rec = {"request": getattr(job.req, "rid", None), "step": int(step), "latency_ms": float(latency_ms)}
        for k, v in st.items():
            rec[k] = [float(x) if isinstance(x, float) else int(x) for x in v] if isinstance(v, (list, tuple)) else v
        fh.write(json.dumps(rec) + "\n")
    return log


def gpu_backend(precision: int, workload_cache: Optional[Dict] = None, **over):
    """bytes_of / open_problem / step_many / close_problem / points_of on the C ABI; `over`
    overrides method options of every problem (e.g. newton_rtol, krylov_rtol)."""
    import ctypes

    from . import binding as B

    cache = workload_cache if workload_cache is not None else {}

    def wl(r):
        w = cache.get(r.rid)
        if w is None:
            w = r.workload()
            cache[r.rid] = w
        return w

    def bytes_of(r):
        w = wl(r)
        g = B.make_grid(w.grid)
        o = B.make_options(w.options, precision=precision, **over)
        return int(B.lib().ppmpm_workspace_bytes(ctypes.byref(g), w.particles.n, ctypes.byref(o)))

    def open_problem(r):
        return B.Problem.from_workload(wl(r), precision=precision, **over)

    def step_many(handles, reqs, steps):
        ws = [wl(r) for r in reqs]
        return B.step_batched(handles, [w.dt for w in ws], [w.bc(n) for w, n in zip(ws, steps)])

    def close_problem(h, r):
        h.close()
        cache.pop(r.rid, None)

    def points_of(r):
        return wl(r).particles.n

    return dict(bytes_of=bytes_of, open_problem=open_problem, step_many=step_many,
                close_problem=close_problem, points_of=points_of)
