"""Serving loop: admission and batching bookkeeping on the CPU with a fake backend; on the GPU,
results of requests served in a mixed batch equal the same requests stepped alone, bit for bit."""
from dataclasses import dataclass

import numpy as np
import pytest

from paper_1905_00671_amd import serving as S
from paper_1905_00671_amd import workloads as W


@dataclass
class FakeReq:
    rid: int
    arrival: float
    nbytes: int
    nsteps: int
    fail_at: int = -1


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def _fake_backend(clock, budget, log, step_cost=0.01):
    live = {}

    def bytes_of(r):
        return r.nbytes

    def open_problem(r):
        live[r.rid] = r.nbytes
        assert sum(live.values()) <= budget
        log.append(("open", r.rid, clock.t))
        return r.rid

    def step_many(handles, reqs, steps):
        clock.t += step_cost
        out = []
        for r, n in zip(reqs, steps):
            out.append(dict(status=1 if n == r.fail_at else 0, newton_iters=3, krylov_total=10))
        return out

    def close_problem(h, r):
        del live[h]
        log.append(("close", r.rid, clock.t))

    return dict(bytes_of=bytes_of, open_problem=open_problem, step_many=step_many, close_problem=close_problem,
                points_of=lambda r: 100)


def test_admission_respects_budget_and_order():
    clock = FakeClock()
    budget = 100
    reqs = [FakeReq(0, 0.00, 60, 3), FakeReq(1, 0.001, 50, 2), FakeReq(2, 0.002, 30, 1),
            FakeReq(3, 0.5, 200, 1), FakeReq(4, 0.6, 40, 2)]
    log = []
    rep = S.serve(reqs, budget, clock=clock, sleep=clock.sleep, realtime=True, **_fake_backend(clock, budget, log))
    opens = [e[1] for e in log if e[0] == "open"]
    # FIFO: request 2 (30 B) must not overtake request 1 (50 B), which waits for request 0 to leave
    assert opens == [0, 1, 2, 4]
    assert rep.rejected == 1 and rep.completed == 4 and rep.failed == 0
    assert rep.peak_bytes <= budget
    # request 1 was admitted only after request 0 closed
    t_close0 = [e[2] for e in log if e == ("close", 0, e[2])][0]
    t_open1 = [e[2] for e in log if e[0] == "open" and e[1] == 1][0]
    assert t_open1 >= t_close0
    # the idle gap before request 4 was slept through on the wall clock
    t_open4 = [e[2] for e in log if e[0] == "open" and e[1] == 4][0]
    assert t_open4 >= 0.6
    assert rep.particle_steps == 100 * (3 + 2 + 1 + 2)
    assert len(rep.step_latency_ms) == 3 + 2 + 1 + 2
    s = rep.summary()
    assert s["completed"] == 4 and s["step_latency_ms"]["p50"] > 0


def test_failure_retires_request_and_frees_budget():
    clock = FakeClock()
    reqs = [FakeReq(0, 0.0, 80, 5, fail_at=2), FakeReq(1, 0.0, 80, 1)]
    log = []
    rep = S.serve(reqs, 100, clock=clock, sleep=clock.sleep, realtime=False, **_fake_backend(clock, 100, log))
    assert rep.failed == 1 and rep.completed == 1
    assert [e[:2] for e in log] == [("open", 0), ("close", 0), ("open", 1), ("close", 1)]


def test_jsonl_step_log():
    """One JSON line per request step, failed steps included, with the runtime's statistics."""
    import io
    import json
    clock = FakeClock()
    reqs = [FakeReq(0, 0.0, 40, 3), FakeReq(1, 0.0, 40, 4, fail_at=2)]
    fh = io.StringIO()
    rep = S.serve(reqs, 100, clock=clock, sleep=clock.sleep, realtime=False, on_step=S.jsonl_step_log(fh),
                  **_fake_backend(clock, 100, []))
    lines = [json.loads(x) for x in fh.getvalue().splitlines()]
    assert len(lines) == len(rep.step_latency_ms) == 3 + 2
    assert [(x["request"], x["step"], x["status"]) for x in lines if x["request"] == 1] == [(1, 1, 0), (1, 2, 1)]
    assert [x["step"] for x in lines if x["request"] == 0] == [1, 2, 3]
    assert all(x["newton_iters"] == 3 and x["krylov_total"] == 10 and x["latency_ms"] > 0 for x in lines)


def test_zero_budget_rejects_everything():
    clock = FakeClock()
    reqs = [FakeReq(0, 0.0, 10, 2), FakeReq(1, 0.1, 20, 1)]
    log = []
    rep = S.serve(reqs, 0, clock=clock, sleep=clock.sleep, realtime=False, **_fake_backend(clock, 0, log))
    assert rep.rejected == 2 and rep.completed == 0 and log == [] and rep.peak_bytes == 0


def test_skip_idle_gaps_when_not_realtime():
    clock = FakeClock()
    reqs = [FakeReq(0, 0.0, 10, 1), FakeReq(1, 100.0, 10, 1)]
    log = []
    rep = S.serve(reqs, 100, clock=clock, sleep=clock.sleep, realtime=False, **_fake_backend(clock, 100, log))
    assert rep.completed == 2 and clock.t < 1.0


def test_trace_statistics():
    tr = W.serving_trace()
    assert len(tr) == 256
    gaps = np.diff([0.0] + [r.arrival for r in tr])
    assert 0.03 < gaps.mean() < 0.07
    ns = np.array([r.n for r in tr])
    assert ns.min() >= 16 and ns.max() <= 256 and 40 < np.median(ns) < 100
    kinds = [r.kind for r in tr]
    assert 0.35 < kinds.count("footing") / len(kinds) < 0.65


@pytest.mark.gpu
def test_served_results_equal_alone():
    from paper_1905_00671_amd import binding as B
    reqs = [W.Request(0, 0.0, "consolidation", 12, 1e-12, 3), W.Request(1, 0.0, "footing", 16, 1e-14, 2),
            W.Request(2, 0.0, "consolidation", 20, 1e-15, 2), W.Request(3, 0.01, "footing", 10, 1e-11, 3),
            W.Request(4, 0.02, "consolidation", 8, 1e-13, 2)]
    for precision in (0, 1):
        print(f"[serving] precision={precision}", flush=True)
        be = S.gpu_backend(precision)
        got = {}
        opener = be["open_problem"]

        def open_logged(r):
            print(f"  open request {r.rid} ({r.kind}, n={r.n})", flush=True)
            return opener(r)

        be["open_problem"] = open_logged

        def fin(job):
            got[job.req.rid] = (job.handle.get("u"), job.handle.get("p"), job.steps_done)

        rep = S.serve(reqs, 1 << 40, realtime=False, on_finish=fin, **be)
        assert rep.completed == len(reqs) and rep.failed == 0
        assert max(rep.batch_sizes) >= 3
        for r in reqs:
            w = r.workload()
            p = B.Problem.from_workload(w, precision=precision)
            try:
                for n in range(1, r.nsteps + 1):
                    st = p.step(w.dt, w.bc(n))
                    assert st["status"] == 0
                u, pp = p.get("u"), p.get("p")
            finally:
                p.close()
            assert got[r.rid][2] == r.nsteps
            assert np.array_equal(u, got[r.rid][0]) and np.array_equal(pp, got[r.rid][1]), r


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1])
def test_served_results_match_oracle(precision):
    """Requests served in mixed batches (consolidation on original MPM and footings on GIMP, so
    two kernel-variant groups overlap) against the CPU oracle run of each request alone: FP64
    within 1e-10, mixed within 1e-6 on u and p (Newton driven to 1e-10 on both sides)."""
    from oracle import oracle as O
    from tests.gpu_common import field_errors
    reqs = [W.Request(0, 0.0, "consolidation", 12, 1e-12, 3), W.Request(1, 0.0, "footing", 16, 1e-14, 3),
            W.Request(2, 0.0, "consolidation", 10, 1e-15, 2), W.Request(3, 0.005, "footing", 12, 1e-11, 2)]
    be = S.gpu_backend(precision, newton_rtol=1e-10, krylov_rtol=1e-12)
    got = {}

    def fin(job):
        got[job.req.rid] = {k: job.handle.get(k) for k in ("u", "p", "x", "F", "vol", "sig", "lp")}

    print(f"[serving vs oracle] precision={precision}", flush=True)
    rep = S.serve(reqs, 1 << 40, realtime=False, on_finish=fin, **be)
    assert rep.completed == len(reqs) and rep.failed == 0
    assert max(rep.batch_sizes) >= 3
    tol = 1e-10 if precision == 0 else 1e-6
    for r in reqs:
        w = r.workload()
        w.options.newton_rtol = 1e-10
        pr = O.from_workload(w)
        for n in range(1, r.nsteps + 1):
            pr.step(w.dt, w.bc(n))
        ref = dict(u=pr.u, p=pr.p, x=pr.x, F=pr.F, vol=pr.V, sig=pr.sig, lp=pr.lp)
        fe = field_errors(got[r.rid], ref, False, w.options.shape == W.GIMP)
        print(f"  request {r.rid} ({r.kind}, n={r.n}): " + " ".join(f"{k}={v:.1e}" for k, v in fe.items()),
              flush=True)
        assert fe["u"] < tol and fe["p"] < tol, (r, fe)
        assert max(fe.values()) < 10 * tol, (r, fe)
