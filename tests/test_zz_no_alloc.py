"""The allocation-free entry point (ppmpm_eval_residual_static, workspace in a device array of
the library) against the entry points it stands for (ppmpm_create with a caller workspace,
ppmpm_set_particles, ppmpm_eval_residual): two calls in a row, the second on a smaller problem,
each compared with the caller-workspace path on the same inputs."""
import numpy as np
import pytest

from paper_1905_00671_amd import workloads as W

pytestmark = pytest.mark.gpu


def _state(w, seed):
    from oracle import oracle as O
    rng = np.random.default_rng(seed)
    pr = O.from_workload(w)
    nodal = pr.p2g()
    act = nodal["active"]
    g, d = w.grid, w.grid.dim
    U = 2e-3 * g.h * (rng.random((g.nnode, d)) - 0.5) * act[:, None]
    P = (nodal["Pn"] + 3e3 * (rng.random(g.nnode) - 0.5)) * act
    return U, P


def test_static_workspace_matches_caller_workspace():
    from paper_1905_00671_amd import binding as B
    cases = [W.config(3, nx=48, ny=24, width=3.0, empty_rows=3, nsteps=1),     # 2D GIMP, larger
             W.consolidation2d(10, 1e-12, nsteps=1)]                          # 2D linear, smaller
    for n, w in enumerate(cases):
        w.particles.p0 = 1e4 * np.random.default_rng(n).random(w.particles.n)
        bc = w.bc(1)
        U, P = _state(w, 10 + n)
        print(f"[static workspace] call {n + 1}: {w.name}, {w.particles.n} points", flush=True)
        R_static = B.eval_residual_static(w, w.dt, bc, U, P)
        p = B.Problem.from_workload(w)
        try:
            R_ref = p.eval_residual(w.dt, bc, U, P)
        finally:
            p.close()
        assert np.abs(R_ref).max() > 0
        assert np.array_equal(R_static, R_ref), np.abs(R_static - R_ref).max()


def test_static_workspace_rejects_large_problems():
    from paper_1905_00671_amd import binding as B
    w = W.config(3)
    bc = w.bc(1)
    nn = w.grid.nnode
    with pytest.raises(B.PPMPMError) as e:
        B.eval_residual_static(w, w.dt, bc, np.zeros((nn, 2)), np.zeros(nn))
    assert e.value.status == B.E_OOM
