"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

Assembly parity compares the masked residual element by element and J v for random v at a shared
random nodal state (FP64: 1e-11 of each block's scale; mixed: FP32 Jacobian, 2e-6).  Step parity
runs whole time steps on both sides and compares every material-point field element by element
after every step (gpu_common.field_errors: u and p within 1e-10 in FP64 and 1e-6 mixed, the
fields formed from them within ten times that; pressure errors are measured against
max(|p|, |sigma'|) so that drained steps with p -> 0 stay meaningful).  Further: batched stepping
equals stepping alone bit for bit, repeated runs are bit-identical, a checkpoint resumes bit for
bit, and invalid inputs are refused with their status codes."""
import zlib

import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_00671_amd import workloads as W
from tests.gpu_common import (block_err, dyn_oracle_nodal, field_errors, free_mask, gpu_state, oracle_jv,
                              oracle_masked_residual, oracle_state, rel_l2)

pytestmark = pytest.mark.gpu


def _binding():
    from paper_1905_00671_amd import binding as B
    return B


def _kc(w):
    """The workload with Kozeny-Carman permeability (eq. kozeny-carman) from its porosity."""
    w.material.kozeny_carman = True
    return w


def _seed(name):
    """Stable per-case seed (Python's str hash is salted per process)."""
    return zlib.crc32(name.encode()) % 1000


def _assembly_case(name):
    rng = np.random.default_rng(_seed(name))
    if name == "box_linear_qs":
        w = W.jittered_box(8, 8, shape=W.LINEAR, seed=1)
    elif name == "box_gimp_qs":
        w = W.jittered_box(8, 8, shape=W.GIMP, seed=2)
    elif name == "box_gimp_dyn":
        w = W.jittered_box(8, 8, shape=W.GIMP, dynamic=1, seed=3)
        w.particles.v0 = 0.05 * (rng.random((w.particles.n, 2)) - 0.5)
    elif name == "box_linear_dyn_hencky":
        w = W.jittered_box(8, 8, shape=W.LINEAR, dynamic=1, model=W.HENCKY, seed=4)
        w.particles.v0 = 0.05 * (rng.random((w.particles.n, 2)) - 0.5)
    elif name == "terzaghi":
        w = W.config(1)
    elif name == "footing_gimp":
        w = W.config(3, nx=32, ny=16, width=2.0, empty_rows=3, nsteps=2)
    elif name == "footing3d":
        w = W.footing3d(n=5, size=1.25, half_b=0.25, nsteps=2)
    elif name == "footing_gimp_kc":
        w = _kc(W.config(3, nx=32, ny=16, width=2.0, empty_rows=3, nsteps=2))
    elif name == "footing3d_kc":
        w = _kc(W.footing3d(n=5, size=1.25, half_b=0.25, nsteps=2))
    elif name == "box_gimp_dyn_damped":
        w = W.jittered_box(8, 8, shape=W.GIMP, dynamic=1, seed=5)
        w.material.alpha_vis = 0.04
        w.particles.v0 = 0.05 * (rng.random((w.particles.n, 2)) - 0.5)
    elif name == "box_linear_dyn_hencky_damped":
        w = W.jittered_box(8, 8, shape=W.LINEAR, dynamic=1, model=W.HENCKY, seed=6)
        w.material.alpha_vis = 0.04
        w.particles.v0 = 0.05 * (rng.random((w.particles.n, 2)) - 0.5)
    elif name == "footing3d_dyn_damped":
        w = W.footing3d(n=4, size=1.0, half_b=0.25, nsteps=2)
        w.options.dynamic = 1
        w.material.alpha_vis = 0.04
        w.particles.v0 = 0.05 * (rng.random((w.particles.n, 3)) - 0.5)
    elif name == "footing3d_dyn":
        w = W.footing3d(n=4, size=1.0, half_b=0.25, nsteps=2)
        w.options.dynamic = 1
        w.particles.v0 = 0.05 * (rng.random((w.particles.n, 3)) - 0.5)
    else:
        raise ValueError(name)
    w.particles.p0 = 1e4 * rng.random(w.particles.n)
    return w, rng


ASSEMBLY_CASES = ["box_linear_qs", "box_gimp_qs", "box_gimp_dyn", "box_linear_dyn_hencky", "terzaghi",
                  "footing_gimp", "footing3d", "footing3d_dyn", "footing_gimp_kc", "footing3d_kc",
                  "box_gimp_dyn_damped", "box_linear_dyn_hencky_damped", "footing3d_dyn_damped"]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ASSEMBLY_CASES)
def test_assembly_parity(name, precision):
    B = _binding()
    w, rng = _assembly_case(name)
    print(f"[assembly] case={name} precision={precision} np={w.particles.n} seed={_seed(name)}", flush=True)
    g, d = w.grid, w.grid.dim
    pr = O.from_workload(w)
    bc = w.bc(1)
    nodal = dyn_oracle_nodal(pr, bc)
    act = nodal["active"]
    U = 2e-3 * w.grid.h * (rng.random((g.nnode, d)) - 0.5) * act[:, None]
    P = (nodal["Pn"] + 3e3 * (rng.random(g.nnode) - 0.5)) * act
    R_or, J, free = oracle_masked_residual(pr, nodal, U, P, bc, w.dt)
    gp = B.Problem.from_workload(w, precision=precision)
    try:
        R_gpu = gp.eval_residual(w.dt, bc, U, P)
        # P2G and the dof masks agree exactly (same decisions) and to rounding (values)
        assert np.array_equal(gp.get_nodal(2).astype(bool), free)
        M_gpu = gp.get_nodal(0)
        assert np.abs(M_gpu - nodal["M"]).max() <= 1e-13 * nodal["M"].max()
        eu, ep = block_err(R_gpu, R_or, d)
        assert eu < 1e-11 and ep < 1e-11, (eu, ep)
        tol = 1e-11 if precision == 0 else 2e-6
        for trial in range(3):
            v = rng.random(g.nnode * (d + 1)) - 0.5
            v.reshape(-1, d + 1)[:, d] *= 1e6      # pressure increments are O(1e6) x displacement ones
            y_or = oracle_jv(J, free, v)
            y_gpu = gp.apply_jacobian(v)
            eu, ep = block_err(y_gpu, y_or, d)
            assert eu < tol and ep < tol, (trial, eu, ep)
    finally:
        gp.close()


def _run_steps(w, nsteps, precision, **over):
    """Steps the oracle and the HIP path side by side; after every step, the element-wise error of
    every material-point field (gpu_common.field_errors) and the Newton / Krylov counts."""
    B = _binding()
    pr = O.from_workload(w)
    gp = B.Problem.from_workload(w, precision=precision, **over)
    dyn, gimp = bool(w.options.dynamic), w.options.shape == W.GIMP
    dt_of = w.meta.get("dt_of", lambda n: w.dt)
    errs = []
    try:
        for n in range(1, nsteps + 1):
            bc = w.bc(n)
            st_o = pr.step(dt_of(n), bc)
            st_g = gp.step(dt_of(n), bc)
            fe = field_errors(gpu_state(gp), oracle_state(pr), dyn, gimp, w.material.E, dt_of(n))
            errs.append(dict(step=n, f=fe, newton=(st_o["newton_iters"], st_g["newton_iters"]),
                             krylov=st_g["krylov_total"]))
            print(f"  step {n}: " + " ".join(f"{k}={v:.1e}" for k, v in fe.items()) +
                  f" newton oracle/gpu={st_o['newton_iters']}/{st_g['newton_iters']} krylov={st_g['krylov_total']}",
                  flush=True)
    finally:
        gp.close()
    return errs


def _assert_fields(errs, tol, tol_other=None):
    """u and p within tol (the parity bar), every other field within tol_other (default 10 tol:
    they are formed from u, p through the basis, the constitutive law and the Newmark formulas)."""
    tol_other = 10 * tol if tol_other is None else tol_other
    for e in errs:
        f = e["f"]
        assert f["u"] < tol and f["p"] < tol, e
        for k, v in f.items():
            if k not in ("u", "p"):
                lim = tol_other.get(k, 10 * tol) if isinstance(tol_other, dict) else tol_other
                assert v < lim, (k, e)


STEP_CASES = {
    "terzaghi": (lambda: W.config(1), 10),
    "footing2d_dyn_gimp": (lambda: W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=4), 4),
    "footing2d_qs_gimp": (lambda: W.config(3, nx=32, ny=16, width=2.0, empty_rows=2, nsteps=4), 4),
    "consolidation_linear": (lambda: W.consolidation2d(16, 1e-13, nsteps=3), 3),
    "footing3d": (lambda: W.footing3d(n=6, size=1.5, half_b=0.25, nsteps=2), 2),
    "footing2d_qs_gimp_kc": (lambda: _kc(W.config(3, nx=32, ny=16, width=2.0, empty_rows=2, nsteps=4)), 4),
    # large enough for per-level multigrid kernels on two 3D levels below the fine grid
    "footing3d_mg": (lambda: W.footing3d(n=12, size=1.5, half_b=0.25, nsteps=2), 2),
    # gravity: body force m S g in eq. residual-momentum, rho_f g in eq. darcy-law
    "terzaghi_gravity": (lambda: _gravity(W.config(1, nsteps=3)), 3),
    "footing2d_dyn_gravity": (lambda: _gravity(W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=4)), 4),
    "footing3d_dyn_gravity": (lambda: _gravity(_dyn(W.footing3d(n=6, size=1.5, half_b=0.25, nsteps=2, delta=1e-4))), 2),
    # stabilization parameters of Sec. 4.3 other than tau_W
    "consolidation_tau_sun": (lambda: _tau(W.consolidation2d(16, 1e-15, nsteps=3), W.TAU_SUN), 3),
    "footing2d_dyn_tau_monforte": (lambda: W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=4,
                                                    tau_kind=W.TAU_MONFORTE), 4),
    # Kelvin-type viscous damping (Sec. 2.2) with the paper's alpha_vis = 0.04 s
    "footing2d_dyn_damped": (lambda: _damped(W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=4)), 4),
    "footing3d_dyn_damped": (lambda: _damped(_dyn(W.footing3d(n=6, size=1.5, half_b=0.25, nsteps=2, delta=1e-4))), 2),
    # the paper's Newmark parameters (Sec. 3.2)
    "footing2d_dyn_paper_newmark": (lambda: W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=4,
                                                     beta=0.3025, gamma=0.6), 4),
    # consolidation under self weight (Sec. 5.3) at the paper's coarser resolution: Hencky,
    # Kozeny-Carman, gravity, drained free surface following the settling top, dt growing 1.2x
    "self_weight_gimp": (lambda: W.self_weight(), 40),
    "self_weight_linear_closed": (lambda: W.self_weight(h=0.25, ppa=2, shape=W.LINEAR, right_drained=False), 40),
    # Sec. 5.2 harmonic strip footing: consistent-mass mapping, tractions on the top faces of the
    # points under the footing, Hencky, Kelvin damping, Newmark 0.3025 / 0.6
    "harmonic_footing": (lambda: W.harmonic_footing(), 10),
    # consistent-mass mapping on its own: quasi-static GIMP, 3D dynamic, original MPM dynamic
    "consistent_qs_gimp": (lambda: _cons(W.config(3, nx=32, ny=16, width=2.0, empty_rows=2, nsteps=4)), 4),
    "consistent_dyn_3d": (lambda: _cons(_dyn(W.footing3d(n=6, size=1.5, half_b=0.25, nsteps=3, delta=1e-4))), 3),
    "consistent_dyn_linear": (lambda: _cons(W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=4,
                                                     shape=W.LINEAR)), 4),
    # point tractions on their own: the Terzaghi column loaded through its top points' faces
    "terzaghi_point_load": (lambda: _point_load_terzaghi(), 6),
    # Sec. 5.4 two-body impact: coarse discs started close, 300 steps into the contact; and the
    # paper's size (40,216 points) for its first steps; point pressure conditions, no grid BCs
    "impact_coarse_contact": (lambda: W.two_body_impact(h=0.05, ppa=2, centre=0.3, nsteps=300), 300),
    "impact_paper_prefix": (lambda: W.two_body_impact(nsteps=3), 3),
    # the two Schur-block forms of the preconditioner (Sec. 3.4) where the workloads do not pick
    # them: the fixed-stress form on an undrained dynamic footing, and the diagonal-inverse form
    # in 3D, where the product C - B2 diag(A)^-1 B1 is truncated to the trilinear stencil
    "footing2d_dyn_fixed_stress": (lambda: _schur(W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=4), 0), 4),
    "footing3d_dyn_schur_diag": (lambda: _schur(_dyn(W.footing3d(n=6, size=1.5, half_b=0.25, nsteps=2, delta=1e-4)), 1), 2),
}


# The Newmark rates are differences of the step's solution divided by beta dt^2 (pddot) or
# beta dt (pdot): at dt = 1 ms and a load of 100 rad/s, pddot ~ omega^2 p, so a relative p
# difference reaches pddot amplified by p / (beta dt^2 pddot) ~ 1 / (beta (omega dt)^2) ~ 330.
STEP_TOL_OTHER = {"harmonic_footing": {"pdd": 5e-8, "pd": 5e-9}}
CONDITION_LIMITED = ("impact_coarse_contact", "impact_paper_prefix")


def _cons(w):
    w.options.consistent_mass = 1
    return w


def _schur(w, form):
    w.options.schur = form
    return w


def _point_load_terzaghi():
    w = W.config(1)
    H, q = w.meta["H"], w.meta["load"]
    top = w.particles.x[:, 1] > H - w.grid.h / 2
    F = np.zeros_like(w.particles.x)
    F[top, 1] = -q * 2.0 * w.particles.lp[top, 0]
    N = np.zeros_like(w.particles.x)
    N[top, 1] = 1.0
    nodal = w.bc

    def bc(n):
        b = nodal(n)
        b["f_ext"][:] = 0.0
        b["point_force"], b["point_normal"] = F, N
        return b

    w.bc = bc
    return w


def _gravity(w):
    w.material.g = (0.0, -9.81, 0.0) if w.grid.dim == 2 else (0.0, 0.0, -9.81)
    return w


def _damped(w):
    w.material.alpha_vis = 0.04
    return w


def _dyn(w):
    w.options.dynamic = 1
    w.dt = 1e-3
    return w


def _tau(w, kind):
    w.options.tau_kind = kind
    return w


@pytest.mark.parametrize("name", list(STEP_CASES))
def test_step_parity_fp64(name):
    make, nsteps = STEP_CASES[name]
    w = make()
    w.options.newton_rtol = 1e-10
    w.options.krylov_rtol = 1e-12
    print(f"[steps fp64] case={name} np={w.particles.n}", flush=True)
    errs = _run_steps(w, nsteps, 0)
    if name in CONDITION_LIMITED:
        # free-flying undrained bodies: the pore pressure is fixed only through the near-singular
        # mass block, so the Newton test (per-block floors) accepts pressures that differ between
        # the direct and the iterative solve; displacements and positions are compared
        for e in errs:
            assert e["f"]["u"] < 1e-6 and e["f"]["x"] < 1e-6, e
        return
    _assert_fields(errs, 1e-10, STEP_TOL_OTHER.get(name))
    if name in ("footing3d_mg", "footing2d_qs_gimp", "consolidation_linear"):
        # the block preconditioner keeps BiCGStab short on these quasi-static problems (Krylov
        # 1e-12 here, so about 1.5x the iterations of the default 1e-8)
        for e in errs:
            assert e["krylov"] <= 60 * e["newton"][1], errs


@pytest.mark.parametrize("name", ["terzaghi", "footing2d_qs_gimp", "footing3d", "footing2d_qs_gimp_kc",
                                  "footing2d_dyn_gimp", "footing2d_dyn_paper_newmark", "footing2d_dyn_damped",
                                  "self_weight_gimp", "harmonic_footing", "consistent_dyn_3d",
                                  "footing3d_dyn_schur_diag"])
def test_step_parity_mixed(name):
    make, nsteps = STEP_CASES[name]
    w = make()
    w.options.newton_rtol = 1e-8
    print(f"[steps mixed] case={name} np={w.particles.n}", flush=True)
    errs = _run_steps(w, nsteps, 1)
    _assert_fields(errs, 1e-6)


def test_step_parity_default_tolerances():
    """At the paper's tolerances (Newton 1e-8 per residual block, Krylov 1e-8 |R|) both sides stop
    wherever their own iterates first pass the Newton test, so the states agree to the Newton
    tolerance (the 1e-10 bar is checked with Newton driven to 1e-10, above)."""
    w = W.config(3, nx=32, ny=16, width=2.0, empty_rows=2, nsteps=3)
    print("[steps default tol]", flush=True)
    errs = _run_steps(w, 3, 0)
    _assert_fields(errs, 1e-8)


def test_batched_equals_alone():
    """Problems stepped together (one launch per phase) give bit-identical results to the same
    problems stepped alone."""
    B = _binding()
    ws = [W.consolidation2d(12, 1e-12, nsteps=2), W.consolidation2d(20, 1e-14, nsteps=2),
          W.config(3, nx=16, ny=8, width=4.0, empty_rows=2, nsteps=2)]
    alone = []
    for w in ws:
        p = B.Problem.from_workload(w)
        for n in (1, 2):
            p.step(w.dt, w.bc(n))
        alone.append((p.get("u"), p.get("p")))
        p.close()
    ps = [B.Problem.from_workload(w) for w in ws]
    try:
        for n in (1, 2):
            st = B.step_batched(ps, [w.dt for w in ws], [w.bc(n) for w in ws])
            assert all(s["status"] == 0 for s in st), st
        for (u0, p0), p in zip(alone, ps):
            assert np.array_equal(p.get("u"), u0)
            assert np.array_equal(p.get("p"), p0)
    finally:
        for p in ps:
            p.close()


def test_batched_schur_forms_equal_alone():
    """A batch that mixes the two Schur-block forms (an undrained dynamic footing with each, and a
    quasi-static footing with its truncated fixed-stress hierarchy) gives bit-identical results
    to the problems stepped alone: the level-0 Schur operator is formed only for the problems
    that ask for it, and each problem's hierarchy keeps its own depth."""
    B = _binding()

    def make():
        a = W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=3)
        b = _schur(W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=3), 0)
        c = W.config(3, nx=16, ny=8, width=4.0, empty_rows=2, nsteps=3)
        return [a, b, c]

    ws = make()
    assert [w.options.schur for w in ws] == [1, 0, 0]
    alone = []
    for w in ws:
        p = B.Problem.from_workload(w)
        for n in (1, 2, 3):
            p.step(w.dt, w.bc(n))
        alone.append((p.get("u"), p.get("p")))
        p.close()
    ps = [B.Problem.from_workload(w) for w in ws]
    try:
        for n in (1, 2, 3):
            st = B.step_batched(ps, [w.dt for w in ws], [w.bc(n) for w in ws])
            assert all(s["status"] == 0 for s in st), st
        for (u0, p0), p in zip(alone, ps):
            assert np.array_equal(p.get("u"), u0)
            assert np.array_equal(p.get("p"), p0)
    finally:
        for p in ps:
            p.close()


@pytest.mark.parametrize("name", ["footing2d_dyn_gimp", "harmonic_footing", "footing3d_mg", "self_weight_gimp"])
def test_checkpoint_resume_bitwise(name):
    """A problem restored from a checkpoint (ppmpm_save_state / ppmpm_load_state) into a fresh
    problem steps on bit for bit like the problem it was saved from: the committed material
    points are the whole state between steps (dynamic: with their Newmark history; consistent
    mass; the 3D multigrid; the self-weight column's growing steps and drained surface)."""
    B = _binding()
    make, _ = STEP_CASES[name]
    w = make()
    dt = w.meta.get("dt_of", lambda n: w.dt)
    fields = ("x", "u", "p", "F", "vol", "sig", "v", "a", "pd", "pdd", "lp")
    a = B.Problem.from_workload(w)
    b = B.Problem.from_workload(w)
    try:
        a.step(dt(1), w.bc(1))
        ck = a.save_state()
        for n in (2, 3):
            a.step(dt(n), w.bc(n))
        ref = {k: a.get(k).copy() for k in fields}
        print(f"[checkpoint] case={name} np={w.particles.n} bytes={ck.nbytes}", flush=True)
        b.load_state(ck)
        for n in (2, 3):
            b.step(dt(n), w.bc(n))
        for k in fields:
            assert np.array_equal(b.get(k), ref[k]), k
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["footing2d_qs_gimp", "footing3d_mg", "harmonic_footing", "terzaghi_point_load"])
def test_repeat_runs_bitwise_identical(name, precision):
    """Five fresh runs of the same steps leave bit-identical states: the hot path has no
    floating-point atomics (reductions run in a fixed order, the largest nodal mass is an integer
    maximum, point tractions are gathered per node in the sort's order), so results do not depend
    on how the GPU schedules the work."""
    B = _binding()
    make, _ = STEP_CASES[name]
    ref = None
    for rep in range(5):
        w = make()
        p = B.Problem.from_workload(w, precision=precision)
        try:
            for n in (1, 2, 3):
                p.step(w.dt, w.bc(n))
            got = {k: p.get(k) for k in ("x", "u", "p", "sig", "v", "pd")}
        finally:
            p.close()
        if ref is None:
            ref = got
            print(f"[repeat] case={name} precision={precision} np={w.particles.n}", flush=True)
        else:
            for k in got:
                assert np.array_equal(got[k], ref[k]), (rep, k)


def test_point_outside_grid_refused():
    """A material point placed outside the background grid (or a GIMP half-length above h/2) is
    refused at set-up with PPMPM_E_OUT_OF_GRID; the set-up kernel only flags it."""
    B = _binding()
    for bad in ("x", "lp"):
        w = W.config(3, nx=16, ny=8, width=4.0, empty_rows=2, nsteps=1)
        if bad == "x":
            w.particles.x[5, 1] = w.grid.h * (w.grid.ncell[1] + 3)
        else:
            w.particles.lp[5, 0] = 0.75 * w.grid.h
        with pytest.raises(B.PPMPMError) as e:
            B.Problem.from_workload(w).close()
        assert e.value.status == B.E_OUT_OF_GRID, (bad, e.value.status)


def test_checkpoint_mismatch_refused():
    """A checkpoint of another problem (other point count and grid), a truncated one and one with
    a damaged header are refused with PPMPM_E_INVALID, and the problem keeps its points."""
    B = _binding()
    w1 = W.config(2, nx=16, ny=16, width=2.5, empty_rows=2, nsteps=2)
    w2 = W.config(2, nx=12, ny=12, width=2.5, empty_rows=2, nsteps=2)
    a = B.Problem.from_workload(w1)
    b = B.Problem.from_workload(w2)
    try:
        ck = a.save_state()
        x0 = b.get("x").copy()
        bad = ck.copy()
        bad[:8] = np.frombuffer(b"NOTASTAT", np.uint8)
        own = b.save_state()
        for buf in (ck, own[: own.nbytes - 8], bad[: own.nbytes]):
            with pytest.raises(B.PPMPMError) as e:
                b.load_state(buf)
            assert e.value.status == B.E_INVALID
        assert np.array_equal(b.get("x"), x0)
    finally:
        a.close()
        b.close()


def test_transactional_failure_leaves_state():
    """A step that cannot converge (one Newton iteration allowed on a loaded step that needs two)
    reports PPMPM_E_NEWTON and leaves the material points untouched."""
    B = _binding()
    w = W.config(1)
    p = B.Problem.from_workload(w, newton_max=1)
    try:
        x0 = p.get("x").copy()
        st = p.step(w.dt, w.bc(1), raise_on_error=False)
        assert st["status"] == B.E_NEWTON
        assert np.array_equal(p.get("x"), x0)
    finally:
        p.close()


def test_failure_parity_overconstrained():
    """A rigid footing as wide as an undrained, laterally confined box forces a volume change the
    incompressible mixture cannot take: the oracle inverts a material point, and the HIP path
    reports PPMPM_E_NONFINITE (or E_NEWTON) and leaves the state unchanged."""
    B = _binding()
    w = W.config(3, nx=16, ny=8, width=1.0, empty_rows=2, nsteps=2)
    pr = O.from_workload(w)
    with pytest.raises(O.NewtonFailure):
        for n in (1, 2):
            pr.step(w.dt, w.bc(n))
    p = B.Problem.from_workload(w)
    try:
        x0 = p.get("x").copy()
        status = 0
        for n in (1, 2):
            st = p.step(w.dt, w.bc(n), raise_on_error=False)
            status = st["status"]
            if status:
                break
            x0 = p.get("x").copy()
        assert status in (B.E_NONFINITE, B.E_NEWTON)
        assert np.array_equal(p.get("x"), x0)
    finally:
        p.close()


def test_batch_larger_than_one_launch():
    """More problems than one batched launch holds (64): the library splits the batch, and every
    problem still matches its alone run bit for bit."""
    B = _binding()
    ks = [10.0 ** (-16 + 6 * i / 69) for i in range(70)]
    ws = [W.consolidation2d(4 + (i % 3), ks[i], nsteps=1) for i in range(70)]
    ps = [B.Problem.from_workload(w) for w in ws]
    try:
        st = B.step_batched(ps, [w.dt for w in ws], [w.bc(1) for w in ws])
        assert all(s["status"] == 0 for s in st), [s["status"] for s in st]
        got = [(p.get("u"), p.get("p")) for p in ps]
    finally:
        for p in ps:
            p.close()
    for i in (0, 33, 63, 64, 69):
        w = ws[i]
        p = B.Problem.from_workload(w)
        try:
            p.step(w.dt, w.bc(1))
            assert np.array_equal(p.get("u"), got[i][0]) and np.array_equal(p.get("p"), got[i][1]), i
        finally:
            p.close()


@pytest.mark.parametrize("case", ["undrained_k0", "no_stabilization", "one_point_per_cell"])
def test_degenerate_cases_parity(case):
    """Limits of the method: zero permeability (the pressure block is the stabilization term
    alone), no PPP term (tau = 0, well-posed here because the column drains), and one point per
    cell (the original-MPM projection equals the point value, so the PPP term vanishes)."""
    if case == "undrained_k0":
        w = W.terzaghi(k=0.0, nsteps=3)
    elif case == "no_stabilization":
        w = W.terzaghi(tau_kind=W.TAU_OFF, nsteps=3)
    else:
        w = W.consolidation2d(8, 1e-12, nsteps=2)
        g = w.grid
        xs = (np.arange(8) + 0.37) * g.h
        X, Y = np.meshgrid(xs, xs, indexing="xy")
        w.particles.x = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
        w.particles.vol = np.full(64, g.h * g.h)
        w.particles.mass = w.material.rho0 * w.particles.vol
        w.particles.lp = np.full((64, 2), 0.25 * g.h)
    w.options.newton_rtol = 1e-10
    w.options.krylov_rtol = 1e-12
    print(f"[degenerate] {case}", flush=True)
    errs = _run_steps(w, w.nsteps, 0)
    _assert_fields(errs, 1e-10)


def test_step_parity_two_smoothing_sweeps():
    """V(2,2) cycles (the per-operation multigrid kernels) reach the same states as the oracle."""
    make, nsteps = STEP_CASES["footing2d_qs_gimp"]
    w = make()
    w.options.newton_rtol = 1e-10
    w.options.krylov_rtol = 1e-12
    print("[steps fp64, mg_smooth=2]", flush=True)
    errs = _run_steps(w, nsteps, 0, mg_smooth=2)
    _assert_fields(errs, 1e-10)


def test_kozeny_carman_changes_the_solution_and_rejects_bad_porosity():
    """The porosity law is live on the device (the states differ from constant permeability once
    the footing compacts the soil) and an initial porosity outside [0, 1) is refused."""
    B = _binding()
    make, nsteps = STEP_CASES["footing2d_qs_gimp"]
    out = []
    for kc in (False, True):
        w = make()
        w.material.kozeny_carman = kc
        gp = B.Problem.from_workload(w, precision=0)
        try:
            for n in range(1, 3):
                gp.step(w.dt, w.bc(n))
            out.append(gp.get("p"))
        finally:
            gp.close()
    assert rel_l2(out[1], out[0]) > 1e-6
    w = make()
    w.material.kozeny_carman = True
    w.material.phi0 = 1.2
    with pytest.raises(B.PPMPMError):
        B.Problem.from_workload(w, precision=0)


def test_batched_invalid_problem_reports_invalid():
    """A problem with dt = 0 in a batch is refused on the host (PPMPM_E_INVALID in its statistics)
    and not stepped; the other problems are stepped and equal their alone runs bit for bit."""
    B = _binding()
    ws = [W.consolidation2d(12, 1e-12, nsteps=1), W.consolidation2d(10, 1e-13, nsteps=1),
          W.config(3, nx=16, ny=8, width=4.0, empty_rows=2, nsteps=1)]
    alone = []
    for w in ws:
        p = B.Problem.from_workload(w)
        p.step(w.dt, w.bc(1))
        alone.append((p.get("u"), p.get("p")))
        p.close()
    ps = [B.Problem.from_workload(w) for w in ws]
    try:
        x1 = ps[1].get("x").copy()
        st = B.step_batched(ps, [ws[0].dt, 0.0, ws[2].dt], [w.bc(1) for w in ws])
        assert [s["status"] for s in st] == [0, B.E_INVALID, 0], [s["status"] for s in st]
        assert np.array_equal(ps[1].get("x"), x1)
        for i in (0, 2):
            assert np.array_equal(ps[i].get("u"), alone[i][0]) and np.array_equal(ps[i].get("p"), alone[i][1])
    finally:
        for p in ps:
            p.close()


def test_batched_per_problem_krylov_options():
    """Problems with different Krylov tolerances in one batch each solve with their own options:
    the results equal their alone runs bit for bit."""
    B = _binding()
    ws = [W.consolidation2d(12, 1e-12, nsteps=2), W.consolidation2d(12, 1e-12, nsteps=2)]
    ws[1].options.krylov_rtol = 1e-11
    alone = []
    for w in ws:
        p = B.Problem.from_workload(w)
        for n in (1, 2):
            p.step(w.dt, w.bc(n))
        alone.append((p.get("u"), p.get("p")))
        p.close()
    assert not np.array_equal(alone[0][1], alone[1][1])
    ps = [B.Problem.from_workload(w) for w in ws]
    try:
        for n in (1, 2):
            st = B.step_batched(ps, [w.dt for w in ws], [w.bc(n) for w in ws])
            assert all(s["status"] == 0 for s in st), st
        for (u0, p0), p in zip(alone, ps):
            assert np.array_equal(p.get("u"), u0) and np.array_equal(p.get("p"), p0)
    finally:
        for p in ps:
            p.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_krylov_graph_replay_equals_direct_launches(precision):
    """The Krylov iterations are replayed from captured HIP graphs unless kernel timing is on (the
    timing records events around launches).  Stepping the same problems both ways gives the same
    bits: a 2D GIMP footing (every chunk replayed many times per step, with the assembly and the
    Newton update launched directly in between) and a 3D footing with multigrid levels."""
    B = _binding()
    cases = (lambda: W.config(3, nx=32, ny=16, width=2.0, empty_rows=2, nsteps=3),
             lambda: W.footing3d(n=12, size=1.5, half_b=0.25, nsteps=2))
    for make in cases:
        outs, krylov = [], []
        for timing in (False, True):
            w = make()
            B.timing_enable(timing)
            try:
                gp = B.Problem.from_workload(w, precision=precision)
                ks = []
                for n in range(1, w.nsteps + 1):
                    ks.append(gp.step(w.dt, w.bc(n))["krylov_total"])
                outs.append({k: gp.get(k) for k in ("u", "p", "F", "sig")})
                krylov.append(ks)
                gp.close()
            finally:
                B.timing_enable(False)
        print(f"[graph vs direct] np={w.particles.n} krylov {krylov}", flush=True)
        assert krylov[0] == krylov[1]
        for k in outs[0]:
            assert np.array_equal(outs[0][k], outs[1][k]), k


@pytest.mark.parametrize("precision", [0, 1])
def test_truncated_krylov_solves_still_converge(precision):
    """Krylov solves cut off far above their tolerance (6 iterations): each hands the better of its
    last and its best iterate to the Newton update, which keeps it only if the residual drops, so
    Newton still converges (linearly) to the oracle's state at the parity bar."""
    make, nsteps = STEP_CASES["footing2d_qs_gimp"]
    w = make()
    w.options.newton_rtol = 1e-10 if precision == 0 else 1e-8
    w.options.krylov_max = 6
    w.options.krylov_check = 2
    w.options.newton_max = 60
    print(f"[truncated krylov] precision={precision}", flush=True)
    errs = _run_steps(w, 2, precision)
    _assert_fields(errs, 1e-10 if precision == 0 else 1e-6)
    for e in errs:
        assert e["krylov"] <= 6 * e["newton"][1], e
        assert e["newton"][1] > e["newton"][0], e      # the truncated solves cost Newton iterations


def test_multigrid_large_coarse_levels_3d():
    """3D footing at 32^3 cells: the first coarse level has 17 x 17 x 18 = 5,202 rows, above the
    size from which the Galerkin operators are built as three one-axis products (each pass keeping
    the 27-point stencil).  The right-preconditioned Krylov solution does not depend on the
    preconditioner, so a wrong coarse operator shows as Krylov counts, not in the state: the counts
    stay at those of the single-pass product (16-19 per Newton iteration at Krylov 1e-8), and the
    FP64 and mixed paths agree at the mixed bar."""
    B = _binding()
    res = {}
    for prec in (0, 1):
        w = W.footing3d(n=32, size=4.0, half_b=0.5, nsteps=2)
        print(f"[multigrid 32^3] precision={prec} np={w.particles.n}", flush=True)
        gp = B.Problem.from_workload(w, precision=prec)
        try:
            for n in (1, 2):
                st = gp.step(w.dt, w.bc(n))
                print(f"  step {n}: levels={st['ngrid_levels']} newton={st['newton_iters']} krylov={st['krylov_iters']}",
                      flush=True)
                assert st["ngrid_levels"] == 5 and st["newton_iters"] == 3, st
                if prec == 0:
                    assert max(st["krylov_iters"]) <= 21, st
            res[prec] = (gp.get("u"), gp.get("p"))
        finally:
            gp.close()
    assert rel_l2(res[1][0], res[0][0]) < 1e-6 and rel_l2(res[1][1], res[0][1]) < 1e-6
