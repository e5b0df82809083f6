"""Physics pins of the oracle's full time step: the Terzaghi closed form (eq. terzaghi-exact),
patch test, rigid translation, conservation of mass, the discrete undrained volume constraint,
properties of the PPP term (Sec. 4.2) and the stabilization effect the paper reports (Sec. 5.1)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_00671_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def terzaghi_exact(Z, T, nterm=20000):
    """P(Z, T) = sum_m 2/M sin(M Z) exp(-M^2 T), M = pi (2m+1)/2 (eq. terzaghi-exact)."""
    m = np.arange(nterm)
    M = np.pi * (2 * m + 1) / 2
    return np.sum(2 / M[None, :] * np.sin(M[None, :] * Z[:, None]) * np.exp(-M[None, :] ** 2 * T), axis=1)


def test_terzaghi_series_limits():
    """The series itself: P(0, T) = 0 (drained top), P -> 1 for T -> 0 below the top."""
    assert abs(terzaghi_exact(np.array([0.0]), 0.01)[0]) < 1e-12
    assert terzaghi_exact(np.array([0.5]), 1e-6)[0] == pytest.approx(1.0, abs=1e-6)


def _reference_depth(pr, H):
    return H - (pr.x[:, 1] - pr.u[:, 1])


def test_terzaghi_config1_matches_closed_form():
    """Terzaghi column of 4 x 40 cells (h = 0.25 m, 640 points), E = 10 MPa, nu = 0.3, k = 1e-10,
    10 kPa, dt = 0.1 s: the pore pressure follows the closed form within 3 % RMS of w at every
    step (first-order implicit Euler and h = 0.25 m discretization error)."""
    w = W.terzaghi()
    pr = O.from_workload(w)
    lam, G = O.lame(w.material.E, w.material.nu)
    cv = (lam + 2 * G) * w.material.k / w.material.mu_f
    H = w.meta["H"]
    errs = []
    for n in range(1, w.nsteps + 1):
        st = pr.step(w.dt, w.bc(n))
        assert st["newton_iters"] <= 3
        Z = _reference_depth(pr, H) / H
        T = cv * n * w.dt / H ** 2
        errs.append(np.sqrt(np.mean((pr.p / w.meta["load"] - terzaghi_exact(Z, T)) ** 2)))
    assert max(errs) < 0.03
    assert errs[-1] < 0.006            # the error decays as the profile spreads over more cells
    # settlement of the top after T = 0.0135: (w H / M) * U(T), U(T) = 2 sqrt(T/pi) for small T
    T = cv * w.nsteps * w.dt / H ** 2
    s_exact = w.meta["load"] * H / (lam + 2 * G) * 2 * np.sqrt(T / np.pi)
    s_num = -pr.u[:, 1].min()
    assert s_num == pytest.approx(s_exact, rel=0.08)


def test_terzaghi_refinement_reduces_error():
    """Halving h and dt reduces the error against the closed form (Sec. 5.1 refinement study)."""
    def err(ny, h, dt, nsteps):
        w = W.terzaghi(ncell_x=2, ncell_y=ny, h=h, dt=dt, nsteps=nsteps)
        pr = O.from_workload(w)
        lam, G = O.lame(w.material.E, w.material.nu)
        cv = (lam + 2 * G) * w.material.k / w.material.mu_f
        H = w.meta["H"]
        for n in range(1, nsteps + 1):
            pr.step(dt, w.bc(n))
        Z = _reference_depth(pr, H) / H
        return np.sqrt(np.mean((pr.p / w.meta["load"] - terzaghi_exact(Z, cv * nsteps * dt / H ** 2)) ** 2))
    e1 = err(20, 0.25, 0.2, 2)
    e2 = err(40, 0.125, 0.1, 4)
    assert e2 < 0.7 * e1


def test_terzaghi_paper_parameters_stabilization():
    """The paper's own Terzaghi parameters (golden fixture, 40 cells over H = 1 m): one step of
    0.1 s lies inside the Vermeer-Verruijt bound dt < h^2/(6 c_v), so without stabilization the
    pressure shows a checkerboard through the column, while with tau_W it is w (undrained)
    below a thin, decaying oscillation next to the drained top (Sec. 5.1)."""
    with open(os.path.join(GOLDEN, "terzaghi_paper.json")) as f:
        gp = json.load(f)
    K, nu, cv, H, wload, dt = gp["K"], gp["nu"], gp["c_v"], gp["H"], gp["w"], gp["dt"]
    E = 3 * K * (1 - 2 * nu)
    lam, G = O.lame(E, nu)
    M = K + 4.0 / 3.0 * G
    assert lam + 2 * G == pytest.approx(M, rel=1e-12)
    kappa = cv / M
    ny = 40
    h = H / ny
    assert dt < h * h / (6 * cv)
    prof = {}
    for kind in (W.TAU_OFF, W.TAU_WHITE):
        w = W.terzaghi(ncell_x=1, ncell_y=ny, h=h, load=wload, k=kappa * 1e-3, dt=dt, nsteps=1,
                       E=E, nu=nu, tau_kind=kind)
        pr = O.from_workload(w)
        pr.step(dt, w.bc(1))
        z = _reference_depth(pr, H)
        o = np.argsort(z, kind="stable")
        prof[kind] = (z[o][::2], pr.p[o][::2] / wload)
    z, p_off = prof[W.TAU_OFF]
    _, p_on = prof[W.TAU_WHITE]
    deep = z > 0.25 * H
    # unstabilized: cell-to-cell oscillation of more than 5 % of w even a third of the way down
    assert np.abs(np.diff(p_off[(z > 0.2 * H) & (z < 0.4 * H)])).max() > 0.1
    # stabilized: undrained value below the boundary layer, oscillation decaying with depth
    assert np.abs(p_on[deep] - 1.0).max() < 1e-3
    near = np.abs(p_on[(z > 2 * h) & (z < 6 * h)] - 1.0).max()
    assert np.abs(p_on[(z > 6 * h) & (z < 12 * h)] - 1.0).max() < 0.5 * near


def _checkerboard(pr, ncx):
    """RMS of the second difference of the particle pressure along the column (one value per
    particle row, averaged across the row)."""
    order = np.argsort(pr.x[:, 1], kind="stable")
    rows = pr.p[order].reshape(-1, 2 * ncx).mean(axis=1)
    return np.sqrt(np.mean(np.diff(rows, 2) ** 2))


def test_stabilization_suppresses_checkerboard():
    """Undrained Terzaghi variant (k = 1e-15: dt = 0.1 s << h^2/(6 c_v)): without the PPP term the
    pressure oscillates from cell to cell; tau_W removes it; 0.1 tau_W is not enough and
    10 tau_W smooths more (Sec. 5.1, parameter study)."""
    idx = {}
    for name, kind, scale in (("off", W.TAU_OFF, 1.0), ("w01", W.TAU_WHITE, 0.1), ("w", W.TAU_WHITE, 1.0),
                              ("w10", W.TAU_WHITE, 10.0)):
        w = W.terzaghi(ncell_x=1, ncell_y=40, k=1e-15, nsteps=1, tau_kind=kind, tau_scale=scale)
        pr = O.from_workload(w)
        pr.step(w.dt, w.bc(1))
        idx[name] = _checkerboard(pr, 1) / w.meta["load"]
    assert idx["off"] > 10 * idx["w"]
    assert idx["w01"] > 2 * idx["w"]
    assert idx["w10"] <= idx["w"]


def test_patch_test_uniform_strain():
    """An affine nodal displacement field gives the same dF at every material point (both bases
    reproduce linear fields), and the internal force vanishes at interior nodes whose support is
    filled with regularly placed points (the point domains tile the cells)."""
    for shape in (0, 1):
        grid = W.Grid(2, (8, 8), 0.25, (0.0, 0.0, 0.0))
        mat = W.Material(model=W.NEO_HOOKEAN, k=0.0)
        opt = W.Options(shape=shape, dynamic=0, tau_kind=W.TAU_OFF)
        parts = W.fill_particles(grid, (0, 0), (8, 8), mat.rho0)
        pr = O.OracleProblem(grid, mat, opt, parts)
        nodal = pr.p2g()
        X = grid.node_coords()
        Hgrad = np.array([[2e-3, 1e-3], [-5e-4, -3e-3]])
        U = X @ Hgrad.T
        P = np.full(grid.nnode, 1234.5)
        R, _, _ = pr.assemble(U, P, nodal, 0.1, want_J=False)
        R = R.reshape(grid.nnode, 3)
        interior = (X[:, 0] > 1.0 * 0.25 + 1e-9) & (X[:, 0] < 7 * 0.25 - 1e-9) & \
                   (X[:, 1] > 0.25 + 1e-9) & (X[:, 1] < 7 * 0.25 - 1e-9)
        tau = O.kirchhoff(1, pr.lam, pr.G, np.eye(2) + Hgrad)
        scale = np.abs(tau).max() * 0.25
        assert np.abs(R[interior, :2]).max() < 1e-9 * scale
        # the mass residual at interior nodes is the same volumetric rate everywhere
        dJ = np.linalg.det(np.eye(2) + Hgrad)
        node_vol = 0.25 ** 2 * dJ
        assert np.abs(R[interior, 2] - node_vol * np.log(dJ) / 0.1).max() < 1e-9 * abs(node_vol * np.log(dJ) / 0.1)


def test_rigid_translation_dynamic():
    """Uniform initial velocity, no supports and no load: the body translates rigidly,
    u = v0 t, with zero pore pressure and effective stress (Newmark + FLIP, Sec. 3.2, 3.5)."""
    for shape in (0, 1):
        grid = W.Grid(2, (10, 10), 0.25, (0.0, 0.0, 0.0))
        mat = W.Material(model=W.NEO_HOOKEAN, k=1e-12)
        opt = W.Options(shape=shape, dynamic=1, beta=0.25, gamma=0.5, tau_kind=W.TAU_WHITE)
        parts = W.fill_particles(grid, (3, 3), (7, 7), mat.rho0)
        v0 = np.array([0.3, -0.2])
        parts.v0 = np.tile(v0, (parts.n, 1))
        pr = O.OracleProblem(grid, mat, opt, parts)
        dt = 0.05
        bc = W.empty_bc(grid)
        for n in range(1, 5):
            pr.step(dt, bc)
        assert np.abs(pr.u - v0 * 4 * dt).max() < 1e-10
        assert np.abs(pr.p).max() < 1e-4
        assert np.abs(pr.F - np.eye(2)).max() < 1e-10          # rounding only
        assert np.abs(pr.v - v0).max() < 1e-10


def test_mass_conservation_and_volume():
    """Lumped P2G preserves the total mass (partition of unity, eq. map-from-particles-to-nodes)
    up to the nodes below 1e-15 of the largest nodal mass, which are outside the material; the
    point volume follows V = det(dF) V_n, so sum V equals sum J V_0 after steps."""
    w = W.config(2, nx=8, ny=8, nsteps=3, dt=1e-2)
    pr = O.from_workload(w)
    m0 = pr.m.sum()
    V0 = pr.V.copy()
    for n in range(1, 4):
        pr.step(w.dt, w.bc(n))
        nodal = pr.p2g()
        nn = nodal["M"].size
        assert nodal["M"].sum() == pytest.approx(m0, rel=1e-13 + nn * 1e-15 * nodal["M"].max() / m0)
        assert nodal["M"].sum() <= m0 * (1 + 1e-13)
    J = np.linalg.det(pr.F)
    assert np.abs(pr.V - J * V0).max() < 1e-13 * V0.max()


def test_undrained_volume_constraint():
    """Impermeable box (k = 0), no PPP, quasi-static: the discrete mass balance reduces to
    sum_mp dv S_i ln(dJ)/dt = 0 at every node, so the total sum_mp dv ln(dJ) vanishes at
    convergence (Sec. 4.1, undrained limit)."""
    grid = W.Grid(2, (6, 6), 0.25, (0.0, 0.0, 0.0))
    mat = W.Material(model=W.NEO_HOOKEAN, k=0.0)
    opt = W.Options(shape=0, dynamic=0, tau_kind=W.TAU_WHITE)
    parts = W.fill_particles(grid, (0, 0), (6, 6), mat.rho0)
    pr = O.OracleProblem(grid, mat, opt, parts)
    bc = W.empty_bc(grid)
    W.box_supports(grid, bc, (1.5,))
    X = grid.node_coords()
    top = np.abs(X[:, 1] - 1.5) < 1e-9
    bc["f_ext"][top, 1] = -1e5 * 0.25
    bc["f_ext"][top & (X[:, 0] > 0.7), 1] *= 3.0
    V_n = pr.V.copy()
    pr.step(0.1, bc, rtol=1e-12)
    dJ = pr.V / V_n
    assert abs(np.sum(pr.V * np.log(dJ))) < 1e-10 * np.sum(pr.V)
    assert np.abs(pr.u).max() > 1e-5     # the load does deform the body (isochorically)


def _stab_matrix(shape, ppc_axis, seed=0):
    grid = W.Grid(2, (5, 5), 0.5, (0.0, 0.0, 0.0))
    rng = np.random.default_rng(seed)
    mat = W.Material(model=W.NEO_HOOKEAN, k=1e-10)
    parts = W.fill_particles(grid, (1, 1), (4, 4), mat.rho0, ppa=ppc_axis, jitter=0.5, rng=rng)
    out = []
    for kind in (W.TAU_WHITE, W.TAU_OFF):
        opt = W.Options(shape=shape, dynamic=0, tau_kind=kind)
        pr = O.OracleProblem(grid, mat, opt, parts)
        nodal = pr.p2g()
        U = 1e-3 * (rng.random((grid.nnode, 2)) - 0.5) * nodal["active"][:, None]
        rng = np.random.default_rng(seed)
        _, J, _ = pr.assemble(U * 0, nodal["Pn"], nodal, 0.1)
        out.append(J.toarray()[2::3, 2::3])
    act = nodal["active"]
    C = (out[0] - out[1])[np.ix_(act, act)]
    return C


@pytest.mark.parametrize("shape", [0, 1])
def test_ppp_matrix_properties(shape):
    """C_stab = tau c_t sum V (S - Pi S)(S - Pi S)^T is symmetric positive semi-definite and has
    the constants in its null space (Pi reproduces constants, eq. projection-operator)."""
    C = _stab_matrix(shape, 2)
    assert np.abs(C - C.T).max() < 1e-14 * np.abs(C).max()
    ev = np.linalg.eigvalsh(0.5 * (C + C.T))
    assert ev.min() > -1e-12 * ev.max()
    assert np.abs(C @ np.ones(C.shape[0])).max() < 1e-12 * np.abs(C).max()


def test_ppp_vanishes_with_one_point_per_cell():
    """Original MPM with the particle-quadrature cell mean: one point per cell makes S - Pi S = 0,
    so the stabilization term vanishes identically (the motivation of Sec. 4.4)."""
    C = _stab_matrix(0, 1)
    assert np.abs(C).max() == 0.0


def test_free_fall_newmark_closed_form():
    """Free fall of an unsupported body from rest with zero initial acceleration, Newmark with the
    paper's beta = 0.3025, gamma = 0.6 (Sec. 3.2): the momentum balance gives a = g at every
    step, so the scalar Newmark recursion u += dt v + dt^2((1/2 - beta) a_n + beta a),
    v += dt((1 - gamma) a_n + gamma a) is the exact discrete answer (FLIP update of Sec. 3.5);
    the pore pressure and the effective stress stay zero (a = a_f, Sec. 2.1)."""
    for shape in (0, 1):
        grid = W.Grid(2, (12, 12), 0.25, (0.0, 0.0, 0.0))
        gvec = np.array([0.0, -9.81])
        mat = W.Material(model=W.NEO_HOOKEAN, k=1e-12, g=(0.0, -9.81, 0.0))
        opt = W.Options(shape=shape, dynamic=1, beta=0.3025, gamma=0.6, tau_kind=W.TAU_WHITE)
        parts = W.fill_particles(grid, (3, 5), (8, 9), mat.rho0)
        v0 = np.array([0.2, 0.5])
        parts.v0 = np.tile(v0, (parts.n, 1))
        pr = O.OracleProblem(grid, mat, opt, parts)
        dt, be, ga = 0.02, 0.3025, 0.6
        u = np.zeros(2); v = v0.copy(); a = np.zeros(2)
        bc = W.empty_bc(grid)
        for n in range(1, 6):
            pr.step(dt, bc, rtol=1e-12)
            u = u + dt * v + dt * dt * ((0.5 - be) * a + be * gvec)
            v = v + dt * ((1 - ga) * a + ga * gvec)
            a = gvec.copy()
        assert np.abs(pr.u - u).max() < 1e-10
        assert np.abs(pr.v - v).max() < 1e-9
        assert np.abs(pr.a - gvec).max() < 1e-8
        # rounding level against the hydrostatic scale rho g h = 5e3 Pa
        assert np.abs(pr.p).max() < 1e-4
        assert np.abs(pr.sig).max() < 1e-4


def test_kozeny_carman_mobility_values():
    """Kozeny-Carman law (eq. kozeny-carman) with phi = 1 - (1 - phi0)/J: the initial state gives
    k0; phi0 = 1/2 and J = 2 give phi = 3/4 and k/k0 = (1/4 / 1/8) (27/64 / 1/16) = 2 x 27/4 = 13.5;
    phi0 = 1/2 and J = 4/5 give phi = 3/8 and k/k0 = 2 (27/512) / (25/64) = 27/100; the derivative
    agrees with central differences; phi0 = 0 keeps the constant mobility."""
    from oracle import oracle as O
    k, _ = O.mobility(2.0, 0.3, 1.0)
    assert abs(k - 2.0) <= 1e-15
    k, _ = O.mobility(1.0, 0.5, 2.0)
    assert abs(k - 13.5) <= 1e-13
    k, _ = O.mobility(1.0, 0.5, 0.8)
    assert abs(k - 27.0 / 100.0) <= 1e-15
    for phi0, J in ((0.33, 0.9), (0.33, 1.2), (0.5, 2.0), (0.1, 1.05)):
        _, dk = O.mobility(1.0, phi0, J)
        e = 1e-6
        fd = (O.mobility(1.0, phi0, J + e)[0] - O.mobility(1.0, phi0, J - e)[0]) / (2 * e)
        assert abs(dk - fd) <= 1e-7 * abs(fd), (phi0, J, dk, fd)
    assert O.mobility(3.0, 0.0, 1.7) == (3.0, 0.0)
    # below the porosity floor the mobility is held: constant, zero derivative
    k1, d1 = O.mobility(1.0, 0.3, 0.7)
    k2, d2 = O.mobility(1.0, 0.3, 0.6)
    assert d1 == 0.0 and d2 == 0.0 and k1 == k2


@pytest.mark.parametrize("shape", [W.LINEAR, W.GIMP])
def test_viscous_damping_dissipates(shape):
    """The Kelvin-type viscous term (Sec. 2.2) only dissipates: with zero nodal kinematics at t_n
    the Newmark velocity is proportional to U (eq. newmark), and the viscous part of the momentum
    residual does negative work, sum_i U_i . R_vis,i < 0, for any increment; it vanishes for a
    rigid translation (l = 0)."""
    r = np.random.default_rng(12)
    res = {}
    Us = None
    for alpha in (0.0, 0.05):
        w = W.jittered_box(5, 5, h=0.25, shape=shape, dynamic=1, seed=6, jitter=0.5, empty=1)
        w.material.alpha_vis = alpha
        pr = O.from_workload(w)
        nodal = pr.p2g()
        nn, d = w.grid.nnode, 2
        nodal["vn"] = np.zeros(nn * d)
        nodal["an"] = np.zeros(nn * d)
        act = nodal["active"]
        if Us is None:
            Us = [1e-4 * (r.random((nn, d)) - 0.5) * act[:, None] for _ in range(4)]
            Us.append(np.tile([3e-4, -2e-4], (nn, 1)) * act[:, None])          # rigid translation
        res[alpha] = [pr.assemble(u, nodal["Pn"], nodal, 1e-3, want_J=False)[0].reshape(nn, d + 1)[:, :d]
                      for u in Us]
    for k, u in enumerate(Us):
        Rv = res[0.05][k] - res[0.0][k]
        work = float(np.sum(Rv * u))
        scale = float(np.abs(Rv).max() * np.abs(u).max()) + 1e-300
        if k < 4:
            assert work < 0.0 and np.abs(Rv).max() > 0.0
        else:
            assert np.abs(Rv).max() <= 1e-9 * np.abs(res[0.0][k]).max(), k


@pytest.mark.parametrize("dim,seed", [(2, 0), (2, 1), (3, 2)])
def test_free_surface_nodes_brute_force(dim, seed):
    """The drained free surface of the self-weight example: active nodes with an inactive neighbour
    among the 3^dim - 1 nodes around them that lie inside the grid, by direct enumeration."""
    rng = np.random.default_rng(seed)
    nc = (5, 4, 3)[:dim]
    grid = W.Grid(dim, nc, 0.5, (0.0, 0.0, 0.0))
    nn = [c + 1 for c in nc]
    act = rng.random(int(np.prod(nn))) < 0.7
    got = O.free_surface_nodes(grid, act)
    want = np.zeros_like(act)
    for idx in np.ndindex(*reversed(nn)):
        ijk = tuple(reversed(idx))                      # x fastest in the natural node order
        lin = sum(ijk[a] * int(np.prod(nn[:a])) for a in range(dim))
        if not act[lin]:
            continue
        for off in np.ndindex(*([3] * dim)):
            q = [ijk[a] + off[a] - 1 for a in range(dim)]
            if all(o == 1 for o in off) or any(q[a] < 0 or q[a] >= nn[a] for a in range(dim)):
                continue
            if not act[sum(q[a] * int(np.prod(nn[:a])) for a in range(dim))]:
                want[lin] = True
    assert np.array_equal(got, want)
    assert got.any() and not got.all()


def test_self_weight_consolidation_end_state():
    """Sec. 5.3 problem (coarse: h = 0.25 m, 2 x 2 points per cell), drained through its free top
    only: gravity at t = 0 is carried by the pore fluid first (undrained: the pressure at the base
    is close to the total weight of the column), the excess pressure then dissipates (dt growing by
    1.2 per step) to the hydrostatic state, in which the effective stress carries the buoyant
    weight of the settled column."""
    w = W.self_weight(h=0.25, ppa=2, nsteps=130, right_drained=False)
    pr = O.from_workload(w)
    lam, G = O.lame(w.material.E, w.material.nu)
    M = lam + 2 * G
    rho0, rf, g = w.material.rho0, w.material.rho_f, 9.81
    H = w.meta["H"]
    st = pr.step(w.meta["dt_of"](1), w.bc(1))
    base = (pr.x[:, 1] < 0.25) & (pr.x[:, 0] < 1.0)     # away from the drained right edge
    # undrained first step: the base pressure carries (nearly) the whole column
    assert pr.p[base].mean() == pytest.approx(rho0 * g * (H - 0.125), rel=0.05)
    for n in range(2, w.nsteps + 1):
        pr.step(w.meta["dt_of"](n), w.bc(n))
    # hydrostatic end state: the pore pressure grows with depth at rho_f g (eq. darcy-law with
    # gravity; zero pressure holds on the surface nodes, up to a cell above the last points)
    fit = np.polyfit(pr.x[:, 1], pr.p, 1)
    assert fit[0] == pytest.approx(-rf * g, rel=0.03)
    assert np.abs(pr.p - np.polyval(fit, pr.x[:, 1])).max() < 0.03 * rf * g * H
    # vertical equilibrium of the mixture (eq. residual-momentum with m g): the total stress at a
    # point carries the weight of the (constant) point masses above it, rho0 g (H - Z) with Z the
    # point's initial elevation, although the column has settled by large strains
    Z = pr.x[:, 1] - pr.u[:, 1]
    total = pr.sig[:, 1, 1] - pr.p
    inner = (Z > 0.3) & (Z < H - 0.3)
    assert np.abs(total[inner] + rho0 * g * (H - Z[inner])).max() < 0.03 * rho0 * g * H
    assert -pr.u[:, 1].min() > 0.2            # large strain: tens of centimetres on a 2 m column
    assert np.linalg.det(pr.F).min() < 0.75


def test_two_body_impact_momentum_and_contact():
    """Sec. 5.4 impact of two poroelastic discs (coarse grid, discs started closer so that they
    meet early): the bodies share the grid's single velocity field (the method's own no-slip
    contact), there are no external forces, and the internal forces of every node sum to zero
    (partition of unity of the basis), so the total momentum stays zero through the contact to
    the Newton tolerance; the collision takes kinetic energy into strain and pore pressure, and
    the points that carry the drained condition keep p = 0 (all nodes of their basis hold it)."""
    w = W.two_body_impact(h=0.05, ppa=2, v0=0.1, dt=1e-3, centre=0.3)
    w.options.negligible_mass = 0.0       # every node with mass (the method's own conservation)
    pr = O.from_workload(w)
    n1 = w.meta["bodies"][0]
    body = np.abs((pr.m[:n1, None] * pr.v[:n1]).sum(0)).max()
    assert body > 10.0 and np.abs((pr.m[:, None] * pr.v).sum(0)).max() < 1e-12 * body
    ke0 = 0.5 * (pr.m * (pr.v ** 2).sum(1)).sum()
    for n in range(1, 601):
        pr.step(w.dt, w.bc(n))
        if n % 100 == 0:
            assert np.abs((pr.m[:, None] * pr.v).sum(0)).max() < 1e-10 * body, n
    ke = 0.5 * (pr.m * (pr.v ** 2).sum(1)).sum()
    assert ke < 0.75 * ke0                      # the collision is under way
    assert np.abs(pr.p).max() > 10.0            # and has raised pore pressure
    assert np.abs(pr.p[w.meta["drained"]]).max() == 0.0
    assert np.linalg.det(pr.F).min() < 0.9


def test_two_body_impact_negligible_mass_cut():
    """The impact workload leaves nodes below 1e-5 of the largest nodal mass out of the material.
    Momentum is then conserved up to what those nodes carried: each step drops at most a few
    nodes of mass < 1e-5 M_max moving at < 2 v0, so over 700 steps the total stays below 1e-4 of
    one body's momentum (measured ~1e-6); and Newton takes at most 4 iterations through the
    contact (with every node kept, the grazed nodes make this run's contact steps take up to 8,
    and 13 on the coarse workload started at 0.2 m)."""
    w = W.two_body_impact(h=0.05, ppa=2, v0=0.1, dt=1e-3, centre=0.3)
    assert w.options.negligible_mass == 1e-5
    pr = O.from_workload(w)
    n1 = w.meta["bodies"][0]
    body = np.abs((pr.m[:n1, None] * pr.v[:n1]).sum(0)).max()
    ke0 = 0.5 * (pr.m * (pr.v ** 2).sum(1)).sum()
    worst = 0
    for n in range(1, 701):
        st = pr.step(w.dt, w.bc(n))
        worst = max(worst, st["newton_iters"])
    assert np.abs((pr.m[:, None] * pr.v).sum(0)).max() < 1e-4 * body
    assert worst <= 4, worst
    assert 0.5 * (pr.m * (pr.v ** 2).sum(1)).sum() < 0.75 * ke0   # through the contact
