"""Pins of the oracle parts that no residual or Jacobian identity reaches: the stabilization
parameters of Sec. 4.3 (hand values), the GIMP domain update of Sec. 3.5 (the symmetric material
stretch, against an independent matrix square root) and the Newmark pressure history of
eq. p-dot-newmark (Newmark integrates quadratic time histories exactly for any beta, gamma, so a
quadratic p(t) must come out exact in G2P and in the stabilization residual)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from paper_1905_00671_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hand():
    with open(os.path.join(GOLDEN, "stab_parameter_hand_values.json")) as f:
        return json.load(f)


def test_tau_white_sun_hand_values():
    """eq. tau-white and eq. tau-sun at lambda = 2, G = 1 (M = 4), h = dt = 1: the values worked
    by hand, including the zero of (1 - 3c) and the clamp at zero beyond it."""
    g = _hand()
    assert O.stab_parameter(1, 1.0, g["E"], g["nu"], 0.0, g["h"], g["dt"], 0.25, 0.5) == pytest.approx(
        g["tau_white"], rel=1e-14)
    for case in g["tau_sun"]:
        got = O.stab_parameter(2, 1.0, g["E"], g["nu"], case["kappa"], g["h"], g["dt"], 0.25, 0.5)
        assert got == pytest.approx(case["value"], rel=1e-12, abs=1e-15), case


def test_tau_monforte_hand_values():
    """eq. tau-monforte: the Newmark ratio beta/gamma enters, the max operator clamps at zero and
    2 kappa / c_v tends to 2/M as the mobility vanishes."""
    g = _hand()
    for case in g["tau_monforte"]:
        got = O.stab_parameter(3, 1.0, g["E"], g["nu"], case["kappa"], g["h"], g["dt"], case["beta"],
                               case["gamma"])
        assert got == pytest.approx(case["value"], rel=1e-12, abs=1e-15), case


def test_tau_scale_multiplies():
    g = _hand()
    for kind in (1, 2, 3):
        a = O.stab_parameter(kind, 1.0, g["E"], g["nu"], 1.0 / 48, g["h"], g["dt"], 0.25, 0.5)
        b = O.stab_parameter(kind, 10.0, g["E"], g["nu"], 1.0 / 48, g["h"], g["dt"], 0.25, 0.5)
        assert b == pytest.approx(10.0 * a, rel=1e-14)


def _affine_g2p(F, shape=W.GIMP, seed=0):
    """G2P of a GIMP block under the affine nodal increment U_i = (F - 1) X_i, for which the
    relative deformation gradient of every point whose domain lies inside the grid is exactly F
    (GIMP reproduces linear fields).  Returns the oracle problem after the update and the mask
    of interior points."""
    w = W.jittered_box(6, 6, h=0.25, shape=shape, seed=seed, jitter=0.5, empty=2)
    pr = O.from_workload(w)
    nodal = pr.p2g()
    X = w.grid.node_coords()
    c = X.mean(axis=0)
    U = (X - c) @ (np.asarray(F) - np.eye(2)).T
    P = np.zeros(w.grid.nnode)
    pr.g2p(U, P, nodal, w.dt)
    return w, pr


@pytest.mark.parametrize("theta,s,rot", [(0.3, 1.4, 0.0), (0.3, 1.4, 0.7), (1.1, 0.7, -0.4), (0.0, 1.0, 0.9)])
def test_gimp_domain_update_is_right_stretch(theta, s, rot):
    """Sec. 3.5 (domain update after Charlton et al.): lp_d = lp0_d U_dd with U = sqrt(F^T F) the
    symmetric material (right) stretch.  F = R A with A a stretch s along an axis at angle theta
    and R a rotation: U = A whatever R is, while the spatial (left) stretch R A R^T differs once
    R is not the identity.  U is taken here from SciPy's matrix square root."""
    q = np.array([[np.cos(theta), -np.sin(theta)], [np.sin(theta), np.cos(theta)]])
    A = q @ np.diag([s, 1.0]) @ q.T
    R = np.array([[np.cos(rot), -np.sin(rot)], [np.sin(rot), np.cos(rot)]])
    F = R @ A
    w, pr = _affine_g2p(F)
    h = w.grid.h
    Uref = np.real(scipy.linalg.sqrtm(F.T @ F))
    assert np.allclose(Uref, A, atol=1e-12)
    assert np.allclose(pr.F, F[None], atol=1e-12)        # every point is interior here
    expect = np.minimum(pr.lp0 * np.diag(Uref)[None, :], 0.5 * h)
    assert np.abs(pr.lp - expect).max() <= 1e-13 * h
    if abs(rot) > 0.1 and abs(theta) > 0.1 and s != 1.0:
        V = F @ R.T                                        # left stretch R A R^T
        wrong = np.minimum(pr.lp0 * np.diag(V)[None, :], 0.5 * h)
        assert np.abs(pr.lp - wrong).max() > 1e-3 * h


def test_gimp_domain_update_clamps_at_half_cell():
    """A stretch that would make a domain longer than the cell is held at lp = h/2."""
    F = np.diag([2.5, 0.9])
    w, pr = _affine_g2p(F)
    h = w.grid.h
    assert np.allclose(pr.lp[:, 0], 0.5 * h, atol=1e-15)
    assert np.allclose(pr.lp[:, 1], pr.lp0[:, 1] * 0.9, atol=1e-15)


def _quadratic_history(beta, gamma, shape):
    """Every displacement fixed, every pressure prescribed as p(t) = a + b t + c t^2, points
    starting with the exact p, pdot and pddot at t = 0."""
    w = W.jittered_box(4, 4, h=0.25, shape=shape, dynamic=1, seed=5, jitter=0.5, empty=1)
    w.options.beta, w.options.gamma = beta, gamma
    pr = O.from_workload(w)
    a, b, c = 1.0e4, 3.0e3, -2.0e4
    pr.p[:] = a
    pr.pd[:] = b
    pr.pdd[:] = 2 * c
    return w, pr, (a, b, c)


@pytest.mark.parametrize("shape", [W.LINEAR, W.GIMP])
@pytest.mark.parametrize("beta,gamma", [(0.3025, 0.6), (0.25, 0.5)])
def test_newmark_pressure_history_exact_for_quadratic(beta, gamma, shape):
    """eq. p-dot-newmark: a Newmark scheme reproduces p, pdot, pddot exactly when p(t) is quadratic
    in time (for any beta, gamma).  The pressure is prescribed on every node and the material
    points must carry p(t_n), p'(t_n) = b + 2 c t_n and p'' = 2 c through the G2P update."""
    w, pr, (a, b, c) = _quadratic_history(beta, gamma, shape)
    nn, d = w.grid.nnode, w.grid.dim
    dt = 0.05
    for n in range(1, 5):
        t = n * dt
        bc = W.empty_bc(w.grid)
        bc["u_fixed"][:] = 1
        bc["p_fixed"][:] = 1
        bc["p_val"][:] = a + b * t + c * t * t
        st = pr.step(dt, bc)
        assert st["newton_iters"] == 0
        scale = abs(a) + abs(b) + abs(c)
        assert np.abs(pr.p - (a + b * t + c * t * t)).max() <= 1e-12 * scale
        assert np.abs(pr.pd - (b + 2 * c * t)).max() <= 1e-10 * scale
        assert np.abs(pr.pdd - 2 * c).max() <= 1e-8 * scale
        assert np.abs(pr.u).max() == 0.0


@pytest.mark.parametrize("shape", [W.LINEAR, W.GIMP])
def test_stabilization_rate_newmark_equals_exact_rate(shape):
    """eq. stab-term-ppp with eq. p-dot-newmark: for nodal pressure histories that are quadratic in
    time (random in space), the Newmark rate at t_{n+1} is the exact rate b_j + 2 c_j t_{n+1}.  The
    mass residual of the dynamic path (with U = 0, zero nodal kinematics and zero mobility, so
    only the stabilization term is left) must equal that of the quasi-static path, whose rate
    (P - P_n)/dt (eq. p-dot-implicit-euler) is given the exact value directly."""
    beta, gamma = 0.3025, 0.6
    rng = np.random.default_rng(7)
    out = {}
    dt, t1 = 0.05, 0.15
    for dyn in (1, 0):
        w = W.jittered_box(5, 5, h=0.25, shape=shape, dynamic=dyn, seed=9, jitter=0.5, empty=1, k=0.0)
        w.options.beta, w.options.gamma = beta, gamma
        pr = O.from_workload(w)
        nn, d = w.grid.nnode, w.grid.dim
        if dyn:
            r = np.random.default_rng(11)
            A = 1e4 * r.random(nn)
            Bq = 3e3 * (r.random(nn) - 0.5)
            C = 2e4 * (r.random(nn) - 0.5)
        nodal = pr.p2g()
        if dyn:
            t0 = t1 - dt
            nodal["Pn"] = A + Bq * t0 + C * t0 * t0
            nodal["pdn"] = Bq + 2 * C * t0
            nodal["pddn"] = 2 * C
            nodal["vn"] = np.zeros(nn * d)
            nodal["an"] = np.zeros(nn * d)
            P = A + Bq * t1 + C * t1 * t1
        else:
            nodal["Pn"] = np.zeros(nn)
            P = dt * (Bq + 2 * C * t1)
        U = np.zeros((nn, d))
        R, _, _ = pr.assemble(U, P, nodal, dt, want_J=False)
        out[dyn] = R.reshape(nn, d + 1)[:, d]
    scale = np.abs(out[0]).max()
    assert scale > 0
    assert np.abs(out[1] - out[0]).max() <= 1e-10 * scale
