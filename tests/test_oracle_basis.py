"""Pins of the oracle's basis functions (Sec. 3.1, eq. gimp-basis / gimp-basis-gradient; Sec. 4.4)
against brute-force quadrature of their definitions, partition of unity and linear reproduction."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1905_00671_amd.workloads import Grid


def _hat(r, h):
    return np.maximum(0.0, 1.0 - np.abs(r) / h)


def _dhat(r, h):
    return np.where(np.abs(r) < h, -np.sign(r) / h, 0.0)


def _brute_gimp_1d(xp, lp, xi, h, lo, hi, n=200000):
    """Midpoint quadrature of S = (1/V) int chi N dxi, dS = (1/V) int chi N' dxi over the particle
    domain clipped to the grid."""
    a, b = max(xp - lp, lo), min(xp + lp, hi)
    s = a + (np.arange(n) + 0.5) * (b - a) / n
    return float(np.mean(_hat(s - xi, h))), float(np.mean(_dhat(s - xi, h)))


@pytest.mark.parametrize("seed", range(6))
def test_gimp_matches_quadrature_2d(seed):
    rng = np.random.default_rng(seed)
    h = 0.5
    g = Grid(2, (6, 5), h, (0.0, 0.0, 0.0))
    lp = rng.uniform(0.05, 0.5, 2) * h
    xp = np.array([rng.uniform(0.0, 6 * h), rng.uniform(0.0, 5 * h)])
    nodes, S, G, S0 = O.basis(g, 1, xp, lp)
    X = g.node_coords()
    for k, nid in enumerate(nodes):
        wx, dx = _brute_gimp_1d(xp[0], lp[0], X[nid, 0], h, 0.0, 6 * h)
        wy, dy = _brute_gimp_1d(xp[1], lp[1], X[nid, 1], h, 0.0, 5 * h)
        assert abs(S[k] - wx * wy) < 1e-8
        # N' jumps by up to 2/h; a midpoint rule misplaces at most one sample per jump,
        # so the brute-force gradient is exact to 2/(h n) per factor
        assert abs(G[k, 0] - dx * wy) < 4.0 / (h * 200000)
        assert abs(G[k, 1] - wx * dy) < 4.0 / (h * 200000)


def test_gimp_worked_values():
    """lp = h/4, particle on a node: S = 1 - lp/(2h) = 0.875 there, (h + lp - h)^2/(4 h lp) = 0.0625
    on each neighbour (closed form of eq. gimp-basis)."""
    h = 1.0
    g = Grid(2, (4, 4), h, (0.0, 0.0, 0.0))
    nodes, S, G, S0 = O.basis(g, 1, np.array([2.0, 2.0]), np.array([0.25, 0.25]))
    X = g.node_coords()
    w = {tuple(X[n]): s for n, s in zip(nodes, S)}
    assert w[(2.0, 2.0)] == pytest.approx(0.875 ** 2, abs=1e-14)
    assert w[(1.0, 2.0)] == pytest.approx(0.0625 * 0.875, abs=1e-14)
    assert w[(1.0, 1.0)] == pytest.approx(0.0625 ** 2, abs=1e-14)
    assert sum(S) == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("shape", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_partition_of_unity_and_linear_reproduction(shape, dim):
    rng = np.random.default_rng(7 + dim + shape)
    h = 0.3
    nc = (5, 4, 3)[:dim]
    g = Grid(dim, nc + (1,) * (3 - dim), h, (0.1, -0.2, 0.05))
    X = g.node_coords()
    for _ in range(40):
        xp = np.array([g.origin[a] + rng.uniform(0, nc[a] * h) for a in range(dim)])
        lp = rng.uniform(0.05, 0.5, dim) * h
        nodes, S, G, S0 = O.basis(g, shape, xp, lp)
        assert abs(S.sum() - 1.0) < 1e-13
        assert np.abs(G.sum(axis=0)).max() < 1e-12 / h
        # sum S x_i = x_p holds for the hat basis; for GIMP it holds inside the grid (the
        # domain average of the identity is the domain centre, shifted when the domain is clipped)
        xs = (S[:, None] * X[nodes]).sum(axis=0)
        if shape == 0:
            assert np.abs(xs - xp).max() < 1e-12
        # sum x_i (x) grad S_i = I
        I = (X[nodes][:, :, None] * G[:, None, :]).sum(axis=0)
        assert np.abs(I - np.eye(dim)).max() < 1e-12
        if shape == 1:
            assert abs(S0.sum() - 1.0) < 1e-13
            assert np.all(S0 >= 0)


def test_gimp_reduces_to_hat_for_vanishing_domain():
    """lp -> 0: GIMP weights tend to the hat functions of the original MPM."""
    g = Grid(2, (4, 4), 1.0, (0.0, 0.0, 0.0))
    xp = np.array([1.3, 2.6])
    n1, S1, G1, _ = O.basis(g, 1, xp, np.array([1e-7, 1e-7]))
    n0, S0_, G0, _ = O.basis(g, 0, xp, None)
    d1 = {n: s for n, s in zip(n1, S1)}
    for n, s in zip(n0, S0_):
        assert abs(d1.get(n, 0.0) - s) < 1e-6


def test_s0_inside_one_cell():
    """S0 = 2^-d on the nodes of the containing cell when the domain lies inside it (Sec. 4.4)."""
    g = Grid(2, (4, 4), 1.0, (0.0, 0.0, 0.0))
    nodes, S, G, S0 = O.basis(g, 1, np.array([1.5, 2.5]), np.array([0.25, 0.25]))
    X = g.node_coords()
    for n, s0 in zip(nodes, S0):
        inside = (1.0 <= X[n, 0] <= 2.0) and (2.0 <= X[n, 1] <= 3.0)
        assert s0 == pytest.approx(0.25 if inside else 0.0, abs=1e-15)
