"""Shared helpers of the GPU parity tests: the same seeded inputs go to the HIP library (through
the C ABI) and to the CPU oracle; comparisons follow the element-wise / per-block rules of the
parity tests."""
import numpy as np

from oracle import oracle as O
from paper_1905_00671_amd import workloads as W


def oracle_masked_residual(pr, nodal, U, P, bc, dt):
    """Oracle residual with the nodal loads and the Dirichlet / inactive rows removed, in the
    node-interleaved layout of the library."""
    g, d = pr.grid, pr.grid.dim
    nn = g.nnode
    R, J, _ = pr.assemble(U, P, nodal, dt, want_J=True)
    fext = np.zeros((nn, d + 1))
    fext[:, :d] = bc["f_ext"].reshape(nn, d)
    fext[:, d] = -bc["q_ext"]
    free = free_mask(nodal, bc, d)
    return (R + fext.reshape(-1)) * free, J, free


def free_mask(nodal, bc, d):
    nn = nodal["active"].shape[0]
    fixed = np.zeros((nn, d + 1), bool)
    fixed[:, :d] = bc["u_fixed"].astype(bool).reshape(nn, d)
    fixed[:, d] = bc["p_fixed"].astype(bool)
    return ((~fixed) & nodal["active"][:, None]).reshape(-1)


def oracle_jv(J, free, v):
    """J v with non-free rows/columns replaced by the identity."""
    vf = v * free
    y = J @ vf
    return np.where(free, y, v)


def block_err(a, b, d):
    """max |a - b| / max |b| per dof block (u components together, p separately)."""
    a = a.reshape(-1, d + 1)
    b = b.reshape(-1, d + 1)
    out = []
    for sl in (slice(0, d), slice(d, d + 1)):
        den = np.abs(b[:, sl]).max()
        out.append(np.abs(a[:, sl] - b[:, sl]).max() / (den if den > 0 else 1.0))
    return out


def rel_l2(a, b, floor=0.0):
    den = max(np.linalg.norm(b), floor)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def dyn_oracle_nodal(pr, bc):
    nodal = pr.p2g()
    g, d = pr.grid, pr.grid.dim
    if pr.opt.dynamic:
        ufix = bc["u_fixed"].astype(bool).reshape(g.nnode, d)
        for k in ("vn", "an"):
            v = nodal[k].reshape(g.nnode, d)
            v[ufix] = 0.0
            nodal[k] = v.reshape(-1)
    return nodal


def field_errors(got, ref, dynamic, gimp, E=None, dt=None):
    """Element-wise errors of the material-point state: for each field the largest absolute
    difference over the points, divided by the field's own scale (u, v, a, pdot, pddot, sigma':
    their largest magnitude; p: max(|p|, 1e-3 |sigma'|) so that drained states with p -> 0 stay
    meaningful; x: the displacement scale, since x - x0 = u on both sides; F, and the relative
    volume and GIMP-length changes: the strain scale max |F - 1|).  Fields that vanish in exact
    arithmetic (a body in free flight: F = 1, p = sigma' = a = 0) hold rounding noise only, so the
    scales have floors: strain 1e-6, stresses and pressure 1e-6 E, and with the step dt the rates
    1e-6 |v| / dt (a), 1e-6 E / dt (pdot) and 1e-6 E / dt^2 (pddot)."""
    def mx(a):
        return float(np.abs(a).max()) if np.size(a) else 0.0

    def rel(a, b, scale):
        return mx(np.asarray(a) - np.asarray(b)) / (scale if scale > 0 else 1.0)

    d = ref["F"].shape[-1]
    fl_s = 1e-6 * E if E else 0.0
    strain = max(mx(ref["F"] - np.eye(d)[None]), 1e-6 if E else 0.0)
    out = {
        "u": rel(got["u"], ref["u"], mx(ref["u"])),
        "p": rel(got["p"], ref["p"], max(mx(ref["p"]), 1e-3 * mx(ref["sig"]), fl_s)),
        "x": rel(got["x"], ref["x"], mx(ref["u"])),
        "F": rel(got["F"], ref["F"], strain),
        "vol": mx((np.asarray(got["vol"]) - ref["vol"]) / ref["vol"]) / (strain if strain > 0 else 1.0),
        "sig": rel(got["sig"], ref["sig"], max(mx(ref["sig"]), fl_s)),
    }
    if gimp:
        out["lp"] = mx((np.asarray(got["lp"]) - ref["lp"]) / ref["lp"]) / (strain if strain > 0 else 1.0)
    if dynamic:
        floors = {"v": 0.0, "a": 0.0, "pd": 0.0, "pdd": 0.0}
        if E and dt:
            floors = {"v": 0.0, "a": 1e-6 * mx(ref["v"]) / dt, "pd": fl_s / dt, "pdd": fl_s / dt ** 2}
        for k in ("v", "a", "pd", "pdd"):
            out[k] = rel(got[k], ref[k], max(mx(ref[k]), floors[k]))
    return out


GPU_FIELDS = ("u", "p", "x", "F", "vol", "sig", "lp", "v", "a", "pd", "pdd")


def gpu_state(gp, idx=None):
    out = {}
    for k in GPU_FIELDS:
        v = gp.get(k)
        out[k] = v if idx is None else v[idx]
    return out


def oracle_state(pr, idx=None):
    s = dict(u=pr.u, p=pr.p, x=pr.x, F=pr.F, vol=pr.V, sig=pr.sig, lp=pr.lp, v=pr.v, a=pr.a, pd=pr.pd,
             pdd=pr.pdd)
    return s if idx is None else {k: v[idx] for k, v in s.items()}
