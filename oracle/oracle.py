"""CPU oracle for the stabilized implicit MPM of Zhao & Choo (arXiv 1905.00671).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the CPU-baseline
leg of the benchmark, never by the product library.  It shares no code with the HIP path.

Plain FP64, single-threaded.  The particle loops (basis, constitutive law, residual, exact
Jacobian, P2G, G2P) are in ``oracle.c``; this module drives one time step in the order of the
four MPM stages of Sec. 3.1 and solves each Newton system with a sparse direct solve (SciPy's
SuperLU) instead of a Krylov method:

  Stage 1  lumped P2G of mass, pressure (and, dynamic, v, a, pdot, pddot)  eq. map-from-particles-to-nodes
  Stage 2  Newton on [U, P] (Sec. 3.4): R and exact J at the material points, Dirichlet and
           inactive degrees of freedom removed, solve J d = -R, stop on eq. newton-tolerance
  Stage 3  G2P update (Sec. 3.5)
  Stage 4  convection / GIMP domain update (Sec. 3.5)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import time
from typing import Dict, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nc", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("x0", ctypes.c_double * 3)]


class _Mat(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("lam", ctypes.c_double), ("G", ctypes.c_double),
                ("kappa", ctypes.c_double), ("rho_f", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("phi0", ctypes.c_double), ("alpha_vis", ctypes.c_double)]


class _Opt(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int), ("dynamic", ctypes.c_int), ("beta", ctypes.c_double),
                ("gamma", ctypes.c_double), ("dt", ctypes.c_double), ("tau", ctypes.c_double)]


class _Nodal(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("U", "P", "Pn", "pdn", "pddn", "vn", "an", "Ve", "qe")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d, i, l, vp = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        _lib.or_basis.restype = i
        _lib.or_basis.argtypes = [vp, i, vp, vp, vp, vp, vp, vp]
        _lib.or_kirchhoff.argtypes = [i, d, d, i, vp, vp]
        _lib.or_dkirchhoff.argtypes = [i, d, d, i, vp, vp, vp]
        _lib.or_p2g.argtypes = [vp, i, l] + [vp] * 14
        _lib.or_cell_proj.argtypes = [vp, l, vp, vp, vp, vp]
        _lib.or_particle.restype = i
        _lib.or_particle.argtypes = [vp, vp, vp, vp, vp, vp, d, d, i, vp, vp, vp, vp]
        _lib.or_mobility.argtypes = [d, d, d, vp, vp]
        _lib.or_viscous_stress.argtypes = [vp, i, vp, vp]
        _lib.or_assemble.restype = l
        _lib.or_assemble.argtypes = [vp, vp, vp, l, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, l, vp, vp]
        _lib.or_g2p.restype = l
        _lib.or_mass_matrix.restype = l
        _lib.or_mass_matrix.argtypes = [vp, i, l] + [vp] * 6
        _lib.or_surface_force.argtypes = [vp, i, l] + [vp] * 5
        _lib.or_g2p.argtypes = [vp, vp, vp, l] + [vp] * 13
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _a(s) -> int:
    return ctypes.addressof(s)


def lame(E: float, nu: float):
    """Lame parameters from Young's modulus and Poisson's ratio."""
    return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def mobility(kappa0: float, phi0: float, J: float):
    """Kozeny-Carman mobility at volume ratio J (Sec. 2.2, eq. kozeny-carman) and its derivative
    d kappa / d J, from ``or_mobility``; phi0 <= 0 gives the constant kappa0."""
    k, dk = ctypes.c_double(), ctypes.c_double()
    lib().or_mobility(float(kappa0), float(phi0), float(J), ctypes.byref(k), ctypes.byref(dk))
    return k.value, dk.value


def stab_parameter(kind: int, scale: float, E: float, nu: float, kappa: float, h: float,
                   dt: float, beta: float, gamma: float) -> float:
    """Stabilization parameter of Sec. 4.3: tau_W = 1/(2G) (eq. tau-white), tau_S (eq. tau-sun,
    clamped at zero), tau_M (eq. tau-monforte); kind 0 switches the PPP term off."""
    lam, G = lame(E, nu)
    if kind == 0:
        return 0.0
    if kind == 1:
        return scale / (2.0 * G)
    M = lam + 2.0 * G              # K + 4/3 G
    cv = M * kappa
    c = cv * dt / (h * h)
    if kind == 2:
        return scale * max(0.0, (1.0 / M) * (1.0 - 3.0 * c) * (1.0 + math.tanh(2.0 - 12.0 * c)))
    if kind == 3:
        # 2 kappa / c_v = 2 / M (c_v = M kappa), which also holds in the limit kappa -> 0
        return scale * max(2.0 / M - (beta / gamma) * 12.0 * kappa * dt / (h * h), 0.0)
    raise ValueError(kind)


class NewtonFailure(RuntimeError):
    pass


class OracleProblem:
    """One MPM problem: fixed grid, material, options and the material-point state."""

    def __init__(self, grid, material, options, particles):
        self.grid, self.mat, self.opt = grid, material, options
        d = grid.dim
        if material.model == 0 and d == 3:
            raise ValueError("the Hencky reference is plane strain only")
        n = particles.n
        self.np = n
        self.x = np.array(particles.x, np.float64).reshape(n, d).copy()
        self.V = np.array(particles.vol, np.float64).copy()
        self.m = np.array(particles.mass, np.float64).copy()
        self.lp = np.array(particles.lp, np.float64).reshape(n, d).copy()
        self.lp0 = self.lp.copy()
        self.F = np.tile(np.eye(d), (n, 1, 1))
        self.p = np.zeros(n) if particles.p0 is None else np.array(particles.p0, np.float64).copy()
        self.u = np.zeros((n, d))
        self.v = np.zeros((n, d)) if particles.v0 is None else np.array(particles.v0, np.float64).reshape(n, d).copy()
        self.a = np.zeros((n, d))
        self.pd = np.zeros(n)
        self.pdd = np.zeros(n)
        self.sig = np.zeros((n, 3, 3))
        lam, G = lame(material.E, material.nu)
        self.lam, self.G = lam, G
        self.kappa = material.k / material.mu_f
        self._g = _Grid(d, (ctypes.c_int * 3)(*(list(grid.ncell) + [1] * (3 - d))[:3]), grid.h,
                        (ctypes.c_double * 3)(*(list(grid.origin) + [0.0] * 3)[:3]))
        gv = list(material.g) + [0.0] * 3
        # initial porosity of the Kozeny-Carman law when the material asks for it, else 0
        kc = material.phi0 if getattr(material, "kozeny_carman", False) else 0.0
        self._m = _Mat(material.model, lam, G, self.kappa, material.rho_f,
                       (ctypes.c_double * 3)(*gv[:3]), kc, float(getattr(material, "alpha_vis", 0.0)))
        self.history = []
        self.rtol = options.newton_rtol
        self.newton_max = options.newton_max

    # ------------------------------------------------------------------------------------------
    def _opt(self, dt: float) -> _Opt:
        o = self.opt
        tau = stab_parameter(o.tau_kind, o.tau_scale, self.mat.E, self.mat.nu, self.kappa,
                             self.grid.h, dt, o.beta, o.gamma)
        return _Opt(o.shape, o.dynamic, o.beta, o.gamma, dt, tau)

    def _nodal_struct(self, nod):
        keep = {k: np.ascontiguousarray(v) for k, v in nod.items()}
        s = _Nodal(*[_p(keep.get(n)) for n in ("U", "P", "Pn", "pdn", "pddn", "vn", "an", "Ve", "qe")])
        return s, keep

    def p2g(self) -> Dict[str, np.ndarray]:
        """Stage 1: eq. map-from-particles-to-nodes (lumped mass), or, with the consistent_mass
        option, eq. map-from-particles-to-nodes-consistent (solve M f = sum S m f_mp with the
        consistent mass matrix over the active nodes) for every mapped field."""
        g, d = self.grid, self.grid.dim
        nn = g.nnode
        M = np.zeros(nn)
        Mp = np.zeros(nn)
        dyn = self.opt.dynamic
        Mv = np.zeros(nn * d) if dyn else None
        Ma = np.zeros(nn * d) if dyn else None
        Mpd = np.zeros(nn) if dyn else None
        Mpdd = np.zeros(nn) if dyn else None
        lib().or_p2g(_a(self._g), self.opt.shape, self.np, _p(self.x), _p(self.lp), _p(self.m),
                     _p(self.p), _p(self.v) if dyn else None, _p(self.a) if dyn else None,
                     _p(self.pd) if dyn else None, _p(self.pdd) if dyn else None,
                     _p(M), _p(Mp), _p(Mv), _p(Ma), _p(Mpd), _p(Mpdd))
        # a node whose mass is a negligible fraction of the largest (a point domain that only just
        # reaches its support) is inactive: its rows would otherwise be ~1e-18 of the others and
        # the Newton update there unbounded (reading: below NEGLIGIBLE_MASS of the step's largest
        # nodal mass, or the option negligible_mass when it is positive, the node is treated as
        # outside the material)
        cut = getattr(self.opt, "negligible_mass", 0.0)
        act = M > (cut if cut > 0 else self.NEGLIGIBLE_MASS) * M.max()
        M = np.where(act, M, 0.0)
        safe = np.where(act, M, 1.0)
        out = dict(M=M, active=act, Pn=np.where(act, Mp / safe, 0.0))
        if dyn:
            out["vn"] = np.where(act[:, None], Mv.reshape(nn, d) / safe[:, None], 0.0).reshape(-1)
            out["an"] = np.where(act[:, None], Ma.reshape(nn, d) / safe[:, None], 0.0).reshape(-1)
            out["pdn"] = np.where(act, Mpd / safe, 0.0)
            out["pddn"] = np.where(act, Mpdd / safe, 0.0)
        if getattr(self.opt, "consistent_mass", 0):
            cols = {"Pn": Mp}
            if dyn:
                cols.update(vn=Mv, an=Ma, pdn=Mpd, pddn=Mpdd)
            for k, f in self.consistent_map(M, cols).items():
                out[k] = f
        if self.opt.shape == 0:
            nc = g.ncells
            Ve = np.zeros(nc)
            qe = np.zeros(nc * (1 << d))
            lib().or_cell_proj(_a(self._g), self.np, _p(self.x), _p(self.V), _p(Ve), _p(qe))
            out["Ve"], out["qe"] = Ve, qe
        return out

    def mass_matrix(self):
        """Consistent mass matrix M_ij = sum_mp S_i S_j m (eq. map-from-particles-to-nodes-consistent), CSR."""
        g, d = self.grid, self.grid.dim
        nb = 4 ** d if self.opt.shape == 1 else 2 ** d
        cap = self.np * nb * nb
        ri = np.empty(cap, np.int64)
        ci = np.empty(cap, np.int64)
        v = np.empty(cap)
        n = lib().or_mass_matrix(_a(self._g), self.opt.shape, self.np, _p(self.x), _p(self.lp), _p(self.m),
                                 _p(ri), _p(ci), _p(v))
        return sp.coo_matrix((v[:n], (ri[:n], ci[:n])), shape=(g.nnode, g.nnode)).tocsr()

    NEGLIGIBLE_MASS = 1e-15

    # Nodes whose lumped mass is below this fraction of the step's largest nodal mass keep the
    # lumped value in the consistent mapping (reading: the consistent mass matrix is singular in
    # the limit of nodes that a point domain barely reaches).
    LIGHT_NODE = 1e-2

    def consistent_map(self, mass, sums):
        """Nodal fields f of eq. map-from-particles-to-nodes-consistent from their right-hand sides
        b = sum_mp S_i m f_mp (dict of flat arrays, vector fields node-major).  Nodes with lumped
        mass M_i >= LIGHT_NODE max M ("heavy") solve sum_j M_ij f_j = b_i, the other active nodes
        ("light") keep the lumped value b_i / M_i and enter the heavy rows as known values
        (M_HH f_H = b_H - M_HL f_L, sparse direct, one factorization); inactive nodes get 0."""
        nn = self.grid.nnode
        act = mass > 0
        heavy = act & (mass >= self.LIGHT_NODE * mass.max())
        light = act & ~heavy
        H, L = np.flatnonzero(heavy), np.flatnonzero(light)
        Mall = self.mass_matrix()
        lu = spla.splu(Mall[H][:, H].tocsc())
        MHL = Mall[H][:, L]
        safe = np.where(act, mass, 1.0)
        out = {}
        for k, b in sums.items():
            nc = b.size // nn
            B = b.reshape(nn, nc)
            X = np.where(act[:, None], B / safe[:, None], 0.0)       # lumped values
            for c in range(nc):
                X[H, c] = lu.solve(np.ascontiguousarray(B[H, c] - MHL @ X[L, c]))
            out[k] = X.reshape(-1) if nc > 1 else X[:, 0].copy()
        return out

    def surface_force(self, F, nrm=None):
        """Nodal forces [nnode*dim] of the tractions carried by the points (or_surface_force)."""
        g, d = self.grid, self.grid.dim
        F = np.ascontiguousarray(F, np.float64).reshape(self.np, d)
        nr = None if nrm is None else np.ascontiguousarray(nrm, np.float64).reshape(self.np, d)
        out = np.zeros(g.nnode * d)
        lib().or_surface_force(_a(self._g), self.opt.shape, self.np, _p(self.x), _p(self.lp), _p(F), _p(nr),
                               _p(out))
        return out

    def assemble(self, U, P, nodal, dt, want_J=True, vin=None):
        """Residual (and Jacobian as CSR, and/or J vin) at the nodal state (U, P)."""
        g, d = self.grid, self.grid.dim
        ndof = g.nnode * (d + 1)
        nod = dict(U=np.ascontiguousarray(U, np.float64).reshape(-1), P=np.ascontiguousarray(P, np.float64),
                   Pn=nodal["Pn"])
        for k in ("pdn", "pddn", "vn", "an", "Ve", "qe"):
            if k in nodal:
                nod[k] = nodal[k]
        s, keep = self._nodal_struct(nod)
        opt = self._opt(dt)
        R = np.zeros(ndof)
        Jv = np.zeros(ndof) if vin is not None else None
        vin_c = np.ascontiguousarray(vin, np.float64) if vin is not None else None
        nn = 4 ** d if self.opt.shape == 1 else 2 ** d
        cap = self.np * (nn * (d + 1)) ** 2 if want_J else 0
        ci = np.empty(cap, np.int64) if want_J else None
        cj = np.empty(cap, np.int64) if want_J else None
        cv = np.empty(cap, np.float64) if want_J else None
        Fflat = np.ascontiguousarray(self.F.reshape(-1))
        cnt = lib().or_assemble(_a(self._g), _a(self._m), _a(opt), self.np,
                                _p(self.x), _p(self.lp), _p(Fflat), _p(self.V), _p(self.m), _a(s),
                                _p(R), _p(ci), _p(cj), _p(cv), cap, _p(vin_c), _p(Jv))
        if cnt < 0:
            raise NewtonFailure(f"inverted material point {-1 - cnt}")
        J = None
        if want_J:
            J = sp.coo_matrix((cv[:cnt], (ci[:cnt], cj[:cnt])), shape=(ndof, ndof)).tocsr()
        return R, J, Jv

    # ------------------------------------------------------------------------------------------
    def step(self, dt: float, bc: Dict[str, np.ndarray], rtol: Optional[float] = None,
             newton_max: Optional[int] = None) -> Dict:
        """One implicit time step (Stages 1-4).  The particle state is updated only when Newton
        converges; otherwise NewtonFailure is raised and the state is left unchanged."""
        rtol = self.rtol if rtol is None else rtol
        nmax = self.newton_max if newton_max is None else newton_max
        g, d = self.grid, self.grid.dim
        nn = g.nnode
        t0 = time.perf_counter()
        nodal = self.p2g()
        act = nodal["active"]
        ufix = bc["u_fixed"].astype(bool).reshape(nn, d)
        pfix = bc["p_fixed"].astype(bool).reshape(nn)
        p_val = np.asarray(bc["p_val"], np.float64).reshape(nn)
        if getattr(self.opt, "drained_surface", 0):
            surf = free_surface_nodes(g, act)
            pfix = pfix | surf
            p_val = np.where(surf, 0.0, p_val)
        if bc.get("point_p_fixed") is not None:
            # pressure conditions carried by material points (Sec. 5.4, reading: every grid node
            # in the basis of a flagged point holds the point's value)
            pfix = pfix.copy()
            p_val = p_val.copy()
            val = bc.get("point_p_val")
            for q in np.flatnonzero(np.asarray(bc["point_p_fixed"]).astype(bool)):
                nodes, S, _, _ = basis(g, self.opt.shape, self.x[q], self.lp[q])
                nodes = nodes[S > 0.0]
                pfix[nodes] = True
                p_val[nodes] = 0.0 if val is None else float(val[q])
        if self.opt.dynamic:
            # constrained components of the nodal kinematics start from rest
            for k in ("vn", "an"):
                v = nodal[k].reshape(nn, d)
                v[ufix] = 0.0
                nodal[k] = v.reshape(-1)
        fixed = np.zeros((nn, d + 1), bool)
        fixed[:, :d] = ufix
        fixed[:, d] = pfix
        free = (~fixed) & act[:, None]
        free_f = free.reshape(-1)
        U = np.where(ufix, bc["u_inc"].reshape(nn, d), 0.0) * act[:, None]
        P = np.where(pfix, p_val, nodal["Pn"]) * act
        fext = np.zeros((nn, d + 1))
        fext[:, :d] = bc["f_ext"].reshape(nn, d)
        if bc.get("point_force") is not None:
            fext[:, :d] += self.surface_force(bc["point_force"], bc.get("point_normal")).reshape(nn, d)
        fext[:, d] = -bc["q_ext"]
        fext = fext.reshape(-1)
        scale_u = self.mat.E * g.h ** (d - 1)
        scale_p = g.h ** d / dt
        atol_u = self.opt.newton_atol_u if self.opt.newton_atol_u > 0 else 1e-12 * scale_u
        atol_p = self.opt.newton_atol_p if self.opt.newton_atol_p > 0 else 1e-12 * scale_p
        hist = []
        t_asm = t_sol = 0.0
        umask = np.zeros((nn, d + 1), bool)
        umask[:, :d] = True
        umask = umask.reshape(-1)
        converged = False
        for it in range(nmax + 1):
            ta = time.perf_counter()
            R, J, _ = self.assemble(U, P, nodal, dt, want_J=True)
            t_asm += time.perf_counter() - ta
            R = R + fext
            R[~free_f] = 0.0
            ru = float(np.linalg.norm(R[umask]))
            rp = float(np.linalg.norm(R[~umask]))
            if it == 0:
                ru0, rp0 = ru, rp
            hist.append((ru, rp, math.hypot(ru, rp)))
            if ru <= max(rtol * ru0, atol_u) and rp <= max(rtol * rp0, atol_p):
                converged = True
                break
            if it == nmax:
                break
            ts = time.perf_counter()
            idx = np.nonzero(free_f)[0]
            Jf = J[idx][:, idx].tocsc()
            delta = spla.splu(Jf).solve(-R[idx])
            t_sol += time.perf_counter() - ts
            dfull = np.zeros(nn * (d + 1))
            dfull[idx] = delta
            dfull = dfull.reshape(nn, d + 1)
            U = U + dfull[:, :d]
            P = P + dfull[:, d]
        if not converged:
            raise NewtonFailure(f"Newton did not converge in {nmax} iterations: {hist[-1]}")
        tg = time.perf_counter()
        self.g2p(U, P, nodal, dt)
        t_g2p = time.perf_counter() - tg
        stats = dict(newton_iters=len(hist) - 1, res_hist=hist, t_assemble=t_asm, t_solve=t_sol,
                     t_g2p=t_g2p, t_step=time.perf_counter() - t0, U=U, P=P, nodal=nodal)
        self.history.append(stats)
        return stats

    def g2p(self, U, P, nodal, dt):
        """Stages 3-4 (Sec. 3.5)."""
        g, d = self.grid, self.grid.dim
        nod = dict(U=np.ascontiguousarray(U, np.float64).reshape(-1), P=np.ascontiguousarray(P, np.float64),
                   Pn=nodal["Pn"])
        for k in ("pdn", "pddn", "vn", "an"):
            if k in nodal:
                nod[k] = nodal[k]
        s, keep = self._nodal_struct(nod)
        opt = self._opt(dt)
        x = self.x.copy(); lp = self.lp.copy(); F = self.F.reshape(-1).copy(); V = self.V.copy()
        p = self.p.copy(); u = self.u.copy(); v = self.v.copy(); a = self.a.copy()
        pd = self.pd.copy(); pdd = self.pdd.copy(); sig = np.zeros(self.np * 9)
        rc = lib().or_g2p(_a(self._g), _a(self._m), _a(opt), self.np,
                          _p(x), _p(lp), _p(self.lp0), _p(F), _p(V), _p(p), _p(u), _p(v), _p(a), _p(pd),
                          _p(pdd), _p(sig), _a(s))
        if rc < 0:
            raise NewtonFailure(f"inverted material point {-1 - rc} in the update")
        self.x, self.lp, self.F, self.V = x, lp, F.reshape(self.np, d, d), V
        self.p, self.u, self.v, self.a, self.pd, self.pdd = p, u, v, a, pd, pdd
        self.sig = sig.reshape(self.np, 3, 3)


def free_surface_nodes(grid, active):
    """Nodes on the current free surface of the material: active nodes with an inactive node among
    their 3^d - 1 neighbours inside the grid (the edges of the grid are supports or symmetry
    planes, not free surfaces).  A drained free surface (zero pore pressure) is imposed there."""
    d = grid.dim
    shape = tuple(reversed(grid.nnode_axis))          # natural order: x fastest
    act = np.asarray(active, bool).reshape(shape)
    inact = ~act
    near = np.zeros_like(act)
    offs = [(dz, dy, dx) for dz in ((-1, 0, 1) if d == 3 else (0,)) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    for off in offs:
        if not any(off):
            continue
        if d == 2:
            off = off[1:]
        # near[j] |= inact[j + off] wherever both lie inside the grid
        dst = [slice(max(0, -o), n - max(0, o)) for o, n in zip(off, shape)]
        src = [slice(max(0, o), n - max(0, -o)) for o, n in zip(off, shape)]
        near[tuple(dst)] |= inact[tuple(src)]
    return (act & near).reshape(-1)


def from_workload(w) -> OracleProblem:
    return OracleProblem(w.grid, w.material, w.options, w.particles)


# ---- thin wrappers used by the pins ------------------------------------------------------------

def basis(grid, shape, xp, lp=None):
    g = _Grid(grid.dim, (ctypes.c_int * 3)(*(list(grid.ncell) + [1] * 3)[:3]), grid.h,
              (ctypes.c_double * 3)(*(list(grid.origin) + [0.0] * 3)[:3]))
    xp = np.ascontiguousarray(xp, np.float64)
    lp = np.ascontiguousarray(lp if lp is not None else np.zeros(grid.dim), np.float64)
    nodes = np.zeros(64, np.int32)
    S = np.zeros(64); G = np.zeros(64 * 3); S0 = np.zeros(64)
    n = lib().or_basis(_a(g), shape, _p(xp), _p(lp), _p(nodes), _p(S), _p(G), _p(S0))
    return nodes[:n].copy(), S[:n].copy(), G[: n * grid.dim].reshape(n, grid.dim).copy(), S0[:n].copy()


def viscous_stress(lam, G, alpha_vis, L):
    """Kelvin-type viscous stress of ``or_viscous_stress`` for the velocity gradient L (d x d)."""
    L = np.ascontiguousarray(L, np.float64)
    d = L.shape[0]
    m = _Mat(1, lam, G, 0.0, 0.0, (ctypes.c_double * 3)(0.0, 0.0, 0.0), 0.0, alpha_vis)
    out = np.zeros(d * d)
    lib().or_viscous_stress(_a(m), d, _p(L), _p(out))
    return out.reshape(d, d)


def kirchhoff(model, lam, G, F):
    F = np.ascontiguousarray(F, np.float64)
    d = F.shape[0]
    tau = np.zeros(9)
    lib().or_kirchhoff(model, lam, G, d, _p(F), _p(tau))
    return tau.reshape(3, 3)


def dkirchhoff(model, lam, G, F, L):
    F = np.ascontiguousarray(F, np.float64)
    L = np.ascontiguousarray(L, np.float64)
    d = F.shape[0]
    out = np.zeros(9)
    lib().or_dkirchhoff(model, lam, G, d, _p(F), _p(L), _p(out))
    return out.reshape(3, 3)
