"""ctypes binding of libppmpm.so (the C ABI declared in include/ppmpm.h).

Argument marshalling only: every step of the method runs in the HIP library.  PyTorch supplies
device memory (the caller-owned workspace is a torch uint8 tensor) and the HIP stream.  There is
no fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppmpm.so")
MAX_HIST = 64

OK, E_INVALID, E_OOM, E_DEVICE, E_NEWTON, E_KRYLOV, E_NONFINITE, E_OUT_OF_GRID = range(8)
HOST, DEVICE = 0, 1
FP64, MIXED = 0, 1
FIELDS = {"x": 0, "u": 1, "p": 2, "F": 3, "vol": 4, "sig": 5, "v": 6, "a": 7, "pd": 8, "pdd": 9, "lp": 10}


class PPMPMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ppmpm status {status}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("ncell", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("origin", ctypes.c_double * 3)]


class Material(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("E", ctypes.c_double), ("nu", ctypes.c_double),
                ("k", ctypes.c_double), ("mu_f", ctypes.c_double), ("rho_f", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("phi0", ctypes.c_double), ("alpha_vis", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int), ("dynamic", ctypes.c_int), ("beta", ctypes.c_double),
                ("gamma", ctypes.c_double), ("tau_kind", ctypes.c_int), ("tau_scale", ctypes.c_double),
                ("precision", ctypes.c_int), ("newton_rtol", ctypes.c_double),
                ("newton_atol_u", ctypes.c_double), ("newton_atol_p", ctypes.c_double),
                ("newton_max", ctypes.c_int), ("krylov_rtol", ctypes.c_double),
                ("krylov_max", ctypes.c_int), ("krylov_check", ctypes.c_int), ("mg_smooth", ctypes.c_int),
                ("drained_surface", ctypes.c_int), ("consistent_mass", ctypes.c_int),
                ("negligible_mass", ctypes.c_double), ("schur", ctypes.c_int)]


class BC(ctypes.Structure):
    _fields_ = [("u_fixed", ctypes.c_void_p), ("u_inc", ctypes.c_void_p), ("p_fixed", ctypes.c_void_p),
                ("p_val", ctypes.c_void_p), ("f_ext", ctypes.c_void_p), ("q_ext", ctypes.c_void_p),
                ("where", ctypes.c_int), ("point_force", ctypes.c_void_p), ("point_normal", ctypes.c_void_p),
                ("point_p_fixed", ctypes.c_void_p), ("point_p_val", ctypes.c_void_p)]


class StepStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("newton_iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("krylov_total", ctypes.c_int), ("krylov_iters", ctypes.c_int * MAX_HIST),
                ("res_u", ctypes.c_double * MAX_HIST), ("res_p", ctypes.c_double * MAX_HIST),
                ("t_sort", ctypes.c_double), ("t_assemble", ctypes.c_double), ("t_precond", ctypes.c_double),
                ("t_krylov", ctypes.c_double), ("t_g2p", ctypes.c_double), ("t_total", ctypes.c_double),
                ("krylov_breakdowns", ctypes.c_int), ("ngrid_levels", ctypes.c_int), ("mass_iters", ctypes.c_int)]

    def as_dict(self) -> Dict:
        n = self.newton_iters
        return dict(status=self.status, newton_iters=n, converged=self.converged, krylov_total=self.krylov_total,
                    krylov_iters=list(self.krylov_iters[:n]), res_u=list(self.res_u[: n + 1]),
                    res_p=list(self.res_p[: n + 1]), t_sort=self.t_sort, t_assemble=self.t_assemble,
                    t_precond=self.t_precond, t_krylov=self.t_krylov, t_g2p=self.t_g2p, t_total=self.t_total,
                    krylov_breakdowns=self.krylov_breakdowns, ngrid_levels=self.ngrid_levels,
                    mass_iters=self.mass_iters)


_lib = None


def lib() -> ctypes.CDLL:
    """Loads the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1905_00671_amd/build.py")
        # torch ships its own HIP and HSA runtimes under the same sonames as /opt/rocm's; loading
        # torch first makes the library bind to those instead of starting a second runtime in the
        # process (which would find no device)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.ppmpm_workspace_bytes.restype = ctypes.c_size_t
        L.ppmpm_workspace_bytes.argtypes = [vp, i64, vp]
        L.ppmpm_create.restype = i32
        L.ppmpm_create.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp, i64, ctypes.POINTER(vp)]
        L.ppmpm_set_particles.restype = i32
        L.ppmpm_set_particles.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, i32]
        L.ppmpm_step.restype = i32
        L.ppmpm_step.argtypes = [vp, dbl, vp, vp]
        L.ppmpm_step_batched.restype = i32
        L.ppmpm_step_batched.argtypes = [vp, i32, vp, vp, vp]
        L.ppmpm_get_field.restype = i32
        L.ppmpm_get_field.argtypes = [vp, i32, vp, i32]
        L.ppmpm_state_bytes.restype = i32
        L.ppmpm_state_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.ppmpm_save_state.restype = i32
        L.ppmpm_save_state.argtypes = [vp, vp, ctypes.c_size_t, i32]
        L.ppmpm_load_state.restype = i32
        L.ppmpm_load_state.argtypes = [vp, vp, ctypes.c_size_t, i32]
        L.ppmpm_eval_residual.restype = i32
        L.ppmpm_eval_residual.argtypes = [vp, dbl, vp, vp, vp, vp, i32]
        L.ppmpm_apply_jacobian.restype = i32
        L.ppmpm_apply_jacobian.argtypes = [vp, vp, vp, i32]
        L.ppmpm_get_nodal.restype = i32
        L.ppmpm_get_nodal.argtypes = [vp, i32, vp, i32]
        L.ppmpm_destroy.restype = i32
        L.ppmpm_destroy.argtypes = [vp]
        L.ppmpm_last_error.restype = ctypes.c_char_p
        L.ppmpm_last_error.argtypes = []
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise PPMPMError(status, lib().ppmpm_last_error().decode())


def _ptr(a) -> Optional[int]:
    """Data pointer of a numpy array (host) or a torch tensor (device or host)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _where(a) -> int:
    if isinstance(a, np.ndarray):
        return HOST
    return DEVICE if a.is_cuda else HOST


def make_grid(g) -> Grid:
    nc = list(g.ncell[: g.dim]) + [1] * (3 - g.dim)
    org = list(g.origin[: g.dim]) + [0.0] * (3 - g.dim)
    return Grid(g.dim, (ctypes.c_int * 3)(*nc), g.h, (ctypes.c_double * 3)(*org))


def make_material(m) -> Material:
    gv = list(m.g) + [0.0] * 3
    kc = m.phi0 if getattr(m, "kozeny_carman", False) else 0.0
    return Material(m.model, m.E, m.nu, m.k, m.mu_f, m.rho_f, (ctypes.c_double * 3)(*gv[:3]), kc,
                    float(getattr(m, "alpha_vis", 0.0)))


def make_options(o, precision: int = FP64, **over) -> Options:
    vals = dict(shape=o.shape, dynamic=o.dynamic, beta=o.beta, gamma=o.gamma, tau_kind=o.tau_kind,
                tau_scale=o.tau_scale, precision=precision, newton_rtol=o.newton_rtol,
                newton_atol_u=getattr(o, "newton_atol_u", 0.0), newton_atol_p=getattr(o, "newton_atol_p", 0.0),
                newton_max=o.newton_max, krylov_rtol=o.krylov_rtol, krylov_max=o.krylov_max,
                krylov_check=4, mg_smooth=1, drained_surface=int(getattr(o, "drained_surface", 0)),
                consistent_mass=int(getattr(o, "consistent_mass", 0)),
                negligible_mass=float(getattr(o, "negligible_mass", 0.0)),
                schur=int(getattr(o, "schur", 0)))
    vals.update(over)
    return Options(**vals)


BC_KEYS = ("u_fixed", "u_inc", "p_fixed", "p_val", "f_ext", "q_ext", "point_force", "point_normal", "point_p_fixed",
           "point_p_val")


class BCArrays:
    """Keeps the arrays of one step's boundary data alive and exposes the C struct."""

    def __init__(self, d: Dict):
        self.keep = {}
        for k in BC_KEYS:
            v = d.get(k)
            if v is not None and isinstance(v, np.ndarray):
                dt = np.uint8 if k in ("u_fixed", "p_fixed", "point_p_fixed") else np.float64
                v = np.ascontiguousarray(v, dtype=dt)
            self.keep[k] = v
        first = next((v for v in self.keep.values() if v is not None), None)
        where = HOST if first is None else _where(first)
        ptr = {k: _ptr(self.keep[k]) for k in BC_KEYS}
        self.c = BC(*[ptr[k] for k in BC_KEYS[:6]], where, *[ptr[k] for k in BC_KEYS[6:]])


class Problem:
    """One MPM problem living in a torch-allocated workspace on the current GPU."""

    def __init__(self, grid, material, options, np_count: int, precision: int = FP64, stream=None, **over):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("ppmpm needs a HIP device; none is visible")
        self.L = lib()
        self.grid, self.material, self.options = grid, material, options
        self.dim = grid.dim
        self.np = int(np_count)
        self._g = make_grid(grid)
        self._m = make_material(material)
        self._o = make_options(options, precision, **over)
        nbytes = self.L.ppmpm_workspace_bytes(ctypes.byref(self._g), self.np, ctypes.byref(self._o))
        if nbytes == 0:
            _check(E_INVALID)
        self.workspace_bytes = int(nbytes)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        # 256-byte aligned view into a torch allocation
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        self._base = (base + 255) & ~255
        h = ctypes.c_void_p()
        _check(self.L.ppmpm_create(ctypes.byref(self._g), ctypes.byref(self._m), ctypes.byref(self._o),
                                   ctypes.c_void_p(self._base), nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                   self.np, ctypes.byref(h)))
        self.h = h

    @classmethod
    def from_workload(cls, w, precision: int = FP64, **over) -> "Problem":
        p = cls(w.grid, w.material, w.options, w.particles.n, precision=precision, **over)
        p.set_particles(w.particles)
        return p

    def set_particles(self, parts):
        x = np.ascontiguousarray(parts.x, np.float64)
        vol = np.ascontiguousarray(parts.vol, np.float64)
        mass = np.ascontiguousarray(parts.mass, np.float64)
        lp = np.ascontiguousarray(parts.lp, np.float64) if parts.lp is not None else None
        v0 = np.ascontiguousarray(parts.v0, np.float64) if parts.v0 is not None else None
        p0 = np.ascontiguousarray(parts.p0, np.float64) if parts.p0 is not None else None
        _check(self.L.ppmpm_set_particles(self.h, self.np, _ptr(x), _ptr(vol), _ptr(mass), _ptr(lp), _ptr(v0),
                                          _ptr(p0), HOST))

    def step(self, dt: float, bc: Dict, raise_on_error: bool = True) -> Dict:
        b = BCArrays(bc)
        st = StepStats()
        s = self.L.ppmpm_step(self.h, float(dt), ctypes.byref(b.c), ctypes.byref(st))
        if raise_on_error:
            _check(s)
        return st.as_dict()

    def save_state(self) -> np.ndarray:
        """Checkpoint of the committed material-point state (ppmpm_save_state) as host bytes."""
        n = ctypes.c_size_t()
        _check(self.L.ppmpm_state_bytes(self.h, ctypes.byref(n)))
        buf = np.zeros(n.value, np.uint8)
        _check(self.L.ppmpm_save_state(self.h, buf.ctypes.data_as(ctypes.c_void_p), n.value, HOST))
        return buf

    def load_state(self, buf: np.ndarray) -> None:
        """Restores a checkpoint written by save_state (ppmpm_load_state)."""
        buf = np.ascontiguousarray(buf, np.uint8)
        _check(self.L.ppmpm_load_state(self.h, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes, HOST))

    def get(self, name: str) -> np.ndarray:
        f = FIELDS[name]
        d = self.dim
        ncomp = {0: d, 1: d, 2: 1, 3: d * d, 4: 1, 5: 9, 6: d, 7: d, 8: 1, 9: 1, 10: d}[f]
        out = np.zeros(self.np * ncomp)
        _check(self.L.ppmpm_get_field(self.h, f, _ptr(out), HOST))
        if ncomp == 1:
            return out
        if f == 3:
            return out.reshape(self.np, d, d)
        if f == 5:
            return out.reshape(self.np, 3, 3)
        return out.reshape(self.np, ncomp)

    def eval_residual(self, dt: float, bc: Dict, U: np.ndarray, P: np.ndarray) -> np.ndarray:
        b = BCArrays(bc)
        U = np.ascontiguousarray(U, np.float64)
        P = np.ascontiguousarray(P, np.float64)
        nn = int(np.prod([n + 1 for n in self.grid.ncell[: self.dim]]))
        R = np.zeros(nn * (self.dim + 1))
        _check(self.L.ppmpm_eval_residual(self.h, float(dt), ctypes.byref(b.c), _ptr(U), _ptr(P), _ptr(R), HOST))
        return R

    def apply_jacobian(self, v: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(v, np.float64)
        y = np.zeros_like(v)
        _check(self.L.ppmpm_apply_jacobian(self.h, _ptr(v), _ptr(y), HOST))
        return y

    def get_nodal(self, field: int) -> np.ndarray:
        nn = int(np.prod([n + 1 for n in self.grid.ncell[: self.dim]]))
        out = np.zeros(nn * (self.dim + 1) if field >= 2 else nn)
        _check(self.L.ppmpm_get_nodal(self.h, field, _ptr(out), HOST))
        return out

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.L.ppmpm_destroy(self.h)
            self.h = ctypes.c_void_p()
        self._ws = None      # the workspace goes back to torch's allocator

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_residual_static(w, dt: float, bc: Dict, U: np.ndarray, P: np.ndarray, precision: int = FP64,
                         stream=None) -> np.ndarray:
    """ppmpm_eval_residual_static: the residual of workload w's first step at the nodal state
    (U, P), with the library's own device workspace (no allocation by the call)."""
    import torch
    L = lib()
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.ppmpm_eval_residual_static.restype = i32
    L.ppmpm_eval_residual_static.argtypes = [vp, vp, vp, i64] + [vp] * 6 + [dbl, vp, vp, vp, vp, vp, i32]
    g, m, o = make_grid(w.grid), make_material(w.material), make_options(w.options, precision)
    parts = w.particles
    arr = {k: (np.ascontiguousarray(getattr(parts, k), np.float64) if getattr(parts, k) is not None else None)
           for k in ("x", "vol", "mass", "lp", "v0", "p0")}
    b = BCArrays(bc)
    U = np.ascontiguousarray(U, np.float64)
    P = np.ascontiguousarray(P, np.float64)
    nn = int(np.prod([n + 1 for n in w.grid.ncell[: w.grid.dim]]))
    R = np.zeros(nn * (w.grid.dim + 1))
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(L.ppmpm_eval_residual_static(ctypes.byref(g), ctypes.byref(m), ctypes.byref(o), parts.n,
                                        *[_ptr(arr[k]) for k in ("x", "vol", "mass", "lp", "v0", "p0")],
                                        float(dt), ctypes.byref(b.c), _ptr(U), _ptr(P), _ptr(R),
                                        ctypes.c_void_p(st.cuda_stream), HOST))
    return R


def step_batched(problems: Sequence[Problem], dts: Sequence[float], bcs: Sequence[Dict]) -> List[Dict]:
    """One time step of several problems with one kernel launch per phase (per kernel variant);
    per-problem status in each returned dict."""
    n = len(problems)
    L = lib()
    arr = (ctypes.c_void_p * n)(*[p.h.value for p in problems])
    dt = (ctypes.c_double * n)(*[float(x) for x in dts])
    keep = [BCArrays(b) for b in bcs]
    bptr = (ctypes.c_void_p * n)(*[ctypes.addressof(k.c) for k in keep])
    stats = (StepStats * n)()
    s = L.ppmpm_step_batched(arr, n, dt, bptr, stats)
    if s in (E_DEVICE, E_OOM):
        _check(s)            # a failure of the batch itself, not of one problem
    return [stats[i].as_dict() for i in range(n)]


KERNELS = ["spmv", "jacobian", "records", "residual", "mg0_resid", "p2g", "g2p", "permute", "rap", "cellmat", "mg0_s"]


def timing_enable(on: bool = True):
    L = lib()
    L.ppmpm_timing_enable.restype = ctypes.c_int
    L.ppmpm_timing_enable.argtypes = [ctypes.c_int]
    _check(L.ppmpm_timing_enable(1 if on else 0))


def timing_reset():
    L = lib()
    L.ppmpm_timing_reset.restype = ctypes.c_int
    _check(L.ppmpm_timing_reset())


def timing_get() -> Dict[str, Dict[str, float]]:
    """Launch counts and summed HIP-event durations (ms) of the instrumented kernels."""
    L = lib()
    L.ppmpm_timing_get.restype = ctypes.c_int
    L.ppmpm_timing_get.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    out = {}
    for i, name in enumerate(KERNELS):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(L.ppmpm_timing_get(i, ctypes.byref(n), ctypes.byref(ms)))
        out[name] = dict(launches=int(n.value), total_ms=float(ms.value))
    return out


def header_symbols() -> List[str]:
    """Function names declared in include/ppmpm.h."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "ppmpm.h")
    src = open(hdr).read()
    return sorted(set(re.findall(r"\b(ppmpm_[a-z_]+)\s*\(", src)))
