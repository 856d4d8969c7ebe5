"""ctypes front end of the FP64 CPU oracle (``pd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  It marshals numpy
arrays; every computation happens in the C file, which is a literal, slow
transcription of the paper's definitions (Algorithm 1, the velocity-Verlet
equations, the tangent equation and the implicit flow chart).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pd_oracle.c")
LIB = os.path.join(HERE, "libpd_oracle.so")

BC_FREE, BC_CLAMPED, BC_VELOCITY = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP over nodes)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        i64, i32, dbl, ptr = C.c_int64, C.c_int, C.c_double, C.c_void_p
        L.or_threshold.restype = dbl
        L.or_threshold.argtypes = [dbl]
        L.or_micromodulus.restype = dbl
        L.or_micromodulus.argtypes = [i32, dbl, dbl]
        for name in ("or_nbr_brute", "or_nbr_binned"):
            fn = getattr(L, name)
            fn.restype = i64
            fn.argtypes = [i32, i64, ptr, dbl, ptr, ptr]
        L.or_force.restype = None
        L.or_force.argtypes = [i32, i64, ptr, ptr, ptr, ptr, ptr, dbl, dbl, ptr, ptr, ptr]
        L.or_kinetic.restype = dbl
        L.or_kinetic.argtypes = [i32, i64, ptr, dbl, ptr]
        L.or_potential.restype = dbl
        L.or_potential.argtypes = [i64, ptr, ptr]
        L.or_notch_cut.restype = None
        L.or_notch_cut.argtypes = [i32, i64, ptr, ptr, ptr, i32, ptr, ptr]
        L.or_verlet.restype = None
        L.or_verlet.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, dbl, dbl, ptr, ptr, ptr,
                                i64, dbl, i64, i64, ptr, ptr, ptr, ptr]
        L.or_apply_tangent.restype = None
        L.or_apply_tangent.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, ptr, ptr, ptr, ptr]
        L.or_cg.restype = i32
        L.or_cg.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, ptr, ptr, ptr, ptr, dbl, i32,
                            ptr, ptr]
        L.or_residual.restype = dbl
        L.or_residual.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, ptr, ptr, ptr, ptr, ptr]
        L.or_solve_implicit.restype = i32
        L.or_solve_implicit.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, ptr, ptr, ptr, ptr,
                                        dbl, dbl, i32, i32, ptr, ptr, ptr]
        L.or_force_law.restype = None
        L.or_force_law.argtypes = [i32, i64, ptr, ptr, ptr, ptr, ptr, dbl, dbl, i32, dbl, i32,
                                   ptr, ptr, ptr]
        L.or_tangent_law.restype = None
        L.or_tangent_law.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, i32, dbl, ptr, ptr, ptr,
                                     ptr, ptr]
        L.or_residual_law.restype = dbl
        L.or_residual_law.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, i32, dbl, ptr, ptr,
                                      ptr, ptr, ptr]
        L.or_solve_law.restype = i32
        L.or_solve_law.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, i32, dbl, ptr, ptr, ptr,
                                   ptr, dbl, dbl, i32, i32, ptr, ptr, ptr]
        L.or_verlet_law.restype = None
        L.or_verlet_law.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, dbl, dbl, i32, dbl, i32,
                                    ptr, ptr, ptr, i64, dbl, i64, i64, ptr, ptr, ptr, ptr]
        L.or_lps.restype = None
        L.or_lps.argtypes = [i64, ptr, ptr, ptr, ptr, ptr, dbl, dbl, ptr, ptr, ptr, ptr, ptr]
        L.or_verlet_lps.restype = None
        L.or_verlet_lps.argtypes = [i64, ptr, ptr, ptr, ptr, dbl, dbl, dbl, ptr, ptr, ptr, i64,
                                    dbl, i64, i64, ptr, ptr, ptr, ptr]
        L.or_central_law.restype = None
        L.or_central_law.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, dbl, dbl, i32, dbl, i32,
                                     ptr, ptr, ptr, i64, dbl, i64, i64, ptr, ptr, ptr, ptr]
        L.or_force_law_pv.restype = None
        L.or_force_law_pv.argtypes = [i32, i64, ptr, ptr, ptr, ptr, ptr, dbl, dbl, i32, dbl, i32,
                                      dbl, dbl, ptr, ptr, ptr]
        L.or_lps_pv.restype = None
        L.or_lps_pv.argtypes = [i64, ptr, ptr, ptr, ptr, ptr, dbl, dbl, dbl, dbl, ptr, ptr, ptr,
                                ptr, ptr]
        L.or_verlet_pv.restype = None
        L.or_verlet_pv.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, i32, dbl, dbl, i32, dbl, i32,
                                   dbl, dbl, dbl, dbl, ptr, ptr, ptr, i64, dbl, i64, i64, ptr, ptr,
                                   ptr, ptr]
        L.or_force_law_j.restype = None
        L.or_force_law_j.argtypes = [i32, i64, ptr, ptr, ptr, ptr, ptr, dbl, dbl, i32, dbl, i32,
                                     dbl, dbl, dbl, dbl, dbl, ptr, ptr, ptr]
        for name in ("or_verlet_j", "or_central_j"):
            fn = getattr(L, name)
            fn.restype = None
            fn.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, dbl, dbl, i32, dbl, i32, dbl, dbl,
                           dbl, dbl, dbl, ptr, ptr, ptr, i64, dbl, i64, i64, ptr, ptr, ptr, ptr]
        L.or_band_update.restype = None
        L.or_band_update.argtypes = [i32, i64, ptr, ptr, ptr, ptr, dbl, dbl, dbl, ptr]
        L.or_ccm_bar_1d.restype = None
        L.or_ccm_bar_1d.argtypes = [dbl, dbl, dbl, ptr]
        L.or_ccm_plane_stress.restype = None
        L.or_ccm_plane_stress.argtypes = [i64, ptr, dbl, dbl, dbl, dbl, dbl, ptr]
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [i32]
        L.or_num_threads.restype = i32
        L.or_num_threads.argtypes = []
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def threshold(delta):
    return lib().or_threshold(float(delta))


def ccm_bar_1d(F, A, E):
    """(stress, strain, strain-energy density) of a bar under an end force
    (the classical values of the paper's 1-d implicit validation)."""
    out = np.zeros(3)
    lib().or_ccm_bar_1d(float(F), float(A), float(E), _p(out))
    return float(out[0]), float(out[1]), float(out[2])


def ccm_plane_stress(X, t, E, nu, x0, yc):
    """Classical plane-stress displacement of a plate under a uniform
    traction t along x, held at x = x0 and symmetric about y = yc."""
    X = _f64(X)
    u = np.zeros_like(X)
    lib().or_ccm_plane_stress(X.shape[0], _p(X), float(t), float(E), float(nu), float(x0),
                              float(yc), _p(u))
    return u


def micromodulus(dim, E, delta):
    return lib().or_micromodulus(int(dim), float(E), float(delta))


def neighbors(X, delta, method="binned"):
    """CSR (row_ptr int64[n+1], col int32[nnz]) of B_delta, rows ascending."""
    X = _f64(X)
    n, dim = X.shape
    thr = threshold(delta)
    fn = lib().or_nbr_brute if method == "brute" else lib().or_nbr_binned
    row_ptr = np.zeros(n + 1, np.int64)
    nnz = fn(dim, n, _p(X), thr, _p(row_ptr), None)
    if nnz < 0:
        raise ValueError("coincident nodes")
    col = np.zeros(max(int(nnz), 1), np.int32)
    fn(dim, n, _p(X), thr, _p(row_ptr), _p(col))
    return row_ptr, col[:nnz]


class Mesh:
    """Reference configuration + neighbour list, as the oracle sees it."""

    def __init__(self, X, V, delta, method="binned", row_ptr=None, col=None):
        self.X = _f64(X)
        self.V = _f64(V)
        self.n, self.dim = self.X.shape
        self.delta = float(delta)
        if row_ptr is None:
            row_ptr, col = neighbors(self.X, delta, method)
        self.row_ptr = np.ascontiguousarray(row_ptr, np.int64)
        self.col = np.ascontiguousarray(col, np.int32)

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def all_alive(self):
        return np.ones(max(self.nnz, 1), np.uint8)[: self.nnz]

    def force(self, u, c, s_c=0.0, alive=None, energy=False):
        u = _f64(u)
        f = np.zeros_like(self.X)
        U = np.zeros(self.n) if energy else None
        lib().or_force(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X), _p(self.V),
                       _p(u), float(c), float(s_c), _p(alive), _p(f), _p(U))
        return (f, U) if energy else f

    def potential(self, u, c, alive=None):
        _, U = self.force(u, c, 0.0, alive, energy=True)
        return lib().or_potential(self.n, _p(self.V), _p(U))

    def kinetic(self, v, rho):
        v = _f64(v)
        return lib().or_kinetic(self.dim, self.n, _p(self.V), float(rho), _p(v))

    def notch_cut(self, notch, alive):
        seg = _f64(np.asarray(notch).reshape(-1, 4))
        lib().or_notch_cut(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                           int(seg.shape[0]), _p(seg), _p(alive))
        return alive

    def verlet(self, state, c, rho, s_c, dt, nsteps, bc_kind=None, bc_vel=None, b=None,
               ramp=0):
        """Advance ``state`` (dict u, v, f, alive, step) by nsteps in place."""
        bc_kind = None if bc_kind is None else np.ascontiguousarray(bc_kind, np.uint8)
        bc_vel = None if bc_vel is None else _f64(bc_vel)
        b = None if b is None else _f64(b)
        lib().or_verlet(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                        _p(self.V), float(rho), float(c), float(s_c), _p(bc_kind), _p(bc_vel),
                        _p(b), int(ramp), float(dt), int(state["step"]), int(nsteps),
                        _p(state["u"]), _p(state["v"]), _p(state["f"]), _p(state["alive"]))
        state["step"] += nsteps
        return state

    def band_update(self, band, u, s_c, tol=1e-6, tol_eta=0.0):
        """band |= (|S/s_c - 1| <= tol or |S - s_c| <= tol_eta |eta|/|xi|) per
        bond at displacement u (in place).  The second term covers arithmetic
        whose rounding of S scales with |eta|/|xi| rather than with S (float32
        bond terms)."""
        u = _f64(u)
        lib().or_band_update(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X), _p(u),
                             float(s_c), float(tol), float(tol_eta), _p(band))
        return band

    def verlet_banded(self, state, c, rho, s_c, dt, nsteps, bc_kind=None, bc_vel=None, b=None,
                      ramp=0, band=None, tol=1e-6, tol_eta=0.0):
        """Verlet steps one at a time, collecting in ``band`` (uint8 per bond)
        every bond whose strain came within tol of s_c at a force evaluation
        of these steps (the state on entry included)."""
        if band is None:
            band = np.zeros(max(self.nnz, 1), np.uint8)[: self.nnz]
        self.band_update(band, state["u"], s_c, tol, tol_eta)
        for _ in range(nsteps):
            self.verlet(state, c, rho, s_c, dt, 1, bc_kind, bc_vel, b, ramp)
            self.band_update(band, state["u"], s_c, tol, tol_eta)
        return band

    def start(self, u0, v0, c, s_c=0.0, alive=None):
        """Initial state: f^0 = force(u^0), with the damage test at u^0."""
        alive = self.all_alive() if alive is None else np.ascontiguousarray(alive, np.uint8).copy()
        u = _f64(u0).copy()
        v = _f64(v0).copy()
        f = self.force(u, c, s_c, alive)
        return {"u": u, "v": v, "f": f, "alive": alive, "step": 0}

    def apply_tangent(self, w, c, fixed=None, alive=None):
        w = _f64(w)
        y = np.zeros_like(w)
        fixed = None if fixed is None else np.ascontiguousarray(fixed, np.uint8)
        lib().or_apply_tangent(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                               _p(self.V), float(c), _p(alive), _p(fixed), _p(w), _p(y))
        return y

    def cg(self, rhs, c, fixed=None, alive=None, x0=None, rtol=1e-13, maxit=100000):
        rhs = _f64(rhs)
        x = np.zeros_like(rhs) if x0 is None else _f64(x0).copy()
        fixed = None if fixed is None else np.ascontiguousarray(fixed, np.uint8)
        it = C.c_int(0)
        rel = C.c_double(0)
        st = lib().or_cg(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                         _p(self.V), float(c), _p(alive), _p(fixed), _p(rhs), _p(x),
                         float(rtol), int(maxit), C.byref(it), C.byref(rel))
        return x, {"status": st, "iters": it.value, "relres": rel.value}

    def residual(self, u, c, b, fixed=None, alive=None):
        u = _f64(u)
        r = np.zeros_like(u)
        fixed = None if fixed is None else np.ascontiguousarray(fixed, np.uint8)
        b = None if b is None else _f64(b)
        nrm = lib().or_residual(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                                _p(self.V), float(c), _p(alive), _p(fixed), _p(b), _p(u), _p(r))
        return r, nrm

    def solve_implicit(self, u0, c, b, fixed, alive=None, rtol=1e-10, inner_rtol=1e-13,
                       maxit=200000, max_outer=5):
        u = _f64(u0).copy()
        fixed = np.ascontiguousarray(fixed, np.uint8)
        b = _f64(b)
        o, i, rel = C.c_int(0), C.c_int(0), C.c_double(0)
        st = lib().or_solve_implicit(self.dim, self.n, _p(self.row_ptr), _p(self.col),
                                     _p(self.X), _p(self.V), float(c), _p(alive), _p(fixed),
                                     _p(b), _p(u), float(rtol), float(inner_rtol), int(maxit),
                                     int(max_outer), C.byref(o), C.byref(i), C.byref(rel))
        return u, {"status": st, "outer": o.value, "inner": i.value, "relres": rel.value}


LAW_LINEAR, LAW_NP = 0, 1
STRETCH_LINEARISED, STRETCH_EXACT = 0, 1


class LawMesh(Mesh):
    """The general pairwise law of Algorithm 1: linear or NP potential,
    linearised or exact stretch (``or_force_law`` and friends)."""

    def force_law(self, u, c, law=LAW_NP, beta=1.0, stretch=STRETCH_LINEARISED, s_c=0.0,
                  alive=None, energy=False, pv_h=0.0, j=None):
        """pv_h > 0: partial volumes, the neighbour radius (self.delta) being
        delta + pv_h/2.  j = (c1, c2): the influence function
        J(r) = c1 r exp(-r^2/c2) of r = |xi|/delta on every bond (None: J = 1)."""
        u = _f64(u)
        f = np.zeros_like(self.X)
        U = np.zeros(self.n) if energy else None
        if j is None:
            lib().or_force_law_pv(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                                  _p(self.V), _p(u), float(c), float(s_c), int(law),
                                  float(beta), int(stretch), float(pv_h), self.delta,
                                  _p(alive), _p(f), _p(U))
        else:
            lib().or_force_law_j(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                                 _p(self.V), _p(u), float(c), float(s_c), int(law), float(beta),
                                 int(stretch), float(pv_h), self.delta, float(j[0]),
                                 float(j[1]), self.delta - 0.5 * float(pv_h), _p(alive), _p(f),
                                 _p(U))
        return (f, U) if energy else f

    def energy_law(self, u, c, law=LAW_NP, beta=1.0, stretch=STRETCH_LINEARISED, alive=None,
                   pv_h=0.0, j=None):
        """Total strain energy sum_i V_i U_i."""
        _, U = self.force_law(u, c, law, beta, stretch, 0.0, alive, energy=True, pv_h=pv_h, j=j)
        return lib().or_potential(self.n, _p(self.V), _p(U))

    def steps_j(self, state, c, rho, s_c, dt, nsteps, j, law=LAW_LINEAR, beta=1.0,
                stretch=STRETCH_LINEARISED, pv_h=0.0, central=False, bc_kind=None,
                bc_vel=None, b=None, ramp=0):
        """Velocity-Verlet (central=False) or central-difference steps of a
        pairwise law with the influence function j = (c1, c2), in place."""
        bc_kind = None if bc_kind is None else np.ascontiguousarray(bc_kind, np.uint8)
        bc_vel = None if bc_vel is None else _f64(bc_vel)
        b = None if b is None else _f64(b)
        fn = lib().or_central_j if central else lib().or_verlet_j
        fn(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X), _p(self.V), float(rho),
           float(c), float(s_c), int(law), float(beta), int(stretch), float(pv_h), self.delta,
           float(j[0]), float(j[1]), self.delta - 0.5 * float(pv_h), _p(bc_kind), _p(bc_vel),
           _p(b), int(ramp), float(dt), int(state["step"]), int(nsteps), _p(state["u"]),
           _p(state["v"]), _p(state["f"]), _p(state["alive"]))
        state["step"] += nsteps
        return state

    def verlet_pv(self, state, rho, dt, nsteps, pv_h, lps=False, c=0.0, s_c=0.0, law=LAW_LINEAR,
                  beta=1.0, stretch=STRETCH_LINEARISED, K=0.0, mu=0.0, bc_kind=None,
                  bc_vel=None, b=None, ramp=0):
        """Velocity-Verlet steps with partial volumes, a pairwise law or
        (lps=True) the peridynamic solid."""
        bc_kind = None if bc_kind is None else np.ascontiguousarray(bc_kind, np.uint8)
        bc_vel = None if bc_vel is None else _f64(bc_vel)
        b = None if b is None else _f64(b)
        lib().or_verlet_pv(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                           _p(self.V), float(rho), int(bool(lps)), float(c), float(s_c), int(law),
                           float(beta), int(stretch), float(K), float(mu), float(pv_h),
                           self.delta, _p(bc_kind), _p(bc_vel), _p(b), int(ramp), float(dt),
                           int(state["step"]), int(nsteps), _p(state["u"]), _p(state["v"]),
                           _p(state["f"]), _p(state["alive"]))
        state["step"] += nsteps
        return state

    def tangent_law(self, w, c, law=LAW_NP, beta=1.0, ulin=None, fixed=None, alive=None):
        w = _f64(w)
        y = np.zeros_like(w)
        ulin = None if ulin is None else _f64(ulin)
        fixed = None if fixed is None else np.ascontiguousarray(fixed, np.uint8)
        lib().or_tangent_law(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                             _p(self.V), float(c), int(law), float(beta), _p(ulin), _p(alive),
                             _p(fixed), _p(w), _p(y))
        return y

    def start_law(self, u0, v0, c, law=LAW_NP, beta=1.0, stretch=STRETCH_LINEARISED, s_c=0.0,
                  alive=None):
        alive = self.all_alive() if alive is None else np.ascontiguousarray(alive, np.uint8).copy()
        u = _f64(u0).copy()
        v = _f64(v0).copy()
        f = self.force_law(u, c, law, beta, stretch, s_c, alive)
        return {"u": u, "v": v, "f": f, "alive": alive, "step": 0}

    def verlet_law(self, state, c, rho, s_c, dt, nsteps, law=LAW_NP, beta=1.0,
                   stretch=STRETCH_LINEARISED, bc_kind=None, bc_vel=None, b=None, ramp=0):
        bc_kind = None if bc_kind is None else np.ascontiguousarray(bc_kind, np.uint8)
        bc_vel = None if bc_vel is None else _f64(bc_vel)
        b = None if b is None else _f64(b)
        lib().or_verlet_law(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                            _p(self.V), float(rho), float(c), float(s_c), int(law), float(beta),
                            int(stretch), _p(bc_kind), _p(bc_vel), _p(b), int(ramp), float(dt),
                            int(state["step"]), int(nsteps), _p(state["u"]), _p(state["v"]),
                            _p(state["f"]), _p(state["alive"]))
        state["step"] += nsteps
        return state

    def central_law(self, state, c, rho, s_c, dt, nsteps, law=LAW_LINEAR, beta=1.0,
                    stretch=STRETCH_LINEARISED, bc_kind=None, bc_vel=None, b=None, ramp=0):
        """Central-difference steps (first step velocity Verlet), in place."""
        bc_kind = None if bc_kind is None else np.ascontiguousarray(bc_kind, np.uint8)
        bc_vel = None if bc_vel is None else _f64(bc_vel)
        b = None if b is None else _f64(b)
        lib().or_central_law(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                             _p(self.V), float(rho), float(c), float(s_c), int(law),
                             float(beta), int(stretch), _p(bc_kind), _p(bc_vel), _p(b),
                             int(ramp), float(dt), int(state["step"]), int(nsteps),
                             _p(state["u"]), _p(state["v"]), _p(state["f"]),
                             _p(state["alive"]))
        state["step"] += nsteps
        return state

    def residual_law(self, u, c, b, law=LAW_NP, beta=1.0, fixed=None, alive=None):
        u = _f64(u)
        r = np.zeros_like(u)
        fixed = None if fixed is None else np.ascontiguousarray(fixed, np.uint8)
        b = None if b is None else _f64(b)
        nrm = lib().or_residual_law(self.dim, self.n, _p(self.row_ptr), _p(self.col),
                                    _p(self.X), _p(self.V), float(c), int(law), float(beta),
                                    _p(alive), _p(fixed), _p(b), _p(u), _p(r))
        return r, nrm

    def solve_law(self, u0, c, b, fixed, law=LAW_NP, beta=1.0, alive=None, rtol=1e-10,
                  inner_rtol=1e-12, maxit=200000, max_outer=50):
        u = _f64(u0).copy()
        fixed = np.ascontiguousarray(fixed, np.uint8)
        b = _f64(b)
        o, i, rel = C.c_int(0), C.c_int(0), C.c_double(0)
        st = lib().or_solve_law(self.dim, self.n, _p(self.row_ptr), _p(self.col), _p(self.X),
                                _p(self.V), float(c), int(law), float(beta), _p(alive),
                                _p(fixed), _p(b), _p(u), float(rtol), float(inner_rtol),
                                int(maxit), int(max_outer), C.byref(o), C.byref(i),
                                C.byref(rel))
        return u, {"status": st, "outer": o.value, "inner": i.value, "relres": rel.value}


def lps_moduli(E, nu):
    """Bulk and shear modulus of an isotropic solid."""
    return E / (3.0 * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


class LpsMesh(Mesh):
    """The linear peridynamic solid of Algorithm 2 (3-d), ``or_lps``."""

    def lps(self, u, K, mu, alive=None, pv_h=0.0):
        """(m, theta, f, W) at the displacement u (pv_h > 0: partial volumes)."""
        u = _f64(u)
        m, th, W = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        f = np.zeros_like(self.X)
        lib().or_lps_pv(self.n, _p(self.row_ptr), _p(self.col), _p(self.X), _p(self.V), _p(u),
                        float(K), float(mu), float(pv_h), self.delta, _p(alive), _p(m), _p(th),
                        _p(f), _p(W))
        return m, th, f, W

    def energy_lps(self, u, K, mu, alive=None, pv_h=0.0):
        _, _, _, W = self.lps(u, K, mu, alive, pv_h)
        return lib().or_potential(self.n, _p(self.V), _p(W))

    def start_lps(self, u0, v0, K, mu, alive=None):
        alive = self.all_alive() if alive is None else np.ascontiguousarray(alive, np.uint8).copy()
        u = _f64(u0).copy()
        v = _f64(v0).copy()
        f = self.lps(u, K, mu, alive)[2]
        return {"u": u, "v": v, "f": f, "alive": alive, "step": 0}

    def verlet_lps(self, state, K, mu, rho, dt, nsteps, bc_kind=None, bc_vel=None, b=None,
                   ramp=0):
        bc_kind = None if bc_kind is None else np.ascontiguousarray(bc_kind, np.uint8)
        bc_vel = None if bc_vel is None else _f64(bc_vel)
        b = None if b is None else _f64(b)
        lib().or_verlet_lps(self.n, _p(self.row_ptr), _p(self.col), _p(self.X), _p(self.V),
                            float(rho), float(K), float(mu), _p(bc_kind), _p(bc_vel), _p(b),
                            int(ramp), float(dt), int(state["step"]), int(nsteps),
                            _p(state["u"]), _p(state["v"]), _p(state["f"]), _p(state["alive"]))
        state["step"] += nsteps
        return state


def num_threads():
    return lib().or_num_threads()


def set_threads(k):
    """Threads of the oracle's OpenMP loops (results are the same for any)."""
    lib().or_set_threads(int(k))
