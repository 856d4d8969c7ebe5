"""Thin Python binding of ``libpd_hip.so`` (the C ABI declared in include/pd.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every computation runs in the library's HIP kernels.  Importing this
module raises if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
# PyTorch first: its HIP runtime is then the one the library binds to, the
# same one that owns the tensors and streams handed over (on hosts whose
# driver the system ROCm runtime does not match, only that one sees the GPU)
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpd_hip.so")

PD_OK, PD_EINVAL, PD_ENOMEM, PD_EDEVICE, PD_ENOCONV, PD_ENONFINITE, PD_ECAPACITY = (
    0, -1, -2, -3, -4, -5, -6)
PD_FP64, PD_MIXED, PD_FP32 = 0, 1, 2
_PREC = {"fp64": PD_FP64, "mixed": PD_MIXED, "fp32": PD_FP32}
PD_REQ_QUEUED, PD_REQ_RUNNING, PD_REQ_DONE, PD_REQ_FAILED = 0, 1, 2, 3
PD_BC_FREE, PD_BC_CLAMPED, PD_BC_VELOCITY = 0, 1, 2


class PDError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


class Material(C.Structure):
    _fields_ = [("dim", C.c_int), ("precision", C.c_int), ("c", C.c_double),
                ("rho", C.c_double), ("s_c", C.c_double), ("law", C.c_int),
                ("stretch", C.c_int), ("beta", C.c_double), ("bulk", C.c_double),
                ("shear", C.c_double), ("pv_h", C.c_double), ("j_c1", C.c_double),
                ("j_c2", C.c_double)]


class Request(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64), ("X", C.c_void_p), ("V", C.c_void_p),
                ("u0", C.c_void_p), ("v0", C.c_void_p), ("bc_kind", C.c_void_p),
                ("bc_vel", C.c_void_p), ("notch", C.c_void_p), ("nseg", C.c_int),
                ("delta", C.c_double), ("mat", Material), ("dt", C.c_double),
                ("nsteps", C.c_int64), ("ramp_steps", C.c_int64), ("keep_state", C.c_int),
                ("t_arrival", C.c_double)]


class RequestInfo(C.Structure):
    _fields_ = [("id", C.c_int64), ("state", C.c_int), ("status", C.c_int),
                ("bytes", C.c_int64), ("bonds", C.c_int64), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("tile", C.c_int), ("lanes", C.c_int), ("kernel", C.c_int),
                ("us_per_step", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("admit_s", C.c_double), ("step_s", C.c_double), ("retire_s", C.c_double),
                ("rounds", C.c_int64), ("admitted", C.c_int64), ("launches", C.c_int64),
                ("replays", C.c_int64), ("admit_overlap_s", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("inner_iters", C.c_int),
                ("rel_residual", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_1806_06917_amd.build or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "pd_version": (i32, []),
        "pd_status_string": (C.c_char_p, [i32]),
        "pd_micromodulus": (dbl, [i32, dbl, dbl]),
        "pd_ctx_create": (i32, [i32, vp, P(vp)]),
        "pd_ctx_destroy": (i32, [vp]),
        "pd_last_error": (C.c_char_p, [vp]),
        "pd_ctx_set_lanes": (i32, [vp, i32]),
        "pd_ctx_set_tuning": (i32, [vp, i32, i32, i32]),
        "pd_build_neighbors": (i32, [vp, i32, i64, vp, dbl, P(vp)]),
        "pd_nbr_info": (i32, [vp, P(i64), P(C.c_int32)]),
        "pd_nbr_export": (i32, [vp, vp, vp]),
        "pd_nbr_permutation": (i32, [vp, vp]),
        "pd_nbr_destroy": (i32, [vp]),
        "pd_internal_force": (i32, [vp, vp, P(Material), vp, vp, vp, vp, vp, vp]),
        "pd_internal_force_noalloc": (i32, [vp, vp, P(Material), vp, vp, vp, vp, vp, vp]),
        "pd_sim_create": (i32, [vp, vp, P(Material), vp, vp, vp, vp, vp, vp, vp, vp, i32, i64,
                                P(vp)]),
        "pd_verlet_step": (i32, [vp, i64, dbl]),
        "pd_central_step": (i32, [vp, i64, dbl]),
        "pd_sim_get": (i32, [vp, vp, vp, vp, vp, vp]),
        "pd_sim_set": (i32, [vp, vp, vp, vp, i64]),
        "pd_sim_destroy": (i32, [vp]),
        "pd_sim_info": (i32, [vp, P(i32), P(i32), P(i32), P(i32)]),
        "pd_batch_create": (i32, [vp, P(vp)]),
        "pd_batch_step": (i32, [vp, vp, i32, vp, vp, i64, i32]),
        "pd_batch_destroy": (i32, [vp]),
        "pd_autotune": (i32, [vp, i32, i64, vp, vp, dbl, i32, i32, P(TuneResult), i32, P(i32),
                              P(TuneResult)]),
        "pd_tune_lookup": (i32, [vp, i32, dbl, i32, P(TuneResult)]),
        "pd_tune_set": (i32, [vp, i32, dbl, i32, i32, i32]),
        "pd_tune_clear": (i32, [vp]),
        "pd_server_clock": (dbl, []),
        "pd_server_create": (i32, [vp, i64, i64, i32, P(vp)]),
        "pd_server_submit": (i32, [vp, P(Request), P(i64)]),
        "pd_server_pump": (i32, [vp, P(i32), P(i32)]),
        "pd_server_info": (i32, [vp, i64, P(RequestInfo)]),
        "pd_server_result": (i32, [vp, i64, vp, vp]),
        "pd_server_usage": (i32, [vp, P(i64), P(i64)]),
        "pd_server_destroy": (i32, [vp]),
        "pd_server_get_stats": (i32, [vp, P(ServerStats)]),
        "pd_apply_tangent": (i32, [vp, vp, P(Material), vp, vp, vp, vp, vp, vp]),
        "pd_apply_tangent_at": (i32, [vp, vp, P(Material), vp, vp, vp, vp, vp, vp, vp]),
        "pd_solve_implicit": (i32, [vp, vp, P(Material), vp, vp, vp, vp, vp, vp, dbl, i32,
                                    P(SolveInfo)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def micromodulus(dim, E, delta):
    return lib.pd_micromodulus(int(dim), float(E), float(delta))


def _ptr(t):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


class Context:
    def __init__(self, device=0, stream=None):
        import torch
        self.device = device
        self._stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = lib.pd_ctx_create(int(device), C.c_void_p(self._stream.cuda_stream), C.byref(h))
        if st != PD_OK:
            raise PDError(st, f"pd_ctx_create: {lib.pd_status_string(st).decode()}")
        self.h = h

    @property
    def stream(self):
        return self._stream

    def check(self, st, what):
        if st != PD_OK:
            msg = lib.pd_last_error(self.h).decode(errors="replace")
            raise PDError(st, f"{what}: {msg}")
        return st

    def set_lanes(self, lanes):
        self.check(lib.pd_ctx_set_lanes(self.h, int(lanes)), "pd_ctx_set_lanes")

    def set_tuning(self, kernel=0, tile=0, block=0):
        """kernel: 0 auto, 1 gather, 2 LDS tiles, 3 streamed tiles (steps); tile/block
        sizes (0 = auto)."""
        kind = {"auto": 0, "gather": 1, "tile": 2, "stream": 3}.get(kernel, kernel)
        self.check(lib.pd_ctx_set_tuning(self.h, int(kind), int(tile), int(block)),
                   "pd_ctx_set_tuning")

    def autotune(self, X, V, delta, precision="mixed", steps=20):
        """Times every tile size x lanes candidate on the mesh (X, V, delta) and
        caches the fastest for meshes of its kind (pd_autotune).  Returns
        (best, table) as dicts."""
        prec = _PREC[precision]
        table = (TuneResult * 16)()
        nt = C.c_int()
        best = TuneResult()
        self.check(lib.pd_autotune(self.h, int(X.shape[1]), int(X.shape[0]), _ptr(X), _ptr(V),
                                   float(delta), prec, int(steps), table, 16, C.byref(nt),
                                   C.byref(best)), "pd_autotune")
        row = lambda r: {k: getattr(r, k) for k, _ in TuneResult._fields_}  # noqa: E731
        return row(best), [row(table[i]) for i in range(nt.value)]

    def tune_lookup(self, dim, mean_neighbors, precision="mixed"):
        prec = _PREC[precision]
        r = TuneResult()
        self.check(lib.pd_tune_lookup(self.h, int(dim), float(mean_neighbors), prec,
                                      C.byref(r)), "pd_tune_lookup")
        return (r.tile, r.lanes) if r.tile else None

    def tune_set(self, dim, mean_neighbors, tile, lanes, precision="mixed"):
        prec = _PREC[precision]
        self.check(lib.pd_tune_set(self.h, int(dim), float(mean_neighbors), prec, int(tile),
                                   int(lanes)), "pd_tune_set")

    def tune_clear(self):
        self.check(lib.pd_tune_clear(self.h), "pd_tune_clear")

    def close(self):
        if getattr(self, "h", None):
            lib.pd_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PD_LAW_LINEAR, PD_LAW_NP, PD_LAW_LPS = 0, 1, 2
PD_STRETCH_LINEARISED, PD_STRETCH_EXACT = 0, 1


def material(dim, c, rho=1.0, s_c=0.0, precision="fp64", law="linear", beta=0.0,
             stretch="linearised", bulk=0.0, shear=0.0, pv_h=0.0, j=None):
    """law: "linear" | "np" (psi(r) = C (1 - exp(-beta r))) | "lps" (the
    3-d linear peridynamic solid with moduli bulk, shear; c unused);
    stretch: "linearised" | "exact"; pv_h > 0: partial volumes (neighbours
    built at delta + pv_h/2); j = (c1, c2): influence function
    J = c1 r exp(-r^2/c2) of r = |xi|/delta on every bond (None: J = 1)."""
    prec = _PREC[precision] if isinstance(precision, str) \
        else int(precision)
    lw = {"linear": PD_LAW_LINEAR, "np": PD_LAW_NP, "lps": PD_LAW_LPS}[law] \
        if isinstance(law, str) else int(law)
    sk = {"linearised": PD_STRETCH_LINEARISED, "exact": PD_STRETCH_EXACT}[stretch] \
        if isinstance(stretch, str) else int(stretch)
    j1, j2 = (0.0, 0.0) if j is None else (float(j[0]), float(j[1]))
    return Material(int(dim), prec, float(c), float(rho), float(s_c), lw, sk, float(beta),
                    float(bulk), float(shear), float(pv_h), j1, j2)


class Neighbors:
    """Neighbour lists built on the GPU (pd_build_neighbors)."""

    def __init__(self, ctx: Context, X, delta):
        self.ctx = ctx
        self.X = X
        self.n, self.dim = int(X.shape[0]), int(X.shape[1])
        h = C.c_void_p()
        ctx.check(lib.pd_build_neighbors(ctx.h, self.dim, self.n, _ptr(X), float(delta),
                                         C.byref(h)), "pd_build_neighbors")
        self.h = h
        nnz, mr = C.c_int64(), C.c_int32()
        lib.pd_nbr_info(h, C.byref(nnz), C.byref(mr))
        self.nnz, self.max_row = nnz.value, mr.value

    def export(self):
        rp = np.zeros(self.n + 1, np.int64)
        col = np.zeros(max(self.nnz, 1), np.int32)
        self.ctx.check(lib.pd_nbr_export(self.h, rp.ctypes.data_as(C.c_void_p),
                                         col.ctypes.data_as(C.c_void_p)), "pd_nbr_export")
        return rp, col[: self.nnz]

    def permutation(self):
        p = np.zeros(self.n, np.int32)
        self.ctx.check(lib.pd_nbr_permutation(self.h, p.ctypes.data_as(C.c_void_p)),
                       "pd_nbr_permutation")
        return p

    def close(self):
        if getattr(self, "h", None):
            lib.pd_nbr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def internal_force(ctx, nbr, mat, X, V, u, f, alive=None, U=None):
    ctx.check(lib.pd_internal_force(ctx.h, nbr.h, C.byref(mat), _ptr(X), _ptr(V), _ptr(u),
                                    _ptr(alive), _ptr(f), _ptr(U)), "pd_internal_force")


def internal_force_noalloc(ctx, nbr, mat, X, V, u, f, alive=None, U=None):
    """pd_internal_force with the library's fixed device scratch array (no
    allocation; meshes above PD_NOALLOC_MAX_BYTES of working copies fail)."""
    ctx.check(lib.pd_internal_force_noalloc(ctx.h, nbr.h, C.byref(mat), _ptr(X), _ptr(V),
                                            _ptr(u), _ptr(alive), _ptr(f), _ptr(U)),
              "pd_internal_force_noalloc")


NOALLOC_MAX_BYTES = 64 << 20


def apply_tangent(ctx, nbr, mat, X, V, w, y, alive=None, fixed=None):
    ctx.check(lib.pd_apply_tangent(ctx.h, nbr.h, C.byref(mat), _ptr(X), _ptr(V), _ptr(alive),
                                   _ptr(fixed), _ptr(w), _ptr(y)), "pd_apply_tangent")


def apply_tangent_at(ctx, nbr, mat, X, V, u, w, y, alive=None, fixed=None):
    """Tangent linearised at the displacement u (NP law; linear: as apply_tangent)."""
    ctx.check(lib.pd_apply_tangent_at(ctx.h, nbr.h, C.byref(mat), _ptr(X), _ptr(V), _ptr(u),
                                      _ptr(alive), _ptr(fixed), _ptr(w), _ptr(y)),
              "pd_apply_tangent_at")


@dataclass
class SolveResult:
    status: int
    outer: int
    inner: int
    rel_residual: float


def solve_implicit(ctx, nbr, mat, X, V, b, u, fixed=None, alive=None, rtol=1e-10,
                   maxit=100000, raise_on_noconv=True):
    info = SolveInfo()
    st = lib.pd_solve_implicit(ctx.h, nbr.h, C.byref(mat), _ptr(X), _ptr(V), _ptr(alive),
                               _ptr(fixed), _ptr(b), _ptr(u), float(rtol), int(maxit),
                               C.byref(info))
    if st != PD_ENOCONV or raise_on_noconv:
        ctx.check(st, "pd_solve_implicit")
    return SolveResult(st, info.outer_iters, info.inner_iters, info.rel_residual)


class Simulation:
    """Resident explicit simulation (pd_sim_create / pd_verlet_step / ...)."""

    def __init__(self, ctx, nbr, mat, X, V, u0=None, v0=None, bc_kind=None, bc_vel=None, b=None,
                 notch=None, ramp_steps=0):
        self.ctx, self.nbr, self.mat = ctx, nbr, mat
        seg = None
        nseg = 0
        if notch is not None and len(notch):
            seg = np.ascontiguousarray(np.asarray(notch, np.float64).reshape(-1, 4))
            nseg = seg.shape[0]
        h = C.c_void_p()
        ctx.check(lib.pd_sim_create(ctx.h, nbr.h, C.byref(mat), _ptr(X), _ptr(V), _ptr(u0),
                                    _ptr(v0), _ptr(bc_kind), _ptr(bc_vel), _ptr(b),
                                    None if seg is None else seg.ctypes.data_as(C.c_void_p),
                                    nseg, int(ramp_steps), C.byref(h)), "pd_sim_create")
        self.h = h

    def step(self, nsteps, dt):
        self.ctx.check(lib.pd_verlet_step(self.h, int(nsteps), float(dt)), "pd_verlet_step")

    def central_step(self, nsteps, dt):
        """Central-difference steps (the first one of each call velocity Verlet)."""
        self.ctx.check(lib.pd_central_step(self.h, int(nsteps), float(dt)), "pd_central_step")

    def get(self, u=None, v=None, alive=None, energies=False, allow_nonfinite=False):
        kp = np.zeros(2, np.float64)
        step = C.c_int64()
        st = lib.pd_sim_get(self.h, _ptr(u), _ptr(v), _ptr(alive),
                            kp.ctypes.data_as(C.c_void_p) if energies else None, C.byref(step))
        if not (allow_nonfinite and st == PD_ENONFINITE):
            self.ctx.check(st, "pd_sim_get")
        return {"ke": kp[0], "pe": kp[1], "step": step.value, "status": st}

    def info(self):
        """Launch configuration: kernel ('gather' | 'tile' | 'stream'), tile, block, lanes."""
        k, t, b, l = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        self.ctx.check(lib.pd_sim_info(self.h, C.byref(k), C.byref(t), C.byref(b), C.byref(l)),
                       "pd_sim_info")
        return {"kernel": {1: "gather", 2: "tile", 3: "stream"}[k.value], "tile": t.value,
                "block": b.value,
                "lanes": l.value}

    def set(self, u=None, v=None, alive=None, step=0):
        self.ctx.check(lib.pd_sim_set(self.h, _ptr(u), _ptr(v), _ptr(alive), int(step)),
                       "pd_sim_set")

    def close(self):
        if getattr(self, "h", None):
            lib.pd_sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched explicit steps of several simulations (pd_batch_*)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        h = C.c_void_p()
        ctx.check(lib.pd_batch_create(ctx.h, C.byref(h)), "pd_batch_create")
        self.h = h

    def step(self, sims, steps, dts, nsteps, graph=True):
        """sims[k] takes steps[k] <= nsteps steps of dts[k]; one launch per step."""
        n = len(sims)
        handles = (C.c_void_p * n)(*[s.h for s in sims])
        st = np.ascontiguousarray(steps, dtype=np.int64)
        dt = np.ascontiguousarray(dts, dtype=np.float64)
        assert st.shape == (n,) and dt.shape == (n,)
        self.ctx.check(lib.pd_batch_step(self.h, C.cast(handles, C.c_void_p), n,
                                         st.ctypes.data_as(C.c_void_p),
                                         dt.ctypes.data_as(C.c_void_p), int(nsteps),
                                         1 if graph else 0), "pd_batch_step")

    def close(self):
        if getattr(self, "h", None):
            lib.pd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


class Server:
    """Serving loop over the C ABI (pd_server_*): requests with host arrays."""

    def __init__(self, ctx: Context, hbm_budget, chunk_steps=100, lanes=0):
        self.ctx = ctx
        h = C.c_void_p()
        ctx.check(lib.pd_server_create(ctx.h, int(hbm_budget), int(chunk_steps), int(lanes),
                                       C.byref(h)), "pd_server_create")
        self.h = h

    @staticmethod
    def clock():
        return lib.pd_server_clock()

    def submit(self, X, V, mat, delta, dt, nsteps, u0=None, v0=None, bc_kind=None,
               bc_vel=None, notch=None, ramp_steps=0, keep_state=False, t_arrival=0.0):
        X = _host(X, np.float64)
        n, dim = X.shape
        arrs = dict(V=_host(V, np.float64), u0=_host(u0, np.float64), v0=_host(v0, np.float64),
                    bc_kind=_host(bc_kind, np.uint8), bc_vel=_host(bc_vel, np.float64),
                    notch=_host(notch, np.float64))
        ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        nseg = 0 if arrs["notch"] is None else arrs["notch"].reshape(-1, 4).shape[0]
        req = Request(dim, n, ptr(X), ptr(arrs["V"]), ptr(arrs["u0"]), ptr(arrs["v0"]),
                      ptr(arrs["bc_kind"]), ptr(arrs["bc_vel"]), ptr(arrs["notch"]), nseg,
                      float(delta), mat, float(dt), int(nsteps), int(ramp_steps),
                      1 if keep_state else 0, float(t_arrival))
        rid = C.c_int64()
        self.ctx.check(lib.pd_server_submit(self.h, C.byref(req), C.byref(rid)),
                       "pd_server_submit")
        return rid.value

    def pump(self):
        """One scheduling round; returns (running, queued)."""
        r, q = C.c_int(), C.c_int()
        self.ctx.check(lib.pd_server_pump(self.h, C.byref(r), C.byref(q)), "pd_server_pump")
        return r.value, q.value

    def info(self, rid):
        i = RequestInfo()
        self.ctx.check(lib.pd_server_info(self.h, int(rid), C.byref(i)), "pd_server_info")
        return {k: getattr(i, k) for k, _ in RequestInfo._fields_}

    def result(self, rid, n, dim):
        u = np.zeros((n, dim))
        v = np.zeros((n, dim))
        self.ctx.check(lib.pd_server_result(self.h, int(rid), u.ctypes.data_as(C.c_void_p),
                                            v.ctypes.data_as(C.c_void_p)), "pd_server_result")
        return u, v

    def usage(self):
        used, peak = C.c_int64(), C.c_int64()
        self.ctx.check(lib.pd_server_usage(self.h, C.byref(used), C.byref(peak)),
                       "pd_server_usage")
        return used.value, peak.value

    def stats(self):
        st = ServerStats()
        self.ctx.check(lib.pd_server_get_stats(self.h, C.byref(st)), "pd_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib.pd_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
