"""ctypes binding of libbem.so (argument marshalling only; every step runs in the HIP library).

The names mirror the C-ABI in include/bem.h.  Importing this module loads the in-tree
``paper_2310_09204_amd/libbem.so`` and fails loudly if it is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbem.so")

BEM_OK = 0
BEM_PENDING = 1
ERRORS = {
    -1: "BEM_E_INVALID_ARG", -2: "BEM_E_MESH_NONCONFORMING", -3: "BEM_E_DEGENERATE",
    -4: "BEM_E_POINT_CONTACT", -5: "BEM_E_NOT_SPD", -6: "BEM_E_BREAKDOWN", -7: "BEM_E_NOT_CONVERGED",
    -8: "BEM_E_ADMISSION", -9: "BEM_E_OOM", -10: "BEM_E_DEVICE", -11: "BEM_E_UNSUPPORTED",
}
FP64, FP32_REFINE = 0, 1


class BemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code
        self.name = ERRORS.get(code, "?")


class AssembleOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("near_order", ctypes.c_int), ("keep_pair_matrix", ctypes.c_int),
                ("pair_panel_rows", ctypes.c_int64), ("keep_order", ctypes.c_int32)]


class ProblemInfo(ctypes.Structure):
    _fields_ = [("n_dofs", ctypes.c_int64), ("n_tri", ctypes.c_int64), ("n_vert", ctypes.c_int64),
                ("n_near_pairs", ctypes.c_int64), ("bytes_device", ctypes.c_int64),
                ("q_hist", ctypes.c_int64 * 16), ("t_assemble_s", ctypes.c_double),
                ("t_far_s", ctypes.c_double), ("t_near_s", ctypes.c_double), ("t_contract_s", ctypes.c_double),
                ("t_host_s", ctypes.c_double), ("n_pair_panels", ctypes.c_int64), ("dim", ctypes.c_int64),
                ("panels_replanned", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("max_triangles", ctypes.c_int64), ("far_separation", ctypes.c_double),
                ("panel_fraction", ctypes.c_double), ("symv_blocks_fp64", ctypes.c_int32),
                ("symv_blocks_fp32", ctypes.c_int32), ("check_every", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")


def tuning_file(arch: str = "gfx950") -> str:
    """The autotuner's committed table for a device architecture."""
    return os.path.join(TUNING_DIR, arch + ".json")


def load_tuning(path: str):
    """Entries of a tuning table written by tune.py (a list of dicts with the Tuning fields)."""
    with open(path) as f:
        d = json.load(f)
    return d["entries"]


class PrecondOpts(ctypes.Structure):
    _fields_ = [("use_coarse", ctypes.c_int), ("factor_fp32", ctypes.c_int), ("wirebasket", ctypes.c_int),
                ("diag_shift", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("use_precond", ctypes.c_int),
                ("precision", ctypes.c_int), ("refresh_factor", ctypes.c_double), ("check_every", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("x0", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("status", ctypes.c_int),
                ("graph", ctypes.c_int), ("relres", ctypes.c_double), ("est_cond", ctypes.c_double), ("t_total_s", ctypes.c_double),
                ("t_start_s", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [("vertices", ctypes.c_void_p), ("nv", ctypes.c_int64), ("triangles", ctypes.c_void_p),
                ("nt", ctypes.c_int64), ("patch_of_triangle", ctypes.c_void_p),
                ("coarse_vertices", ctypes.c_void_p), ("ncv", ctypes.c_int64),
                ("coarse_triangles", ctypes.c_void_p), ("nct", ctypes.c_int64),
                ("coarse_of_triangle", ctypes.c_void_p), ("g", ctypes.c_void_p), ("k", ctypes.c_int32),
                ("precision", ctypes.c_int), ("tol", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "rejected", "merged_batches",
                                                "cache_hits", "cache_misses", "resident_bytes",
                                                "peak_resident_bytes", "evictions", "admitted_running")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# symbol -> (restype, argtypes)
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_ci = ctypes.c_int
SIGNATURES = {
    "bem_ctx_create": (_ci, [_ci, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "bem_ctx_destroy": (None, [_vp]),
    "bem_ctx_synchronize": (_ci, [_vp]),
    "bem_ctx_release_cached": (_ci, [_vp]),
    "bem_ctx_set_tuning": (_ci, [_vp, ctypes.c_void_p, _i32]),
    "bem_problem_tuning": (_ci, [_vp, ctypes.c_void_p]),
    "bem_double_layer": (_ci, [_vp, _vp, _i32, _vp, _i64, _vp]),
    "bem_assemble_2d": (_ci, [_vp, _vp, _i64, _vp, _i64, _vp, ctypes.POINTER(_vp)]),
    "bem_mesh_analyze_2d": (_ci, [_vp, _i64, _vp, _i64, ctypes.POINTER(_i64), _vp, _vp, _vp, _vp]),
    "bem_problem_bench_matvec": (_ci, [_vp, _ci, _i32, _ci, ctypes.POINTER(ctypes.c_double)]),
    "bem_mesh_analyze": (_ci, [_vp, _i64, _vp, _i64, ctypes.POINTER(_i64), _vp, _vp, _vp]),
    "bem_assemble": (_ci, [_vp, _vp, _i64, _vp, _i64, ctypes.POINTER(AssembleOpts), ctypes.POINTER(_vp)]),
    "bem_assemble_dev": (_ci, [_vp, _vp, _vp, _i64, _vp, _vp, _i64, ctypes.POINTER(AssembleOpts), ctypes.POINTER(_vp)]),
    "bem_problem_destroy": (None, [_vp]),
    "bem_problem_get_info": (_ci, [_vp, ctypes.POINTER(ProblemInfo)]),
    "bem_problem_dofs": (_ci, [_vp, _vp, _vp]),
    "bem_problem_copy_matrix": (_ci, [_vp, _i64, _i64, _vp]),
    "bem_problem_copy_rows": (_ci, [_vp, _vp, _i64, _vp]),
    "bem_problem_pair_integrals": (_ci, [_vp, _vp, _i64, _vp]),
    "bem_rhs": (_ci, [_vp, _vp, _i32, _vp]),
    "bem_matvec": (_ci, [_vp, _vp, _i32, _ci, _vp]),
    "bem_matvec_noalloc": (_ci, [_vp, _vp, _i32, _ci, _vp]),
    "bem_jump_values": (_ci, [_vp, _vp, _vp]),
    "bem_precond_setup": (_ci, [_vp, _vp, _vp, _i64, _vp, _i64, _vp, ctypes.POINTER(PrecondOpts), ctypes.POINTER(_vp)]),
    "bem_precond_setup_2d": (_ci, [_vp, _vp, _vp, _i64, _vp, _i64, _vp, ctypes.POINTER(PrecondOpts), ctypes.POINTER(_vp)]),
    "bem_precond_destroy": (None, [_vp]),
    "bem_precond_sizes": (_ci, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "bem_precond_apply": (_ci, [_vp, _vp, _i32, _vp]),
    "bem_pcg_solve": (_ci, [_vp, _vp, _vp, _i32, ctypes.POINTER(SolveOpts), _vp, _vp]),
    "bem_pcg_solve_rhs": (_ci, [_vp, _vp, _vp, _i32, ctypes.POINTER(SolveOpts), _vp, _vp]),
    "bem_pcg_solve_dev": (_ci, [_vp, _vp, _vp, _i32, ctypes.POINTER(SolveOpts), _vp, _vp]),
    "bem_server_create": (_ci, [_vp, _ci, ctypes.POINTER(_vp)]),
    "bem_server_destroy": (None, [_vp]),
    "bem_serve_submit": (_ci, [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "bem_serve_poll": (_ci, [_vp, ctypes.c_uint64, _i64, _vp, _vp]),
    "bem_serve_ndofs": (_ci, [_vp, ctypes.c_uint64, ctypes.POINTER(_i64)]),
    "bem_server_get_stats": (_ci, [_vp, ctypes.POINTER(ServerStats)]),
    "bem_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbem.so is not built (%s); run `python -m paper_2310_09204_amd.build` "
                               "or __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code < 0:
        raise BemError(code, load().bem_last_error().decode())
    return code


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32a(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def mesh_analyze(V, T):
    """Host-only sectors / dofs (no device work): returns dict(n_dofs, dof_vertex, dof_sector, q)."""
    L = load()
    V, T = _f64(V), _i32a(T)
    n = ctypes.c_int64(0)
    _check(L.bem_mesh_analyze(_p(V), V.shape[0], _p(T), T.shape[0], ctypes.byref(n), None, None, None))
    dv = np.empty(n.value, np.int32)
    ds = np.empty(n.value, np.int32)
    q = np.empty(V.shape[0], np.int32)
    _check(L.bem_mesh_analyze(_p(V), V.shape[0], _p(T), T.shape[0], ctypes.byref(n), _p(dv), _p(ds), _p(q)))
    return {"n_dofs": n.value, "dof_vertex": dv, "dof_sector": ds, "q": q}


class Context:
    """A device context.  tuning: "auto" loads the autotuner's table for gfx950 when it is present
    (paper_2310_09204_amd/tuning/gfx950.json), None keeps the defaults, or a list of entries."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, tuning="auto"):
        self._h = ctypes.c_void_p()
        _check(load().bem_ctx_create(device, hbm_budget_bytes, ctypes.byref(self._h)))
        self.tuning = []
        if tuning == "auto":
            path = tuning_file()
            if os.path.exists(path):
                self.set_tuning(load_tuning(path))
        elif tuning:
            self.set_tuning(tuning)

    def set_tuning(self, entries):
        """bem_ctx_set_tuning with a list of dicts (Tuning fields; missing fields take the defaults)."""
        arr = (Tuning * max(1, len(entries)))()
        for i, e in enumerate(entries):
            for k, v in e.items():
                if k in dict(Tuning._fields_):
                    setattr(arr[i], k, v)
        _check(load().bem_ctx_set_tuning(self._h, ctypes.cast(arr, ctypes.c_void_p), len(entries)))
        self.tuning = [dict(e) for e in entries]

    @property
    def handle(self):
        return self._h

    def synchronize(self):
        _check(load().bem_ctx_synchronize(self._h))

    def release_cached(self):
        """Returns the device buffers the library keeps for reuse to the HIP runtime."""
        _check(load().bem_ctx_release_cached(self._h))

    def close(self):
        if self._h:
            load().bem_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def _hiprt():
    """The HIP runtime that libbem.so links (device buffers for the *_dev entry points)."""
    global _hip
    if _hip is None:
        load()   # loads libamdhip64 as a dependency of libbem.so
        _hip = ctypes.CDLL("libamdhip64.so", mode=ctypes.RTLD_GLOBAL)
        _hip.hipMalloc.argtypes = [ctypes.POINTER(_vp), ctypes.c_size_t]
        _hip.hipFree.argtypes = [_vp]
        _hip.hipMemcpy.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int]
        _hip.hipSetDevice.argtypes = [ctypes.c_int]
    return _hip


class DeviceArray:
    """A numpy array's copy in device memory (hipMalloc / hipMemcpy), for the entry points that take
    device pointers.  .ptr is the device address; .get() copies it back."""

    def __init__(self, a=None, shape=None, dtype=np.float64, device=0):
        h = _hiprt()
        _check_hip(h.hipSetDevice(device))
        if a is not None:
            a = np.ascontiguousarray(a)
            self.shape, self.dtype = a.shape, a.dtype
        else:
            self.shape, self.dtype = tuple(shape), np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        p = _vp()
        _check_hip(h.hipMalloc(ctypes.byref(p), max(self.nbytes, 1)))
        self._p = p
        if a is not None and self.nbytes:
            _check_hip(h.hipMemcpy(p, a.ctypes.data_as(_vp), self.nbytes, 1))   # host to device

    @property
    def ptr(self):
        return self._p.value

    def get(self):
        out = np.empty(self.shape, dtype=self.dtype)
        if self.nbytes:
            _check_hip(_hiprt().hipMemcpy(out.ctypes.data_as(_vp), self._p, self.nbytes, 2))   # device to host
        return out

    def close(self):
        if self._p:
            _hiprt().hipFree(self._p)
            self._p = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_hip(code):
    if code != 0:
        raise RuntimeError("HIP runtime error %d" % code)


class Problem:
    """bem_assemble: W resident on the device.  With device_mesh = (address of V, address of T) in
    device memory (same values as V, T), bem_assemble_dev: the kernels read those copies."""

    def __init__(self, ctx: Context, V, T, precision=FP64, near_order=10, keep_pair_matrix=False, pair_panel_rows=0,
                 device_mesh=None, keep_order=False):
        self.ctx = ctx
        self.V, self.T = _f64(V), _i32a(T)
        o = AssembleOpts(precision, near_order, int(keep_pair_matrix), int(pair_panel_rows), int(keep_order))
        self._h = ctypes.c_void_p()
        if device_mesh is None:
            _check(load().bem_assemble(ctx.handle, _p(self.V), self.V.shape[0], _p(self.T), self.T.shape[0],
                                       ctypes.byref(o), ctypes.byref(self._h)))
        else:
            dV, dT = device_mesh
            _check(load().bem_assemble_dev(ctx.handle, _p(self.V), ctypes.c_void_p(dV), self.V.shape[0], _p(self.T),
                                           ctypes.c_void_p(dT), self.T.shape[0], ctypes.byref(o), ctypes.byref(self._h)))
        self.N = self.get_info()["n_dofs"]

    @property
    def tuning(self):
        """The launch parameters this problem was assembled with (bem_problem_tuning)."""
        t = Tuning()
        _check(load().bem_problem_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    @property
    def info(self):
        """bem_problem_get_info, read at each access (the phase times t_far_s, t_near_s and
        t_contract_s are NaN while device work that bem_assemble leaves running has not finished)."""
        return self.get_info()

    def get_info(self):
        i = ProblemInfo()
        _check(load().bem_problem_get_info(self._h, ctypes.byref(i)))
        d = {f: getattr(i, f) for f, _ in ProblemInfo._fields_ if f != "q_hist"}
        d["q_hist"] = list(i.q_hist)
        return d

    @property
    def handle(self):
        return self._h

    def dofs(self):
        dv = np.empty(self.N, np.int32)
        ds = np.empty(self.N, np.int32)
        _check(load().bem_problem_dofs(self._h, _p(dv), _p(ds)))
        return dv, ds

    def matrix(self, row0=0, nrows=None):
        nrows = self.N - row0 if nrows is None else nrows
        out = np.empty((nrows, self.N))
        _check(load().bem_problem_copy_matrix(self._h, row0, nrows, _p(out)))
        return out

    def rows(self, rows):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.empty((rows.shape[0], self.N))
        _check(load().bem_problem_copy_rows(self._h, _p(rows), rows.shape[0], _p(out)))
        return out

    def pair_integrals(self, pairs):
        pairs = _i32a(pairs).reshape(-1, 2)
        out = np.empty(pairs.shape[0])
        _check(load().bem_problem_pair_integrals(self._h, _p(pairs), pairs.shape[0], _p(out)))
        return out

    def rhs(self, g):
        g = _f64(np.atleast_2d(g))
        out = np.empty((g.shape[0], self.N))
        _check(load().bem_rhs(self._h, _p(g), g.shape[0], _p(out)))
        return out

    def matvec(self, x, fp32=False):
        x = _f64(np.atleast_2d(x))
        y = np.empty_like(x)
        _check(load().bem_matvec(self._h, _p(x), x.shape[0], int(fp32), _p(y)))
        return y

    def matvec_noalloc(self, d_x, k, d_y, fp32=False):
        """y = W x on device buffers (addresses of [k][N] doubles) through bem_matvec_noalloc."""
        _check(load().bem_matvec_noalloc(self._h, _vp(d_x), int(k), int(fp32), _vp(d_y)))

    def bench_matvec(self, fp32=False, k=1, reps=10):
        """Mean seconds per device-resident product W x (k columns), timed with HIP events."""
        t = ctypes.c_double()
        _check(load().bem_problem_bench_matvec(self._h, int(fp32), k, reps, ctypes.byref(t)))
        return t.value

    def jump_values(self, phi):
        phi = _f64(phi)
        out = np.empty((self.T.shape[0], self.T.shape[1]))   # corners of a triangle / ends of a segment
        _check(load().bem_jump_values(self._h, _p(phi), _p(out)))
        return out

    def double_layer(self, phi, targets):
        """U[k][m]: double-layer potential of the solutions phi[k][N] at targets[m][3]."""
        phi = _f64(np.atleast_2d(phi))
        X = _f64(np.atleast_2d(targets))
        if X.shape[1] != 3:
            raise ValueError("targets must be m x 3")
        out = np.empty((phi.shape[0], X.shape[0]))
        _check(load().bem_double_layer(self._h, _p(phi), phi.shape[0], _p(X), X.shape[0], _p(out)))
        return out

    def solve(self, g=None, rhs=None, precond=None, tol=1e-10, max_iter=2000, use_precond=True,
              precision=FP64, refresh_factor=0.0, check_every=0, use_graph=True, raise_on_error=True,
              device_out=None, x0=None):
        """Returns (phi[k][N], [info dict per column], status code).  With device_out (the address
        of k x N doubles in device memory) and g, bem_pcg_solve_dev: phi stays there and None is
        returned in its place.  x0: optional start vectors [k][N] (host)."""
        x0a = None if x0 is None else _f64(np.atleast_2d(x0))
        o = SolveOpts(tol, max_iter, int(use_precond), precision, refresh_factor, check_every, int(use_graph),
                      None if x0a is None else x0a.ctypes.data)
        L = load()
        m = precond.handle if precond is not None else None
        def _check_x0(k):
            if x0a is not None and x0a.shape != (k, self.N):
                raise ValueError("x0 must have shape (k, N)")
        if device_out is not None:
            g = _f64(np.atleast_2d(g))
            k = g.shape[0]
            _check_x0(k)
            info = (SolveInfo * k)()
            rc = L.bem_pcg_solve_dev(self._h, m, _p(g), k, ctypes.byref(o), ctypes.c_void_p(device_out), info)
            if raise_on_error and rc < 0:
                _check(rc)
            return None, [i.as_dict() for i in info], rc
        if g is not None:
            g = _f64(np.atleast_2d(g))
            k = g.shape[0]
            _check_x0(k)
            phi = np.empty((k, self.N))
            info = (SolveInfo * k)()
            rc = L.bem_pcg_solve(self._h, m, _p(g), k, ctypes.byref(o), _p(phi), info)
        else:
            rhs = _f64(np.atleast_2d(rhs))
            k = rhs.shape[0]
            _check_x0(k)
            phi = np.empty((k, self.N))
            info = (SolveInfo * k)()
            rc = L.bem_pcg_solve_rhs(self._h, m, _p(rhs), k, ctypes.byref(o), _p(phi), info)
        if raise_on_error and rc < 0:
            _check(rc)
        return phi, [i.as_dict() for i in info], rc

    def close(self):
        if self._h:
            load().bem_problem_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mesh_analyze_2d(V, S, coefficients=False):
    """Host-only segment-mesh analysis: dict(n_dofs, dof_vertex, dof_sector, q[, c[ns][2][N]])."""
    V, S = _f64(V), _i32a(S)
    n = ctypes.c_int64()
    _check(load().bem_mesh_analyze_2d(_p(V), V.shape[0], _p(S), S.shape[0], ctypes.byref(n), None, None, None, None))
    dv, ds, q = np.empty(n.value, np.int32), np.empty(n.value, np.int32), np.empty(V.shape[0], np.int32)
    c = np.empty((S.shape[0], 2, n.value)) if coefficients else None
    _check(load().bem_mesh_analyze_2d(_p(V), V.shape[0], _p(S), S.shape[0], ctypes.byref(n), _p(dv), _p(ds), _p(q),
                                      _p(c) if coefficients else None))
    out = {"n_dofs": n.value, "dof_vertex": dv, "dof_sector": ds, "q": q}
    if coefficients:
        out["c"] = c
    return out


class Problem2D(Problem):
    """bem_assemble_2d: a segment multiscreen in the plane (vertices nv x 2, segments ns x 2)."""

    def __init__(self, ctx: Context, V, S, precision=FP64):
        self.ctx = ctx
        self.V, self.T = _f64(V), _i32a(S)
        if self.V.shape[1] != 2 or self.T.shape[1] != 2:
            raise ValueError("vertices must be nv x 2 and segments ns x 2")
        o = AssembleOpts(precision, 0, 0, 0, 0)
        self._h = ctypes.c_void_p()
        _check(load().bem_assemble_2d(ctx.handle, _p(self.V), self.V.shape[0], _p(self.T), self.T.shape[0],
                                      ctypes.byref(o), ctypes.byref(self._h)))
        self.N = self.get_info()["n_dofs"]

    def solve(self, g=None, **kw):
        """As Problem.solve; g may be given as 2-vectors."""
        if g is not None:
            g = np.atleast_2d(np.asarray(g, dtype=np.float64))
            if g.shape[1] == 2:
                g = np.concatenate([g, np.zeros((g.shape[0], 1))], axis=1)
        return super().solve(g=g, **kw)

    def rhs(self, g):
        g = np.atleast_2d(np.asarray(g, dtype=np.float64))
        if g.shape[1] == 2:
            g = np.concatenate([g, np.zeros((g.shape[0], 1))], axis=1)
        return super().rhs(g)

    def double_layer(self, phi, targets):
        """U[k][m] at plane targets[m][2]."""
        X = np.atleast_2d(np.asarray(targets, dtype=np.float64))
        if X.shape[1] == 2:
            X = np.concatenate([X, np.zeros((X.shape[0], 1))], axis=1)
        return super().double_layer(phi, X)


class Preconditioner:
    def __init__(self, problem: Problem, patch_of_triangle, coarse_V=None, coarse_T=None, coarse_of_triangle=None,
                 use_coarse=True, factor_fp32=False, wirebasket="exact", diag_shift=0.0):
        self.problem = problem
        self.patch = _i32a(patch_of_triangle)
        if coarse_V is None:
            self.cV, self.cT, self.par = None, None, None
            ncv = nct = 0
        else:
            self.cV, self.cT, self.par = _f64(coarse_V), _i32a(coarse_T), _i32a(coarse_of_triangle)
            ncv, nct = self.cV.shape[0], self.cT.shape[0]
        if wirebasket not in ("exact", "diagonal"):
            raise ValueError("wirebasket must be 'exact' or 'diagonal'")
        o = PrecondOpts(int(use_coarse), int(factor_fp32), int(wirebasket == "diagonal"), float(diag_shift))
        self._h = ctypes.c_void_p()
        # a segment-mesh problem takes coarse vertices n x 2 and coarse segments, patch and parent
        # per segment
        setup = load().bem_precond_setup_2d if isinstance(problem, Problem2D) else load().bem_precond_setup
        _check(setup(problem.handle, _p(self.patch), _p(self.cV), ncv, _p(self.cT), nct,
                     _p(self.par), ctypes.byref(o), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def sizes(self):
        a, b, c, d = (ctypes.c_int64() for _ in range(4))
        _check(load().bem_precond_sizes(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return {"n_faces": a.value, "n_wb": b.value, "n_coarse": c.value, "max_face": d.value}

    def apply(self, r):
        r = _f64(np.atleast_2d(r))
        z = np.empty_like(r)
        _check(load().bem_precond_apply(self._h, _p(r), r.shape[0], _p(z)))
        return z

    def close(self):
        if self._h:
            load().bem_precond_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    def __init__(self, ctx: Context, max_inflight: int = 4):
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        _check(load().bem_server_create(ctx.handle, max_inflight, ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, V, T, patch, cV, cT, parent, g, precision=FP64, tol=1e-10):
        arrs = [_f64(V), _i32a(T), _i32a(patch), _f64(cV), _i32a(cT), _i32a(parent), _f64(np.atleast_2d(g))]
        r = Request(_p(arrs[0]), arrs[0].shape[0], _p(arrs[1]), arrs[1].shape[0], _p(arrs[2]), _p(arrs[3]),
                    arrs[3].shape[0], _p(arrs[4]), arrs[4].shape[0], _p(arrs[5]), _p(arrs[6]), arrs[6].shape[0],
                    precision, tol)
        t = ctypes.c_uint64()
        _check(load().bem_serve_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        n = ctypes.c_int64()
        _check(load().bem_serve_ndofs(self._h, t.value, ctypes.byref(n)))
        self._keep[t.value] = (arrs[6].shape[0], n.value)
        return t.value

    def poll(self, ticket, timeout_us=-1):
        k, n = self._keep[ticket]
        phi = np.empty((k, n))
        info = (SolveInfo * k)()
        rc = load().bem_serve_poll(self._h, ticket, timeout_us, _p(phi), info)
        if rc == BEM_PENDING:
            return None
        del self._keep[ticket]
        self.last_message = load().bem_last_error().decode() if rc < 0 else ""
        return phi, [i.as_dict() for i in info], rc

    def stats(self):
        s = ServerStats()
        _check(load().bem_server_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self._h:
            load().bem_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
