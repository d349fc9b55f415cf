"""ctypes binding of libkfbi.so (the gfx950 KFBI library).  Argument marshalling only:
every numerical step runs in the library's HIP kernels.  Tensors are torch CUDA (HIP)
tensors; their data pointers are passed straight to the C ABI declared in include/kfbi.h.

The library is built in-tree by ``paper_2309_01068_amd.build``; if it is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libkfbi.so")

OK, E_INVALID, E_GEOMETRY, E_NOCONV, E_HIP, E_NOMEM, E_NONFINITE, E_STATE = range(8)
SINGLE, DOUBLE = 0, 1
PLUS, MINUS, AVG = 0, 1, 2
BOX_ZERO, BOX_USER, BOX_FREESPACE, BOX_NEUMANN = 0, 1, 2, 3
FP64, FP32, MIXED = 0, 1, 2

EXPORTS = [
    "kfbi_last_error", "kfbi_create", "kfbi_destroy", "kfbi_set_interface", "kfbi_get_info",
    "kfbi_apply", "kfbi_apply_batch", "kfbi_operator", "kfbi_gmres_solve", "kfbi_gmres_solve_static",
    "kfbi_profile", "kfbi_profile_read",
    "kfbi_profile_kernel",
    "thetaL_create", "thetaL_destroy", "thetaL_init", "thetaL_step", "thetaL_run",
    "thetaL_markers", "thetaL_density", "thetaL_kfbi", "thetaL_get_state", "thetaL_set_state",
    "thetaL_size",
    "kfbi_ws_create", "kfbi_ws_destroy", "kfbi_ws_n_params", "kfbi_ws_get_weights",
    "kfbi_ws_set_weights", "kfbi_ws_predict", "kfbi_ws_record", "kfbi_ws_n_samples",
    "kfbi_ws_clear", "kfbi_ws_train", "kfbi_ws_eval", "kfbi_ws_forward", "kfbi_ws_backward",
    "kfbi_ws_target_scale",
    "stefan_create", "stefan_destroy", "stefan_init", "stefan_step", "stefan_run",
    "stefan_temperature", "stefan_markers", "stefan_density", "stefan_interface",
    "stefan_constants", "stefan_size", "stefan_thetal",
    "stokes_create", "stokes_destroy", "stokes_set_interface", "stokes_apply", "stokes_fields",
    "stokes_operator", "stokes_gmres_solve", "stokes_get_info",
]


class KfbiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"kfbi error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("side", C.c_double), ("N", C.c_int),
                ("c2", C.c_double), ("box_bc", C.c_int), ("max_markers", C.c_int),
                ("stream", C.c_void_p), ("max_batch", C.c_int)]


class Info(C.Structure):
    _fields_ = [("M", C.c_int), ("n_cross_h", C.c_int), ("n_cross_v", C.c_int),
                ("n_arms", C.c_int), ("n_nodes", C.c_int), ("n_rows", C.c_int),
                ("row_lo", C.c_int), ("row_hi", C.c_int), ("n_parts", C.c_int),
                ("sub_batch", C.c_int), ("workspace_bytes", C.c_longlong)]


class Out(C.Structure):
    _fields_ = [("v_plus", C.c_void_p), ("v_minus", C.c_void_p), ("dn_plus", C.c_void_p),
                ("dn_minus", C.c_void_p), ("grid", C.c_void_p)]


class Bie(C.Structure):
    _fields_ = [("layer", C.c_int), ("side", C.c_int), ("a", C.c_double), ("b", C.c_double),
                ("q", C.c_double), ("a_marker", C.c_void_p)]


class GmresOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("maxit", C.c_int),
                ("precision", C.c_int), ("inner_tol", C.c_double)]


class GmresStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer_iters", C.c_int), ("applies64", C.c_int),
                ("applies32", C.c_int), ("relres", C.c_double), ("converged", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class StokesParams(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("side", C.c_double), ("N", C.c_int),
                ("c2", C.c_double), ("max_markers", C.c_int), ("stream", C.c_void_p),
                ("solve_tol", C.c_double), ("solve_maxit", C.c_int)]


class StokesInfo(C.Structure):
    _fields_ = [("M", C.c_int), ("n_crossings", C.c_int), ("cg_iters", C.c_int),
                ("cg_relres", C.c_double)]


class ThetaLParams(C.Structure):
    _fields_ = [("grid", Grid), ("M", C.c_int), ("sigma", C.c_double), ("J", C.c_double),
                ("tau", C.c_double), ("lambda2", C.c_double), ("gmres", GmresOpts),
                ("refine", C.c_double), ("max_M", C.c_int)]


class ThetaLStats(C.Structure):
    _fields_ = [("step", C.c_int), ("t", C.c_double), ("iters", C.c_int), ("applies64", C.c_int),
                ("applies32", C.c_int), ("relres", C.c_double), ("area", C.c_double),
                ("length", C.c_double), ("ms_geometry", C.c_double), ("ms_gmres", C.c_double),
                ("ms_apply", C.c_double), ("ms_update", C.c_double), ("M", C.c_int),
                ("M_next", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ThetaLState(C.Structure):
    _fields_ = [("eta_dev", C.c_void_p), ("phi_prev_dev", C.c_void_p),
                ("phi_prev2_dev", C.c_void_p), ("nhat_prev_dev", C.c_void_p),
                ("scal", C.c_double * 8), ("n", C.c_int), ("M", C.c_int)]


class StefanAniso(C.Structure):
    _fields_ = [("e0", C.c_double), ("e1", C.c_double), ("e2", C.c_double), ("m", C.c_int),
                ("phi0", C.c_double)]


class StefanParams(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("side", C.c_double), ("N", C.c_int),
                ("M", C.c_int), ("tau", C.c_double), ("bdf2", C.c_int), ("ssd", C.c_int),
                ("lambda_", C.c_double), ("eps_c", StefanAniso), ("eps_v", StefanAniso),
                ("gmres", GmresOpts), ("stream", C.c_void_p), ("refine", C.c_double),
                ("max_M", C.c_int)]


class StefanStats(C.Structure):
    _fields_ = [("step", C.c_int), ("t", C.c_double), ("iters", C.c_int), ("applies64", C.c_int),
                ("applies32", C.c_int), ("relres", C.c_double), ("area", C.c_double),
                ("length", C.c_double), ("ms_geometry", C.c_double),
                ("ms_temperature", C.c_double), ("ms_gmres", C.c_double),
                ("ms_update", C.c_double), ("M", C.c_int), ("M_next", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class WsCfg(C.Structure):
    _fields_ = [("M", C.c_int), ("max_batch", C.c_int), ("capacity", C.c_int),
                ("L_ref", C.c_double), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_ulonglong),
                ("target_scale", C.c_double), ("stream", C.c_void_p)]


_lib = None


def load(path: str = LIBPATH):
    """Load libkfbi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2309_01068_amd.build`")
    lib = C.CDLL(path)
    lib.kfbi_last_error.restype = C.c_char_p
    vp = C.c_void_p
    lib.kfbi_create.argtypes = [C.POINTER(Grid), C.POINTER(vp)]
    lib.kfbi_destroy.argtypes = [vp]
    lib.kfbi_set_interface.argtypes = [vp, C.c_int, vp]
    lib.kfbi_get_info.argtypes = [vp, C.POINTER(Info)]
    lib.kfbi_apply.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.POINTER(Out)]
    lib.kfbi_apply_batch.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp, C.POINTER(Out)]
    lib.kfbi_operator.argtypes = [vp, C.POINTER(Bie), C.c_int, vp, vp]
    lib.kfbi_gmres_solve.argtypes = [vp, C.POINTER(Bie), vp, vp, C.POINTER(GmresOpts),
                                     C.POINTER(GmresStats)]
    lib.kfbi_gmres_solve_static.argtypes = [vp, C.POINTER(Bie), vp, vp, C.POINTER(GmresOpts),
                                            C.POINTER(GmresStats)]
    lib.kfbi_profile.argtypes = [vp, C.c_int]
    lib.kfbi_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_long)]
    lib.kfbi_profile_kernel.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_double)]
    lib.thetaL_create.argtypes = [C.POINTER(ThetaLParams), C.POINTER(vp)]
    lib.thetaL_destroy.argtypes = [vp]
    lib.thetaL_init.argtypes = [vp, C.c_int, vp]
    lib.thetaL_step.argtypes = [vp, vp, C.POINTER(ThetaLStats)]
    lib.thetaL_run.argtypes = [vp, C.c_int, C.POINTER(ThetaLStats)]
    lib.thetaL_markers.argtypes = [vp, vp]
    lib.thetaL_density.argtypes = [vp, vp]
    lib.thetaL_kfbi.argtypes = [vp]
    lib.thetaL_kfbi.restype = vp
    lib.thetaL_get_state.argtypes = [vp, C.POINTER(ThetaLState)]
    lib.thetaL_set_state.argtypes = [vp, C.POINTER(ThetaLState)]
    lib.thetaL_size.argtypes = [vp, C.POINTER(C.c_int)]
    lib.stefan_create.argtypes = [C.POINTER(StefanParams), C.POINTER(vp)]
    lib.stefan_destroy.argtypes = [vp]
    lib.stefan_init.argtypes = [vp, C.c_int, vp, vp, C.c_double]
    lib.stefan_step.argtypes = [vp, vp, C.POINTER(StefanStats)]
    lib.stefan_run.argtypes = [vp, C.c_int, C.POINTER(StefanStats)]
    lib.stefan_temperature.argtypes = [vp, vp]
    lib.stefan_markers.argtypes = [vp, vp]
    lib.stefan_density.argtypes = [vp, vp]
    lib.stefan_interface.argtypes = [vp, vp, C.POINTER(C.c_double)]
    lib.stefan_constants.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.stefan_size.argtypes = [vp, C.POINTER(C.c_int)]
    lib.stefan_thetal.argtypes = [vp]
    lib.stefan_thetal.restype = vp
    lib.stokes_create.argtypes = [C.POINTER(StokesParams), C.POINTER(vp)]
    lib.stokes_destroy.argtypes = [vp]
    lib.stokes_set_interface.argtypes = [vp, C.c_int, vp]
    lib.stokes_apply.argtypes = [vp, vp, vp, vp]
    lib.stokes_fields.argtypes = [vp, vp, vp, vp]
    lib.stokes_operator.argtypes = [vp, vp, vp]
    lib.stokes_gmres_solve.argtypes = [vp, vp, vp, C.POINTER(GmresOpts), C.POINTER(GmresStats)]
    lib.stokes_get_info.argtypes = [vp, C.POINTER(StokesInfo)]
    ip, fp = C.POINTER(C.c_int), C.POINTER(C.c_float)
    lib.kfbi_ws_create.argtypes = [C.POINTER(WsCfg), C.POINTER(vp)]
    lib.kfbi_ws_destroy.argtypes = [vp]
    lib.kfbi_ws_n_params.argtypes = [vp, ip]
    lib.kfbi_ws_get_weights.argtypes = [vp, fp]
    lib.kfbi_ws_set_weights.argtypes = [vp, fp]
    lib.kfbi_ws_predict.argtypes = [vp, vp, vp]
    lib.kfbi_ws_record.argtypes = [vp, vp, ip]
    lib.kfbi_ws_n_samples.argtypes = [vp, ip]
    lib.kfbi_ws_clear.argtypes = [vp]
    lib.kfbi_ws_train.argtypes = [vp, C.c_int, C.c_int, C.c_int, fp]
    lib.kfbi_ws_eval.argtypes = [vp, C.c_int, C.c_int, fp]
    lib.kfbi_ws_forward.argtypes = [vp, C.c_int, vp, vp]
    lib.kfbi_ws_backward.argtypes = [vp, C.c_int, vp, vp, vp, fp]
    lib.kfbi_ws_target_scale.argtypes = [vp, C.POINTER(C.c_double)]
    _lib = lib
    return lib


def _check(code: int):
    if code != OK:
        raise KfbiError(code, load().kfbi_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


class Context:
    """A KFBI context: box, grid, operator constant c2, box data mode."""

    def __init__(self, x0, y0, side, N, c2=0.0, box_bc=BOX_ZERO, max_markers=4096, stream=None,
                 max_batch=1):
        self.lib = load()
        self.N = N
        self.box_bc = box_bc
        s = torch.cuda.current_stream() if stream is None else stream
        self.stream = s
        g = Grid(x0, y0, side, N, c2, box_bc, max_markers, C.c_void_p(s.cuda_stream), max_batch)
        h = C.c_void_p()
        _check(self.lib.kfbi_create(C.byref(g), C.byref(h)))
        self.h = h
        self.M = 0

    def close(self):
        if self.h:
            self.lib.kfbi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_interface(self, xy: torch.Tensor):
        """xy: (2, M) float64 device tensor (x row then y row)."""
        xy = xy.contiguous()
        self.M = xy.shape[1]
        _check(self.lib.kfbi_set_interface(self.h, self.M, _ptr(xy)))

    def info(self) -> dict:
        i = Info()
        _check(self.lib.kfbi_get_info(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def apply(self, layer, density, precision=FP64, ring=None, want=("v_plus", "v_minus",
                                                                       "dn_plus", "dn_minus"),
              grid=False, out=None):
        dev = density.device
        res = {} if out is None else out
        for k in want:
            if k not in res:
                res[k] = torch.empty(self.M, dtype=torch.float64, device=dev)
        if grid and "grid" not in res:
            res["grid"] = torch.empty((self.N + 1, self.N + 1), dtype=torch.float64, device=dev)
        o = Out(*[(_ptr(res[k]) if k in res else None)
                  for k in ("v_plus", "v_minus", "dn_plus", "dn_minus", "grid")])
        _check(self.lib.kfbi_apply(self.h, layer, precision, _ptr(density), _ptr(ring), C.byref(o)))
        return res

    def apply_batch(self, layer, density, precision=FP64, ring=None,
                    want=("v_plus", "v_minus", "dn_plus", "dn_minus"), out=None):
        """density: (B, M) float64 device tensor; outputs (B, M); ring (B, 4(N+1)) or None."""
        B = density.shape[0]
        res = {} if out is None else out
        for k in want:
            if k not in res:
                res[k] = torch.empty((B, self.M), dtype=torch.float64, device=density.device)
        o = Out(*[(_ptr(res[k]) if k in res else None)
                  for k in ("v_plus", "v_minus", "dn_plus", "dn_minus")], None)
        _check(self.lib.kfbi_apply_batch(self.h, layer, precision, B, _ptr(density), _ptr(ring),
                                         C.byref(o)))
        return res

    @staticmethod
    def _bie(layer, side, a, b, q):
        """a: a number, or a float64 device tensor of M per-marker values."""
        if torch.is_tensor(a):
            return Bie(layer, side, 0.0, b, q, _ptr(a))
        return Bie(layer, side, a, b, q, None)

    def operator(self, x, layer, side, a, b, q, precision=FP64, y=None):
        y = torch.empty_like(x) if y is None else y
        op = self._bie(layer, side, a, b, q)
        _check(self.lib.kfbi_operator(self.h, C.byref(op), precision, _ptr(x), _ptr(y)))
        return y

    def profile(self, on: bool):
        _check(self.lib.kfbi_profile(self.h, 1 if on else 0))

    def profile_read(self):
        """(ms summed per stage [4], number of profiled applies)."""
        ms = (C.c_double * 4)()
        n = C.c_long()
        _check(self.lib.kfbi_profile_read(self.h, ms, C.byref(n)))
        return list(ms), n.value

    def profile_kernel(self, stage, reps=200):
        """Average duration (us) of kernel `stage` of the last apply, replayed back to back."""
        us = C.c_double()
        _check(self.lib.kfbi_profile_kernel(self.h, stage, reps, C.byref(us)))
        return us.value

    def gmres(self, rhs, x, layer, side, a, b, q, tol=1e-10, restart=50, maxit=1000,
              precision=FP64, inner_tol=1e-5, raise_noconv=True, static_workspace=False):
        """kfbi_gmres_solve, or kfbi_gmres_solve_static (the Krylov workspace in the
        library's static device array, no allocation) with static_workspace=True."""
        op = self._bie(layer, side, a, b, q)
        opts = GmresOpts(tol, restart, maxit, precision, inner_tol)
        st = GmresStats()
        fn = self.lib.kfbi_gmres_solve_static if static_workspace else self.lib.kfbi_gmres_solve
        code = fn(self.h, C.byref(op), _ptr(rhs), _ptr(x), C.byref(opts), C.byref(st))
        if code == E_NOCONV and not raise_noconv:
            return x, st.as_dict()
        _check(code)
        return x, st.as_dict()


class ThetaL:
    """theta-L / SSD Hele-Shaw evolution (include/thetal.h) on the current torch stream."""

    def __init__(self, x0, y0, side, N, M, sigma, J, tau, lambda2=-1.0, tol=1e-10, restart=50,
                 maxit=1000, precision=FP64, inner_tol=1e-5, stream=None, refine=0.0, max_M=0):
        self.lib = load()
        s = torch.cuda.current_stream() if stream is None else stream
        self.stream = s
        g = Grid(x0, y0, side, N, 0.0, BOX_FREESPACE, M, C.c_void_p(s.cuda_stream))
        p = ThetaLParams(g, M, sigma, J, tau, lambda2,
                         GmresOpts(tol, restart, maxit, precision, inner_tol), refine, max_M)
        h = C.c_void_p()
        _check(self.lib.thetaL_create(C.byref(p), C.byref(h)))
        self.h = h

    @property
    def M(self) -> int:
        """Current number of markers (refinement doubles it)."""
        m = C.c_int()
        _check(self.lib.thetaL_size(self.h, C.byref(m)))
        return m.value

    def close(self):
        if self.h:
            self.lib.thetaL_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, xy: torch.Tensor):
        xy = xy.contiguous()
        _check(self.lib.thetaL_init(self.h, xy.shape[1], _ptr(xy)))

    def step(self, x0=None) -> dict:
        st = ThetaLStats()
        _check(self.lib.thetaL_step(self.h, _ptr(x0), C.byref(st)))
        return st.as_dict()

    def run(self, nsteps: int) -> list:
        arr = (ThetaLStats * max(nsteps, 1))()
        _check(self.lib.thetaL_run(self.h, nsteps, arr))
        return [arr[i].as_dict() for i in range(nsteps)]

    def markers(self) -> torch.Tensor:
        xy = torch.empty((2, self.M), dtype=torch.float64, device="cuda")
        _check(self.lib.thetaL_markers(self.h, _ptr(xy)))
        return xy

    def density(self) -> torch.Tensor:
        phi = torch.empty(self.M, dtype=torch.float64, device="cuda")
        _check(self.lib.thetaL_density(self.h, _ptr(phi)))
        return phi

    def get_state(self) -> dict:
        eta = torch.empty(self.M, dtype=torch.float64, device="cuda")
        phi = torch.empty(self.M, dtype=torch.float64, device="cuda")
        phi2 = torch.empty(self.M, dtype=torch.float64, device="cuda")
        nh = torch.empty(2 * self.M, dtype=torch.float64, device="cuda")
        st = ThetaLState(C.c_void_p(eta.data_ptr()), C.c_void_p(phi.data_ptr()),
                         C.c_void_p(phi2.data_ptr()), C.c_void_p(nh.data_ptr()))
        _check(self.lib.thetaL_get_state(self.h, C.byref(st)))
        return {"eta": eta, "phi_prev": phi, "phi_prev2": phi2, "nhat_prev": nh,
                "scal": list(st.scal), "n": st.n, "M": st.M}

    def set_state(self, d: dict):
        st = ThetaLState(_ptr(d["eta"]), _ptr(d["phi_prev"]), _ptr(d["phi_prev2"]),
                         _ptr(d["nhat_prev"]))
        for i in range(8):
            st.scal[i] = d["scal"][i]
        st.n = d["n"]
        st.M = d.get("M", d["eta"].numel())
        _check(self.lib.thetaL_set_state(self.h, C.byref(st)))


class Stefan:
    """Stefan problem (include/stefan.h) on the current torch stream.  eps_c, eps_v:
    (e0, e1, e2, m, phi0) of eps(phi) = e0 (1 + e1 cos(m (phi - phi0)) + e2 cos(2 m (phi - phi0)))."""

    def __init__(self, x0, y0, side, N, M, tau, eps_c, eps_v, bdf2=True, ssd=2, lam=0.0,
                 tol=1e-10, restart=50, maxit=1000, precision=FP64, inner_tol=1e-5, stream=None,
                 refine=0.0, max_M=0):
        self.lib = load()
        s = torch.cuda.current_stream() if stream is None else stream
        self.stream = s
        self.N = N
        p = StefanParams(x0, y0, side, N, M, tau, 1 if bdf2 else 0, ssd, lam,
                         StefanAniso(*eps_c), StefanAniso(*eps_v),
                         GmresOpts(tol, restart, maxit, precision, inner_tol),
                         C.c_void_p(s.cuda_stream), refine, max_M)
        h = C.c_void_p()
        _check(self.lib.stefan_create(C.byref(p), C.byref(h)))
        self.h = h

    @property
    def M(self) -> int:
        m = C.c_int()
        _check(self.lib.stefan_size(self.h, C.byref(m)))
        return m.value

    @property
    def thetal(self):
        """A ThetaL-like view of the interface state for WarmStart.predict / record."""
        return _ThetaLView(self.lib.stefan_thetal(self.h))

    def close(self):
        if self.h:
            self.lib.stefan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, xy: torch.Tensor, T0: torch.Tensor | None = None, St: float = 0.0):
        xy = xy.contiguous()
        _check(self.lib.stefan_init(self.h, xy.shape[1], _ptr(xy),
                                    None if T0 is None else _ptr(T0.contiguous()), St))

    def step(self, x0=None) -> dict:
        st = StefanStats()
        _check(self.lib.stefan_step(self.h, _ptr(x0), C.byref(st)))
        return st.as_dict()

    def run(self, nsteps: int) -> list:
        arr = (StefanStats * max(nsteps, 1))()
        _check(self.lib.stefan_run(self.h, nsteps, arr))
        return [arr[i].as_dict() for i in range(nsteps)]

    def temperature(self) -> torch.Tensor:
        g = torch.empty((self.N + 1, self.N + 1), dtype=torch.float64, device="cuda")
        _check(self.lib.stefan_temperature(self.h, _ptr(g)))
        return g

    def markers(self) -> torch.Tensor:
        xy = torch.empty((2, self.M), dtype=torch.float64, device="cuda")
        _check(self.lib.stefan_markers(self.h, _ptr(xy)))
        return xy

    def density(self) -> torch.Tensor:
        psi = torch.empty(self.M, dtype=torch.float64, device="cuda")
        _check(self.lib.stefan_density(self.h, _ptr(psi)))
        return psi

    def interface(self):
        eta = torch.empty(self.M, dtype=torch.float64, device="cuda")
        sc = (C.c_double * 4)()
        _check(self.lib.stefan_interface(self.h, _ptr(eta), sc))
        return eta, list(sc)

    def constants(self):
        lam, c2 = C.c_double(), C.c_double()
        _check(self.lib.stefan_constants(self.h, C.byref(lam), C.byref(c2)))
        return lam.value, c2.value


class Stokes:
    """Modified Stokes double-layer operator on the MAC grid (include/stokes.h) on the
    current torch stream."""

    def __init__(self, x0, y0, side, N, c2, max_markers=2048, tol=1e-13, maxit=500, stream=None):
        self.lib = load()
        s = torch.cuda.current_stream() if stream is None else stream
        self.stream = s
        self.N = N
        p = StokesParams(x0, y0, side, N, c2, max_markers, C.c_void_p(s.cuda_stream), tol, maxit)
        h = C.c_void_p()
        _check(self.lib.stokes_create(C.byref(p), C.byref(h)))
        self.h = h
        self.M = 0

    def close(self):
        if self.h:
            self.lib.stokes_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_interface(self, xy: torch.Tensor):
        xy = xy.contiguous()
        _check(self.lib.stokes_set_interface(self.h, xy.shape[1], _ptr(xy)))
        self.M = xy.shape[1]

    def apply(self, phi: torch.Tensor):
        """Traces of D phi from inside and outside, each (2, M)."""
        phi = phi.contiguous()
        up = torch.empty((2, self.M), dtype=torch.float64, device="cuda")
        um = torch.empty_like(up)
        _check(self.lib.stokes_apply(self.h, _ptr(phi), _ptr(up), _ptr(um)))
        return up, um

    def fields(self):
        N = self.N
        u = torch.empty((N, N + 1), dtype=torch.float64, device="cuda")
        v = torch.empty((N + 1, N), dtype=torch.float64, device="cuda")
        p = torch.empty((N, N), dtype=torch.float64, device="cuda")
        _check(self.lib.stokes_fields(self.h, _ptr(u), _ptr(v), _ptr(p)))
        return u, v, p

    def operator(self, x: torch.Tensor, y: torch.Tensor | None = None):
        y = torch.empty_like(x) if y is None else y
        _check(self.lib.stokes_operator(self.h, _ptr(x), _ptr(y)))
        return y

    def gmres(self, rhs, x, tol=1e-10, restart=50, maxit=500):
        opts = GmresOpts(tol, restart, maxit, FP64, 0.0)
        st = GmresStats()
        _check(self.lib.stokes_gmres_solve(self.h, _ptr(rhs), _ptr(x), C.byref(opts), C.byref(st)))
        return x, st.as_dict()

    def info(self) -> dict:
        i = StokesInfo()
        _check(self.lib.stokes_get_info(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in i._fields_}


class _ThetaLView:
    """The theta-L state owned by a Stefan object (not destroyed through this handle)."""

    def __init__(self, h):
        self.h = C.c_void_p(h)


def _fptr(t):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 device tensor")
    return C.c_void_p(t.data_ptr())


class WarmStart:
    """Learned GMRES initial guess for a ThetaL evolution (include/warmstart.h)."""

    def __init__(self, M, max_batch=64, capacity=16384, L_ref=2 * 3.141592653589793, lr=1e-3,
                 beta1=0.9, beta2=0.999, eps=1e-8, seed=0, target_scale=0.0, stream=None):
        self.lib = load()
        s = torch.cuda.current_stream() if stream is None else stream
        cfg = WsCfg(M, max_batch, capacity, L_ref, lr, beta1, beta2, eps, seed, target_scale,
                    C.c_void_p(s.cuda_stream))
        h = C.c_void_p()
        _check(self.lib.kfbi_ws_create(C.byref(cfg), C.byref(h)))
        self.h = h
        self.M = M
        n = C.c_int()
        _check(self.lib.kfbi_ws_n_params(self.h, C.byref(n)))
        self.n_params = n.value

    def close(self):
        if self.h:
            self.lib.kfbi_ws_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self):
        import numpy as np
        w = np.empty(self.n_params, dtype=np.float32)
        _check(self.lib.kfbi_ws_get_weights(self.h, w.ctypes.data_as(C.POINTER(C.c_float))))
        return w

    def set_weights(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == self.n_params
        _check(self.lib.kfbi_ws_set_weights(self.h, w.ctypes.data_as(C.POINTER(C.c_float))))

    def predict(self, th, x0=None):
        """Initial guess for the next step of th (x0 None: features only, no guess)."""
        _check(self.lib.kfbi_ws_predict(self.h, th.h, _ptr(x0)))
        return x0

    def record(self, th) -> bool:
        st = C.c_int()
        _check(self.lib.kfbi_ws_record(self.h, th.h, C.byref(st)))
        return bool(st.value)

    def target_scale(self) -> float:
        v = C.c_double()
        _check(self.lib.kfbi_ws_target_scale(self.h, C.byref(v)))
        return v.value

    def n_samples(self) -> int:
        n = C.c_int()
        _check(self.lib.kfbi_ws_n_samples(self.h, C.byref(n)))
        return n.value

    def clear(self):
        _check(self.lib.kfbi_ws_clear(self.h))

    def train(self, n_train, epochs, batch):
        losses = (C.c_float * max(epochs, 1))()
        _check(self.lib.kfbi_ws_train(self.h, n_train, epochs, batch, losses))
        return [losses[i] for i in range(epochs)]

    def eval(self, first, count):
        v = C.c_float()
        _check(self.lib.kfbi_ws_eval(self.h, first, count, C.byref(v)))
        return v.value

    def forward(self, feat):
        """feat: (B, M, 5) float32 device tensor -> (B, M) float32."""
        feat = feat.contiguous()
        out = torch.empty(feat.shape[:2], dtype=torch.float32, device=feat.device)
        _check(self.lib.kfbi_ws_forward(self.h, feat.shape[0], _fptr(feat), _fptr(out)))
        return out

    def backward(self, feat, target):
        feat, target = feat.contiguous(), target.contiguous()
        g = torch.empty(self.n_params, dtype=torch.float32, device=feat.device)
        loss = C.c_float()
        _check(self.lib.kfbi_ws_backward(self.h, feat.shape[0], _fptr(feat), _fptr(target),
                                         _fptr(g), C.byref(loss)))
        return loss.value, g
