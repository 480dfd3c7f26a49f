"""Thin ctypes binding of librtsn (include/rtsn.h).

Argument marshalling only: every step of the method runs in the HIP
library.  Device vectors are torch CUDA tensors (PyTorch-ROCm keeps the
``cuda`` names) passed by ``data_ptr()``; streams are torch streams.  If the
library is not built, importing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtsn.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'`")

_lib = C.CDLL(LIB_PATH)

# enums (rtsn.h)
RT_OK, RT_NOT_CONVERGED = 0, 1
RT_E_INVALID, RT_E_NOMEM, RT_E_DEVICE = -1, -2, -3
RT_E_BREAKDOWN, RT_E_NONFINITE, RT_E_BUSY = -4, -5, -6
GEOM = {"slab": 0, "box": 1}
KERNEL = {"dipole_prd": 0, "explicit": 1}
FORMAL = {"linear_sc": 0, "implicit_euler": 1, "quadratic_sc": 2}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "bf16x3": 4}
RT_BATCH_BASIS_FP16 = 1
KRYLOV = {"gmres": 0, "bicgstab": 1}
SIGMA_FORM = {"dense": 0, "factored": 1, "ozaki": 2}
PRECOND = {"none": 0, "local": 1}

STATUS_NAMES = {0: "RT_OK", 1: "RT_NOT_CONVERGED", -1: "RT_E_INVALID", -2: "RT_E_NOMEM",
                -3: "RT_E_DEVICE", -4: "RT_E_BREAKDOWN", -5: "RT_E_NONFINITE",
                -6: "RT_E_BUSY"}

_dp = C.POINTER(C.c_double)


class ProblemDesc(C.Structure):
    _fields_ = [
        ("geom", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("depth", _dp), ("k_line", _dp),
        ("n_mu", C.c_int), ("n_az", C.c_int), ("n_nu", C.c_int),
        ("x_max", C.c_double), ("r", C.c_double),
        ("eps", C.c_double), ("eps_field", _dp),
        ("planck", C.c_double), ("planck_field", _dp),
        ("i_top", C.c_double), ("i_bot", C.c_double),
        ("kernel", C.c_int), ("kernel_matrix", _dp),
        ("coh_frac", C.c_double), ("coh_width2", C.c_double),
        ("formal", C.c_int),
        ("n_classes", C.c_int), ("point_class", C.POINTER(C.c_int32)),
        ("class_coh_frac", _dp), ("class_kernels", _dp),
    ]


class ProblemInfo(C.Structure):
    _fields_ = [("n_unknowns", C.c_int64), ("n_rays", C.c_int64), ("n_points", C.c_int64),
                ("bytes_problem", C.c_int64), ("bytes_solve_fp64", C.c_int64),
                ("bytes_solve_mixed", C.c_int64), ("sigma_rank", C.c_int32),
                ("sigma_form", C.c_int32)]


class SolverOpts(C.Structure):
    _fields_ = [("krylov", C.c_int), ("restart", C.c_int), ("max_iters", C.c_int),
                ("rtol", C.c_double), ("precision", C.c_int), ("inner_rtol", C.c_double),
                ("max_outer", C.c_int), ("record_history", C.c_int), ("basis_fp16", C.c_int),
                ("two_step", C.c_int), ("precond", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer_iters", C.c_int), ("converged", C.c_int),
                ("relres", C.c_double), ("ms", C.c_double), ("history_len", C.c_int),
                ("history", _dp)]


_vp = C.c_void_p
_sig = {
    "rt_problem_create": (C.c_int, [C.POINTER(ProblemDesc), C.c_int, C.POINTER(_vp)]),
    "rt_problem_destroy": (C.c_int, [_vp]),
    "rt_problem_footprint": (C.c_int, [_vp, C.c_int, C.POINTER(ProblemInfo)]),
    "rt_problem_tables": (C.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "rt_apply_lambda": (C.c_int, [_vp, C.c_int, _vp, _vp, C.c_int, _vp, _vp]),
    "rt_apply_sigma": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp]),
    "rt_apply_operator": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "rt_apply_operator_noalloc": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "rt_problem_set_sigma": (C.c_int, [_vp, C.c_int]),
    "rt_apply_precond": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "rt_precond_local": (C.c_int, [_vp, C.POINTER(C.c_double)]),
    "rt_rhs": (C.c_int, [_vp, _vp, _vp]),
    "rt_intensity": (C.c_int, [_vp, _vp, _vp, _vp]),
    "rt_solver_opts_default": (None, [C.POINTER(SolverOpts)]),
    "rt_solve": (C.c_int, [_vp, C.POINTER(SolverOpts), _vp, _vp, C.c_int,
                           C.POINTER(SolveStats), _vp]),
    "rt_batch_create": (C.c_int, [C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int,
                                  C.POINTER(_vp)]),
    "rt_batch_create_ex": (C.c_int, [C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int,
                                     C.c_int, C.POINTER(_vp)]),
    "rt_batch_info": (C.c_int, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_int64)]),
    "rt_batch_footprint": (C.c_int, [_vp, _vp, C.c_int, C.POINTER(C.c_int64)]),
    "rt_batch_submit": (C.c_int, [_vp, _vp, C.POINTER(SolverOpts), _vp,
                                  C.POINTER(C.c_uint64)]),
    "rt_batch_step": (C.c_int, [_vp, C.POINTER(C.c_int)]),
    "rt_batch_poll": (C.c_int, [_vp, C.c_uint64, C.POINTER(SolveStats)]),
    "rt_batch_wait_all": (C.c_int, [_vp]),
    "rt_batch_destroy": (C.c_int, [_vp]),
    "rt_profile_enable": (C.c_int, [C.c_int]),
    "rt_profile_read": (C.c_int, [C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.c_int]),
    "rt_gemm16_tile": (C.c_char_p, [_vp, C.c_int]),
    "rt_batch_gemm16_tile": (C.c_char_p, [_vp]),
    "rt_last_error": (C.c_char_p, []),
    "rt_version": (C.c_int, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class RtError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.rt_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code: int, where: str, allow=(RT_OK,)) -> int:
    if code not in allow:
        raise RtError(code, where)
    return code


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _darr(a):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return arr, arr.ctypes.data_as(_dp)


def version() -> int:
    return _lib.rt_version()


def default_opts() -> SolverOpts:
    o = SolverOpts()
    _lib.rt_solver_opts_default(C.byref(o))
    return o


class Problem:
    """Device-resident problem built from a spec object with the fields of
    ``rt_problem_desc`` (geom, nx, ny, nz, depth, k_line, n_mu, n_az, n_nu,
    x_max, r, eps, planck, i_top, i_bot, kernel, kernel_matrix, coh_frac,
    coh_width2, formal; optional point_class with class_coh_frac or
    class_kernels).  eps / planck may be scalars or per-point arrays."""

    def __init__(self, spec, device: int = 0):
        self._keep = []
        d = ProblemDesc()
        d.geom = GEOM[spec.geom]
        d.nx, d.ny, d.nz = int(spec.nx), int(spec.ny), int(spec.nz)
        if spec.geom == "slab":
            arr, p = _darr(spec.depth)
            self._keep.append(arr)
            d.depth = p
        else:
            arr, p = _darr(np.asarray(spec.k_line).reshape(-1))
            self._keep.append(arr)
            d.k_line = p
        d.n_mu, d.n_az, d.n_nu = int(spec.n_mu), int(spec.n_az), int(spec.n_nu)
        d.x_max, d.r = float(spec.x_max), float(spec.r)
        eps = np.asarray(spec.eps, dtype=np.float64)
        if eps.ndim == 0:
            d.eps = float(eps)
        else:
            arr, p = _darr(eps.reshape(-1))
            self._keep.append(arr)
            d.eps_field = p
        pl = np.asarray(spec.planck, dtype=np.float64)
        if pl.ndim == 0:
            d.planck = float(pl)
        else:
            arr, p = _darr(pl.reshape(-1))
            self._keep.append(arr)
            d.planck_field = p
        d.i_top, d.i_bot = float(spec.i_top), float(spec.i_bot)
        d.kernel = KERNEL[spec.kernel]
        if spec.kernel == "explicit":
            arr, p = _darr(np.asarray(spec.kernel_matrix).reshape(-1))
            self._keep.append(arr)
            d.kernel_matrix = p
        d.coh_frac, d.coh_width2 = float(spec.coh_frac), float(spec.coh_width2)
        d.formal = FORMAL[spec.formal]
        pc = getattr(spec, "point_class", None)
        if pc is not None:
            pcl = np.ascontiguousarray(np.asarray(pc).reshape(-1), dtype=np.int32)
            self._keep.append(pcl)
            d.point_class = pcl.ctypes.data_as(C.POINTER(C.c_int32))
            if spec.kernel == "explicit":
                arr, p = _darr(np.asarray(spec.class_kernels).reshape(-1))
                d.n_classes = int(np.asarray(spec.class_kernels).shape[0])
                self._keep.append(arr)
                d.class_kernels = p
            else:
                arr, p = _darr(np.asarray(spec.class_coh_frac).reshape(-1))
                d.n_classes = int(arr.size)
                self._keep.append(arr)
                d.class_coh_frac = p
        h = _vp()
        _check(_lib.rt_problem_create(C.byref(d), int(device), C.byref(h)), "rt_problem_create")
        self._keep = []
        self.handle = h
        self.device = device
        info = self.footprint(30)
        self.n = int(info.n_unknowns)
        self.n_r = int(info.n_rays)
        self.n_s = int(info.n_points)
        self.n_nu = int(spec.n_nu)

    # ------------------------------------------------------------------ info
    def footprint(self, restart: int = 30) -> ProblemInfo:
        info = ProblemInfo()
        _check(_lib.rt_problem_footprint(self.handle, int(restart), C.byref(info)),
               "rt_problem_footprint")
        return info

    def gemm16_tile(self, precision: str) -> str:
        """Tile shape of the 16-bit scattering GEMM for this problem."""
        return _lib.rt_gemm16_tile(self.handle, PREC[precision]).decode()

    def tables(self):
        nr = self.n_r
        mhat = np.zeros((nr, nr))
        mu = np.zeros(nr)
        w = np.zeros(nr)
        phi = np.zeros(nr)
        _check(_lib.rt_problem_tables(self.handle, mhat.ctypes.data_as(_dp),
                                      mu.ctypes.data_as(_dp), w.ctypes.data_as(_dp),
                                      phi.ctypes.data_as(_dp)), "rt_problem_tables")
        return dict(mhat=mhat, mu_ray=mu, w_ray=w, phi_ray=phi)

    # ------------------------------------------------------------- operators
    def apply_lambda(self, s, out, with_bc: bool = False, precision: str = "fp64",
                     scale=None, stream=None):
        _check(_lib.rt_apply_lambda(self.handle, PREC[precision], _ptr(s), _ptr(out),
                                    int(bool(with_bc)), _ptr(scale), _stream(stream)),
               "rt_apply_lambda")
        return out

    def apply_sigma(self, L, x, y, precision: str = "fp64", stream=None):
        _check(_lib.rt_apply_sigma(self.handle, PREC[precision], _ptr(L), _ptr(x), _ptr(y),
                                   _stream(stream)), "rt_apply_sigma")
        return y

    def apply(self, x, y, precision: str = "fp64", stream=None):
        _check(_lib.rt_apply_operator(self.handle, PREC[precision], _ptr(x), _ptr(y),
                                      _stream(stream)), "rt_apply_operator")
        return y

    def apply_noalloc(self, x, y, precision: str = "fp64", stream=None):
        """y = A x through rt_apply_operator_noalloc (FP64 / FP32, dense
        scattering form; no device allocation: the library's fixed per-GPU
        array holds Lambda x)."""
        _check(_lib.rt_apply_operator_noalloc(self.handle, PREC[precision], _ptr(x), _ptr(y),
                                              _stream(stream)), "rt_apply_operator_noalloc")
        return y

    def apply_precond(self, x, y, precision: str = "fp64", stream=None):
        """y = P^-1 x with the physics-based preconditioner (FP64 or FP32
        device vectors)."""
        _check(_lib.rt_apply_precond(self.handle, PREC[precision], _ptr(x), _ptr(y),
                                     _stream(stream)), "rt_apply_precond")
        return y

    def precond_local(self):
        """The preconditioner's direction-averaged plane response Dbar
        (n_nu x n_s, numpy)."""
        import numpy as np
        out = np.empty((self.n_nu, self.n_s), dtype=np.float64)
        _check(_lib.rt_precond_local(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))),
               "rt_precond_local")
        return out

    def set_sigma(self, form: str):
        """Scattering form of FP64 / FP32 applications: 'dense' (GEMM),
        'factored' (dipole x PRD kernels) or 'ozaki' (FP64 GEMM emulated
        with exact int8 products)."""
        _check(_lib.rt_problem_set_sigma(self.handle, SIGMA_FORM[form]), "rt_problem_set_sigma")

    def rhs(self, b, stream=None):
        _check(_lib.rt_rhs(self.handle, _ptr(b), _stream(stream)), "rt_rhs")
        return b

    def intensity(self, s, out, stream=None):
        _check(_lib.rt_intensity(self.handle, _ptr(s), _ptr(out), _stream(stream)),
               "rt_intensity")
        return out

    def solve(self, x, b=None, x_is_guess: bool = False, stream=None, **opts):
        """Solve A s = b (b None: physical rhs).  opts: krylov, restart,
        max_iters, rtol, precision, inner_rtol, max_outer, record_history,
        basis_fp16, two_step, precond ('none' or 'local').
        Returns a dict of solve statistics; raises on errors other than
        RT_NOT_CONVERGED."""
        o = default_opts()
        for k, v in opts.items():
            if k == "precision":
                v = PREC[v] if isinstance(v, str) else v
            if k == "krylov":
                v = KRYLOV[v] if isinstance(v, str) else v
            if k == "precond":
                v = PRECOND[v] if isinstance(v, str) else v
            setattr(o, k, v)
        st = SolveStats()
        code = _lib.rt_solve(self.handle, C.byref(o), _ptr(b), _ptr(x), int(bool(x_is_guess)),
                             C.byref(st), _stream(stream))
        _check(code, "rt_solve", allow=(RT_OK, RT_NOT_CONVERGED))
        hist = [st.history[i] for i in range(st.history_len)] if st.history_len else []
        return dict(status=STATUS_NAMES[code], iters=st.iters, outer_iters=st.outer_iters,
                    converged=bool(st.converged), relres=st.relres, ms=st.ms, history=hist)

    def close(self):
        if getattr(self, "handle", None):
            _lib.rt_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Batch / serving engine (rt_batch_*): many independent solves on one
    device, admitted by HBM footprint, advanced together."""

    def __init__(self, precision: str = "fp64", hbm_budget: int = 8 << 30,
                 max_slots: int = 512, queue_cap: int = 100000, use_graph: bool = True,
                 device: int = 0, basis_fp16: bool = False):
        h = _vp()
        _check(_lib.rt_batch_create_ex(int(device), PREC[precision], int(hbm_budget),
                                       int(max_slots), int(queue_cap), int(bool(use_graph)),
                                       RT_BATCH_BASIS_FP16 if basis_fp16 else 0, C.byref(h)),
               "rt_batch_create_ex")
        self.handle = h
        self.precision = precision
        self.basis_fp16 = bool(basis_fp16)

    def submit(self, problem: "Problem", x_out, **opts) -> int:
        o = default_opts()
        o.precision = PREC[self.precision]
        o.basis_fp16 = int(self.basis_fp16)
        for k, v in opts.items():
            if k == "precision":
                v = PREC[v] if isinstance(v, str) else v
            if k == "precond":
                v = PRECOND[v] if isinstance(v, str) else v
            setattr(o, k, v)
        t = C.c_uint64()
        _check(_lib.rt_batch_submit(self.handle, problem.handle, C.byref(o), _ptr(x_out),
                                    C.byref(t)), "rt_batch_submit")
        return int(t.value)

    def step(self) -> int:
        n = C.c_int()
        _check(_lib.rt_batch_step(self.handle, C.byref(n)), "rt_batch_step")
        return int(n.value)

    def poll(self, ticket: int):
        """None while pending, else a dict of solve statistics."""
        st = SolveStats()
        code = _lib.rt_batch_poll(self.handle, C.c_uint64(ticket), C.byref(st))
        if code == RT_E_BUSY:
            return None
        _check(code, "rt_batch_poll", allow=(RT_OK, RT_NOT_CONVERGED, RT_E_NONFINITE))
        hist = [st.history[i] for i in range(st.history_len)] if st.history_len else []
        return dict(status=STATUS_NAMES[code], iters=st.iters, outer_iters=st.outer_iters,
                    converged=bool(st.converged), relres=st.relres, ms=st.ms, history=hist)

    def wait_all(self):
        _check(_lib.rt_batch_wait_all(self.handle), "rt_batch_wait_all")

    def gemm16_tile(self) -> str:
        """Shape of the engine's grouped 16-bit GEMM (tile body, grid)."""
        return _lib.rt_batch_gemm16_tile(self.handle).decode()

    def footprint(self, problem: "Problem", restart: int = 30) -> int:
        b = C.c_int64()
        _check(_lib.rt_batch_footprint(self.handle, problem.handle, int(restart), C.byref(b)),
               "rt_batch_footprint")
        return int(b.value)

    def info(self):
        a, q, b = C.c_int(), C.c_int(), C.c_int64()
        _check(_lib.rt_batch_info(self.handle, C.byref(a), C.byref(q), C.byref(b)),
               "rt_batch_info")
        return dict(active=a.value, queued=q.value, bytes_in_use=b.value)

    def close(self):
        if getattr(self, "handle", None):
            _lib.rt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# kernel classes of rt_profile_read: the formal solver and the GEMM in FP64
# arithmetic, the Arnoldi kernels, and the formal solver and the GEMM in the
# lower precisions (FP32 sweeps, FP32 and 16-bit GEMMs)
KCLASS = {"lambda": 0, "sigma": 1, "arnoldi": 2, "lambda_lo": 3, "sigma_lo": 4,
          "precond": 5}


def profile_enable(on: bool = True) -> None:
    _check(_lib.rt_profile_enable(int(bool(on))), "rt_profile_enable")


def profile_read(kclass: str, reset: bool = True):
    """(launches, total device ms) of one kernel class since the last reset."""
    n = C.c_int64()
    ms = C.c_double()
    _check(_lib.rt_profile_read(KCLASS[kclass], C.byref(n), C.byref(ms), int(reset)),
           "rt_profile_read")
    return int(n.value), float(ms.value)


def lib_path() -> str:
    return LIB_PATH


def raw_lib():
    return _lib
