"""MI355X two-grid algebraic multiscale preconditioner (HIP, gfx950).

Thin ctypes binding over the C ABI in include/amsp.h: it only marshals
arguments.  Every step of setup, apply and PCG runs in the HIP kernels of
libamsp.so; PyTorch tensors provide device memory and the HIP stream.  There
is no CPU fallback: importing this package fails loudly when the library is
missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamsp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2606_04864_amd/build.py` "
                      "(hipcc --offload-arch=gfx950)")
# PyTorch-ROCm ships its own HIP/HSA runtime with the same soname as the
# system one.  Loading torch first makes libamsp.so bind to that runtime, so
# the process holds a single HSA instance that sees the GPU.
try:
    import torch as _torch_preload  # noqa: F401
except ImportError:  # host-only use (planning, error codes) needs no torch
    _torch_preload = None
_lib = ctypes.CDLL(LIB_PATH)

# status codes
AMSP_OK = 0
STATUS = {0: "AMSP_OK", -1: "AMSP_ERR_ARG", -2: "AMSP_ERR_CSR", -3: "AMSP_ERR_NONSYM",
          -4: "AMSP_ERR_PARTITION", -5: "AMSP_ERR_NEUMANN_DIAG", -6: "AMSP_ERR_LOCAL_NOT_SPD",
          -7: "AMSP_ERR_EIG_NOCONV", -8: "AMSP_ERR_COARSE_NOT_SPD", -9: "AMSP_ERR_PCG_NOCONV",
          -10: "AMSP_ERR_BREAKDOWN", -11: "AMSP_ERR_HIP", -12: "AMSP_ERR_OOM"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}
ORDER = {"rcm": 0, "natural": 1}


class AmspError(RuntimeError):
    """A non-OK status.  result holds what the call still wrote where the
    library documents it (a CG breakdown in some columns or recurrences:
    the same tuple the call returns on success), else None."""

    def __init__(self, code: int, msg: str, result=None):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))
        self.msg = msg
        self.result = result


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


# PCG kernel classes of amsp_info.kernel_ms / the timing bit mask
KERNEL_CLASS = {"spmv": 0, "local": 1, "coarse": 2, "scatter": 3, "vector": 4}


class _Options(ctypes.Structure):
    _fields_ = [("overlap", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("pou", ctypes.c_int32), ("local_order", ctypes.c_int32),
                ("dense_tiles", ctypes.c_int32), ("eig_tol", ctypes.c_double),
                ("eig_maxit", ctypes.c_int32), ("eig_shift", ctypes.c_double),
                ("chunk", ctypes.c_int32), ("flexible", ctypes.c_int32),
                ("keep_a0", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("timing_stride", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("singular", ctypes.c_int32), ("cycle", ctypes.c_int32),
                ("smoother_weight", ctypes.c_double), ("coarse_basis", ctypes.c_int32),
                ("coarse_solver", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("relres_recursive", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("restarts", ctypes.c_int32), ("solve_ms", ctypes.c_double),
                ("bytes_per_iter", ctypes.c_int64), ("kernel_ms", ctypes.c_double * 5),
                ("kernel_launches", ctypes.c_int32 * 5), ("local_apply_bytes", ctypes.c_int64),
                ("relres_floor", ctypes.c_double), ("first_segment", ctypes.c_int32)]


class _SetupInfo(ctypes.Structure):
    _fields_ = [("nsub", ctypes.c_int32), ("nc", ctypes.c_int32), ("sum_ni", ctypes.c_int64),
                ("max_ni", ctypes.c_int32), ("factor_tiles", ctypes.c_int64),
                ("eig_sweeps", ctypes.c_int32), ("eig_unconverged", ctypes.c_int32),
                ("n_gap_flags", ctypes.c_int32), ("mu_c", ctypes.c_double),
                ("phase_ms", ctypes.c_double * 8), ("coupling_ms", ctypes.c_double),
                ("coupling_wait_ms", ctypes.c_double), ("plan_host_ms", ctypes.c_double),
                ("plan_upload_ms", ctypes.c_double), ("coarse_solver", ctypes.c_int32),
                ("coarse_fronts", ctypes.c_int32), ("coarse_levels", ctypes.c_int32),
                ("coarse_gflop", ctypes.c_double), ("coarse_factor_mb", ctypes.c_double)]


_vp, _i32, _i64, _d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_lib.amsp_default_options.argtypes = [ctypes.POINTER(_Options)]
_lib.amsp_setup.argtypes = [ctypes.POINTER(_CSR), _vp, _i32, _i32, ctypes.POINTER(_Options),
                            ctypes.POINTER(_vp)]
_lib.amsp_setup.restype = _i32
_lib.amsp_apply.argtypes = [_vp, _vp, _vp, _i32]
_lib.amsp_apply.restype = _i32
_lib.amsp_apply_parts.argtypes = [_vp, _vp, _vp, _i32, _i32]
_lib.amsp_apply_parts.restype = _i32
_lib.amsp_apply_noalloc.argtypes = [_vp, _vp, _vp, _i32, _i32]
_lib.amsp_apply_noalloc.restype = _i32
_lib.amsp_pcg.argtypes = [_vp, _vp, _vp, _i32, _d, _i32, ctypes.POINTER(_Info)]
_lib.amsp_pcg.restype = _i32
_lib.amsp_pcg_batched.argtypes = [_vp, _i32, _vp, _vp, _vp, _i32, _d, _i32, ctypes.POINTER(_Info),
                                  _vp, _vp]
_lib.amsp_pcg_batched.restype = _i32
_lib.amsp_gmres.argtypes = [_vp, _vp, _vp, _i32, _i32, _d, _i32, ctypes.POINTER(_Info)]
_lib.amsp_gmres.restype = _i32
_lib.amsp_spmv.argtypes = [_vp, _vp, _vp]
_lib.amsp_spmv.restype = _i32
_lib.amsp_grad_values.argtypes = [_vp, _vp, _vp, _vp]
_lib.amsp_grad_values.restype = _i32
_lib.amsp_get_setup_info.argtypes = [_vp, ctypes.POINTER(_SetupInfo)]
_lib.amsp_get_setup_info.restype = _i32
_lib.amsp_get_pcg_history.argtypes = [_vp, _vp, _i32, ctypes.POINTER(_i32)]
_lib.amsp_get_pcg_history.restype = _i32
_lib.amsp_get_eigenvalues.argtypes = [_vp, _vp]
_lib.amsp_get_eigenvalues.restype = _i32
_lib.amsp_get_coarse_matrix.argtypes = [_vp, _vp]
_lib.amsp_get_coarse_matrix.restype = _i32
_lib.amsp_get_region.argtypes = [_vp, _i32, ctypes.POINTER(_i32), _vp, _vp]
_lib.amsp_get_region.restype = _i32
_lib.amsp_plan_regions.argtypes = [ctypes.POINTER(_CSR), _vp, _i32, _i32, ctypes.POINTER(_Options),
                                   _vp, _vp, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
_lib.amsp_plan_regions.restype = _i32
_lib.amsp_selftest_mfma.argtypes = [_vp, _vp, _vp]
_lib.amsp_selftest_mfma.restype = _i32
_lib.amsp_destroy.argtypes = [_vp]
_lib.amsp_release_caches.argtypes = []
_lib.amsp_release_caches.restype = None
_lib.amsp_status_string.argtypes = [_i32]
_lib.amsp_status_string.restype = ctypes.c_char_p
_lib.amsp_last_error.argtypes = [_vp]
_lib.amsp_last_error.restype = ctypes.c_char_p
_lib.amsp_setup_error.argtypes = []
_lib.amsp_setup_error.restype = ctypes.c_char_p

EXPORTED = ["amsp_default_options", "amsp_setup", "amsp_apply", "amsp_apply_parts",
            "amsp_apply_noalloc", "amsp_pcg", "amsp_pcg_batched",
            "amsp_gmres",
            "amsp_spmv", "amsp_grad_values", "amsp_get_setup_info", "amsp_get_pcg_history", "amsp_get_eigenvalues", "amsp_get_coarse_matrix",
            "amsp_get_region", "amsp_plan_regions", "amsp_selftest_mfma", "amsp_destroy",
            "amsp_release_caches", "amsp_status_string",
            "amsp_last_error", "amsp_setup_error"]


def plan_regions(row_ptr, col_idx, val, part, nparts: int, nev: int, *, overlap: int = 1,
                 local_order: str = "rcm", dense_tiles: bool = False):
    """Host-only planning: returns (list of region dof arrays in local order,
    tile count of one factor set, number of coupled subdomain pairs)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.float64)
    pa = np.ascontiguousarray(part, dtype=np.int32)
    csr = _CSR(len(rp) - 1, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    o = _Options()
    _lib.amsp_default_options(ctypes.byref(o))
    o.overlap, o.local_order, o.dense_tiles = int(overlap), ORDER[local_order], int(dense_tiles)
    ptr = np.zeros(int(nparts) + 1, dtype=np.int32)
    nt, npairs = _i64(), _i64()
    st = _lib.amsp_plan_regions(ctypes.byref(csr), pa.ctypes.data, int(nparts), int(nev),
                                ctypes.byref(o), ptr.ctypes.data, None, 0, ctypes.byref(nt),
                                ctypes.byref(npairs))
    if st != AMSP_OK:
        raise AmspError(st, _lib.amsp_setup_error().decode())
    dofs = np.empty(int(ptr[-1]), dtype=np.int32)
    st = _lib.amsp_plan_regions(ctypes.byref(csr), pa.ctypes.data, int(nparts), int(nev),
                                ctypes.byref(o), ptr.ctypes.data, dofs.ctypes.data, len(dofs),
                                None, None)
    if st != AMSP_OK:
        raise AmspError(st, _lib.amsp_setup_error().decode())
    return [dofs[ptr[i]:ptr[i + 1]] for i in range(int(nparts))], nt.value, npairs.value


def setup_error_code(row_ptr, col_idx, val, part, nparts: int, nev: int, overlap: int = 1,
                     eig_shift: float = 1e-4) -> tuple:
    """Run amsp_setup's host-side checks on inputs that are expected to fail
    before any device work; returns (status name, message)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.float64)
    pa = np.ascontiguousarray(part, dtype=np.int32)
    csr = _CSR(len(rp) - 1, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    o = _Options()
    _lib.amsp_default_options(ctypes.byref(o))
    o.overlap, o.eig_shift = int(overlap), float(eig_shift)
    ptr = np.zeros(max(int(nparts), 0) + 1, dtype=np.int32)
    st = _lib.amsp_plan_regions(ctypes.byref(csr), pa.ctypes.data, int(nparts), int(nev),
                                ctypes.byref(o), ptr.ctypes.data, None, 0, None, None)
    return STATUS.get(st, st), _lib.amsp_setup_error().decode()


def selftest_mfma(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """D = A B (16x4 times 4x16) by one matrix-core instruction on the device."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    d = np.empty((16, 16), dtype=np.float64)
    st = _lib.amsp_selftest_mfma(a.ctypes.data, b.ctypes.data, d.ctypes.data)
    if st != AMSP_OK:
        raise AmspError(st, "selftest failed")
    return d


def default_options() -> dict:
    o = _Options()
    _lib.amsp_default_options(ctypes.byref(o))
    return {name: getattr(o, name) for name, _ in _Options._fields_ if name != "stream"}


def synchronize(stream=None):
    torch = _torch()
    (stream or torch.cuda.current_stream()).synchronize()


def _torch():
    import torch  # imported lazily so that the C-ABI checks run without a GPU
    return torch


def _check_dev(t, name, n=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on a HIP device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.shape[0] != n:
        raise ValueError(f"{name} must have {n} rows")


class Preconditioner:
    """Handle over amsp_setup / amsp_apply / amsp_pcg.

    A: (row_ptr int64[n+1], col_idx int32[nnz], val float64[nnz]) host arrays
    part: int32[n] host partition with values in [0, nparts)
    """

    def __init__(self, row_ptr, col_idx, val, part, nparts: int, nev: int, *, overlap: int = 1,
                 precision: str = "fp64", pou: int = 0, local_order: str = "rcm",
                 dense_tiles: bool = False, eig_tol: float = 0.0, eig_maxit: int = 80,
                 eig_shift: float = 1e-4, chunk: int = 8, flexible: int = -1,
                 keep_a0: bool = False, timing=False, timing_stride: int = 1, stream=None,
                 singular: bool = False, cycle: str = "additive", smoother_weight: float = 0.0,
                 coarse_basis: str = "stored", coarse_solver: str = "auto"):
        torch = _torch()
        self._h = None
        self._keep = [np.ascontiguousarray(row_ptr, dtype=np.int64),
                      np.ascontiguousarray(col_idx, dtype=np.int32),
                      np.ascontiguousarray(val, dtype=np.float64),
                      np.ascontiguousarray(part, dtype=np.int32)]
        rp, ci, va, pa = self._keep
        self.n = len(rp) - 1
        self.nparts = int(nparts)
        self.nev = int(nev)
        csr = _CSR(self.n, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
        o = _Options()
        _lib.amsp_default_options(ctypes.byref(o))
        o.overlap, o.precision, o.pou = int(overlap), PRECISION[precision], int(pou)
        o.local_order, o.dense_tiles = ORDER[local_order], int(bool(dense_tiles))
        o.eig_tol, o.eig_maxit, o.eig_shift = float(eig_tol), int(eig_maxit), float(eig_shift)
        o.chunk, o.flexible, o.keep_a0 = int(chunk), int(flexible), int(bool(keep_a0))
        # timing: True -> every kernel class, or an int bit mask of classes
        o.timing = 0x1F if timing is True else int(timing)
        o.timing_stride = max(1, int(timing_stride))
        o.singular = int(bool(singular))
        o.cycle = {"additive": 0, "multiplicative": 1}[cycle]
        o.smoother_weight = float(smoother_weight)
        o.coarse_basis = {"stored": 0, "fp64": 1}[coarse_basis]
        o.coarse_solver = {"auto": 0, "dense": 1, "sparse": 2}[coarse_solver]
        if torch.cuda.is_available():
            torch.cuda.init()  # the device context exists before the library's first HIP call
            torch.cuda.synchronize()
            if stream is None:
                stream = torch.cuda.current_stream()
        self.stream = stream
        o.stream = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
        h = ctypes.c_void_p()
        st = _lib.amsp_setup(ctypes.byref(csr), pa.ctypes.data, self.nparts, self.nev,
                             ctypes.byref(o), ctypes.byref(h))
        if st != AMSP_OK:
            raise AmspError(st, _lib.amsp_setup_error().decode())
        self._h = h
        self.precision = precision
        self.info = self.setup_info()

    # -- lifetime
    def close(self):
        if self._h is not None:
            _lib.amsp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st):
        if st != AMSP_OK:
            raise AmspError(st, _lib.amsp_last_error(self._h).decode())

    # -- compute
    def apply(self, r, out=None, parts: int = 3):
        """z = M^{-1} r (r: float64 device tensor of shape (n,) or (n, k))."""
        torch = _torch()
        _check_dev(r, "r", self.n)
        z = out if out is not None else torch.empty_like(r)
        nrhs = 1 if r.dim() == 1 else r.shape[1]
        rr = r if r.dim() == 1 else r.t().contiguous()
        zz = z if r.dim() == 1 else torch.empty_like(rr)
        self._err(_lib.amsp_apply_parts(self._h, rr.data_ptr(), zz.data_ptr(), nrhs, parts))
        if r.dim() == 2:
            z.copy_(zz.t())
        return z

    def apply_columns(self, rt, out=None, parts: int = 3):
        """z_j = M^{-1} r_j for the rows r_j of a (k, n) float64 device tensor
        (the C ABI's layout: right-hand sides n apart, so no transposed copy)."""
        torch = _torch()
        if rt.dim() != 2 or rt.shape[1] != self.n:
            raise ValueError(f"rt must have shape (k, {self.n})")
        _check_dev(rt, "rt")
        z = out if out is not None else torch.empty_like(rt)
        self._err(_lib.amsp_apply_parts(self._h, rt.data_ptr(), z.data_ptr(), rt.shape[0], parts))
        return z

    def pcg_columns(self, ft, rtol: float = 1e-8, maxit: int = 1000, out=None,
                    raise_on_noconv=True):
        """PCG on the rows of a (k, n) float64 device tensor together (one CG
        recurrence per right-hand side); returns (u of shape (k, n), info)."""
        torch = _torch()
        if ft.dim() != 2 or ft.shape[1] != self.n:
            raise ValueError(f"ft must have shape (k, {self.n})")
        _check_dev(ft, "ft")
        u = out if out is not None else torch.empty_like(ft)
        inf = _Info()
        st = _lib.amsp_pcg(self._h, ft.data_ptr(), u.data_ptr(), ft.shape[0], float(rtol),
                           int(maxit), ctypes.byref(inf))
        info = {name: getattr(inf, name) for name, _ in _Info._fields_
                if name not in ("kernel_ms", "kernel_launches")}
        info["status"] = STATUS.get(st, st)
        if st != AMSP_OK and (raise_on_noconv or st != -9):
            res = (u, info) if st == -10 and ft.shape[0] >= 2 else None
            raise AmspError(st, _lib.amsp_last_error(self._h).decode(), res)
        return u, info

    def spmv(self, x, out=None):
        torch = _torch()
        _check_dev(x, "x", self.n)
        y = out if out is not None else torch.empty_like(x)
        self._err(_lib.amsp_spmv(self._h, x.data_ptr(), y.data_ptr()))
        return y

    def apply_noalloc(self, r, out=None, parts: int = 3):
        """z = M^{-1} r through amsp_apply_noalloc (no device allocation; the
        workspace is the library's per-device scratch array).  r: float64
        device tensor of shape (n,) or (n, k)."""
        torch = _torch()
        _check_dev(r, "r", self.n)
        z = out if out is not None else torch.empty_like(r)
        nrhs = 1 if r.dim() == 1 else r.shape[1]
        rr = r if r.dim() == 1 else r.t().contiguous()
        zz = z if r.dim() == 1 else torch.empty_like(rr)
        self._err(_lib.amsp_apply_noalloc(self._h, rr.data_ptr(), zz.data_ptr(), nrhs, parts))
        if r.dim() == 2:
            z.copy_(zz.t())
        return z

    def pcg(self, f, rtol: float = 1e-8, maxit: int = 1000, out=None, raise_on_noconv=True):
        """Solve A u = f by preconditioned CG; returns (u, info dict).  f of
        shape (n, k) solves k systems together (one recurrence per column)."""
        torch = _torch()
        _check_dev(f, "f", self.n)
        u = out if out is not None else torch.empty_like(f)
        inf = _Info()
        if f.dim() == 2:
            ff = f.t().contiguous()
            uu = torch.empty_like(ff)
            st = _lib.amsp_pcg(self._h, ff.data_ptr(), uu.data_ptr(), f.shape[1], float(rtol),
                               int(maxit), ctypes.byref(inf))
            u.copy_(uu.t())
        else:
            st = _lib.amsp_pcg(self._h, f.data_ptr(), u.data_ptr(), 1, float(rtol), int(maxit),
                               ctypes.byref(inf))
        info = {name: getattr(inf, name) for name, _ in _Info._fields_
                if name not in ("kernel_ms", "kernel_launches")}
        info["kernel_ms"] = list(inf.kernel_ms)
        info["kernel_launches"] = list(inf.kernel_launches)
        info["status"] = STATUS.get(st, st)
        if st != AMSP_OK and (raise_on_noconv or st != -9):
            res = (u, info) if st == -10 and f.dim() == 2 and f.shape[1] >= 2 else None
            raise AmspError(st, _lib.amsp_last_error(self._h).decode(), res)
        return u, info

    def pcg_batched(self, F, prob_ptr, rtol: float = 1e-8, maxit: int = 1000,
                    raise_on_noconv=True):
        """Independent problems together: A is block-diagonal with blocks on
        rows [prob_ptr[s], prob_ptr[s+1]); F (n, k) float64 device tensor,
        k <= 16.  One CG recurrence per (problem, column).  Returns (U, info,
        iterations (nprob, k), true relative residuals (nprob, k))."""
        torch = _torch()
        _check_dev(F, "F", self.n)
        k = 1 if F.dim() == 1 else F.shape[1]
        pp = np.ascontiguousarray(prob_ptr, dtype=np.int64)
        nprob = len(pp) - 1
        Ft = F.reshape(self.n, k).t().contiguous()
        Ut = torch.empty_like(Ft)
        its = np.zeros((nprob, k), dtype=np.int32)
        rel = np.zeros((nprob, k), dtype=np.float64)
        inf = _Info()
        st = _lib.amsp_pcg_batched(self._h, nprob, pp.ctypes.data, Ft.data_ptr(), Ut.data_ptr(), k,
                                   float(rtol), int(maxit), ctypes.byref(inf), its.ctypes.data,
                                   rel.ctypes.data)
        info = {name: getattr(inf, name) for name, _ in _Info._fields_
                if name not in ("kernel_ms", "kernel_launches")}
        info["status"] = STATUS.get(st, st)
        U = Ut.t().reshape(F.shape) if F.dim() == 2 else Ut.reshape(-1)
        if st != AMSP_OK and (raise_on_noconv or st != -9):
            res = (U, info, its, rel) if st == -10 else None
            raise AmspError(st, _lib.amsp_last_error(self._h).decode(), res)
        return U, info, its, rel

    def gmres(self, f, rtol: float = 1e-6, restart: int = 30, maxit: int = 1000, out=None,
              raise_on_noconv=True):
        """Solve A u = f by restarted GMRES with the preconditioner (flexible
        right preconditioning); returns (u, info dict).  Defaults: the
        paper's 1e-6 reduction of the residual, restart every 30 steps."""
        torch = _torch()
        _check_dev(f, "f", self.n)
        u = out if out is not None else torch.empty_like(f)
        inf = _Info()
        st = _lib.amsp_gmres(self._h, f.data_ptr(), u.data_ptr(), 1, int(restart), float(rtol),
                             int(maxit), ctypes.byref(inf))
        info = {name: getattr(inf, name) for name, _ in _Info._fields_
                if name not in ("kernel_ms", "kernel_launches")}
        info["status"] = STATUS.get(st, st)
        if st != AMSP_OK and (raise_on_noconv or st != -9):
            raise AmspError(st, _lib.amsp_last_error(self._h).decode())
        return u, info

    def grad_values(self, lam, u, out=None):
        """grad[k] = -lam[row k] * u[col k] over the stored entries of A (the
        adjoint of the solve u = A^{-1} f, given lam = A^{-1} dJ/du)."""
        torch = _torch()
        _check_dev(lam, "lam", self.n)
        _check_dev(u, "u", self.n)
        nnz = len(self._keep[1])
        g = out if out is not None else torch.empty(nnz, dtype=torch.float64, device=u.device)
        self._err(_lib.amsp_grad_values(self._h, lam.data_ptr(), u.data_ptr(), g.data_ptr()))
        return g

    # -- introspection
    def setup_info(self) -> dict:
        si = _SetupInfo()
        self._err(_lib.amsp_get_setup_info(self._h, ctypes.byref(si)))
        d = {name: getattr(si, name) for name, _ in _SetupInfo._fields_ if name != "phase_ms"}
        d["phase_ms"] = list(si.phase_ms)
        return d

    def pcg_history(self) -> np.ndarray:
        """Relative residuals of the last pcg() (recursive) or gmres()
        (estimates) call, one per step from step 0."""
        cnt = ctypes.c_int32()
        self._err(_lib.amsp_get_pcg_history(self._h, None, 0, ctypes.byref(cnt)))
        out = np.empty(cnt.value, dtype=np.float64)
        self._err(_lib.amsp_get_pcg_history(self._h, out.ctypes.data, len(out), ctypes.byref(cnt)))
        return out

    def eigenvalues(self) -> np.ndarray:
        out = np.empty((self.nparts, self.nev + 1), dtype=np.float64)
        self._err(_lib.amsp_get_eigenvalues(self._h, out.ctypes.data))
        return out

    def coarse_matrix(self) -> np.ndarray:
        nc = self.info["nc"]
        out = np.empty((nc, nc), dtype=np.float64)
        self._err(_lib.amsp_get_coarse_matrix(self._h, out.ctypes.data))
        return out

    def region(self, i: int, with_basis: bool = True):
        ni = ctypes.c_int32()
        self._err(_lib.amsp_get_region(self._h, int(i), ctypes.byref(ni), None, None))
        dofs = np.empty(ni.value, dtype=np.int32)
        phi = np.empty((ni.value, max(self.nev, 1)), dtype=np.float64) if with_basis else None
        self._err(_lib.amsp_get_region(self._h, int(i), ctypes.byref(ni), dofs.ctypes.data,
                                       phi.ctypes.data if (with_basis and self.nev > 0) else None))
        return dofs, (phi[:, :self.nev] if with_basis else None)


def setup(A, part, nparts, nev, **kw) -> Preconditioner:
    """A: object with row_ptr, col_idx, val (e.g. workloads.CSR)."""
    return Preconditioner(A.row_ptr, A.col_idx, A.val, part, nparts, nev, **kw)


def _solve_fn():
    """The torch.autograd.Function behind solve() (built on first use, so that
    importing this module does not need torch)."""
    global _SOLVE_FN
    if _SOLVE_FN is not None:
        return _SOLVE_FN
    torch = _torch()

    class _Solve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, vals, f, row_ptr, col_idx, part, nparts, nev, rtol, maxit, kw):
            pc = Preconditioner(row_ptr, col_idx, vals.detach().cpu().numpy(), part, nparts, nev,
                                **kw)
            u, info = pc.pcg(f.detach().contiguous(), rtol, maxit)
            ctx.pc, ctx.rtol, ctx.maxit, ctx.info = pc, rtol, maxit, info
            ctx.save_for_backward(u)
            return u

        @staticmethod
        def backward(ctx, gu):
            (u,) = ctx.saved_tensors
            pc = ctx.pc
            # adjoint system A lam = dJ/du (A symmetric: the same handle)
            lam, _ = pc.pcg(gu.contiguous(), ctx.rtol, ctx.maxit)
            gvals = pc.grad_values(lam, u) if ctx.needs_input_grad[0] else None
            pc.close()
            ctx.pc = None
            return (gvals, lam if ctx.needs_input_grad[1] else None, None, None, None, None,
                    None, None, None, None)

    _SOLVE_FN = _Solve
    return _Solve


_SOLVE_FN = None


def solve(vals, f, row_ptr, col_idx, part, nparts: int, nev: int, rtol: float = 1e-10,
          maxit: int = 2000, **kw):
    """u = A^{-1} f, differentiable in the stored values of A and in f.

    vals: float64 tensor (nnz,) of A's values in the CSR order of
    (row_ptr, col_idx); A must stay symmetric positive definite.  f: float64
    device tensor (n,).  The forward pass sets up the preconditioner for these
    values and runs PCG to rtol; the backward pass solves the adjoint system
    A lam = dJ/du with the same handle and returns dJ/df = lam and
    dJ/dvals[k] = -lam[row k] u[col k] (each stored entry independent).
    Remaining keywords go to Preconditioner (overlap, precision, ...)."""
    return _solve_fn().apply(vals, f, row_ptr, col_idx, part, nparts, nev, float(rtol),
                             int(maxit), kw)
