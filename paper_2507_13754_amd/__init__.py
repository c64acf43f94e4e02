"""Python binding of libtbs (the MI355X traditional-Born-series solver).

A thin ctypes layer over the C ABI in ``include/tbs.h``: it checks and
marshals arguments (torch tensors are passed by device pointer on the current
torch stream) and raises on error codes.  All arithmetic of the method runs in
the library's HIP kernels; there is no fallback path, and every call fails
loudly when ``libtbs.so`` has not been built.

Shapes follow the library: grids are C order, x fastest ((ny, nx) or
(nz, ny, nx)); a batch of B right-hand sides is a leading axis.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# TBS_LIBRARY overrides the library file (e.g. an alternative tuning build).
LIB_PATH = os.environ.get("TBS_LIBRARY", os.path.join(HERE, "libtbs.so"))

TBS_C64, TBS_C128 = 0, 1
TBS_OK = 0
TBS_ERR_INVALID = -1
TBS_WARN_NONFINITE, TBS_WARN_DIVERGING, TBS_WARN_NOT_CONVERGED = 1, 2, 3
TBS_ADJ_STORE, TBS_ADJ_RECOMPUTE, TBS_ADJ_SERIES_ONLY = 0, 1, 2
TBS_ITER_PAPER, TBS_ITER_CBS = 0, 1

# Every entry point of include/tbs.h.
EXPORTS = (
    "tbs_version", "tbs_status_string", "tbs_padded_length", "tbs_wavenumber",
    "tbs_background_k0", "tbs_hankel01", "tbs_self_cell", "tbs_plan_create", "tbs_plan_info",
    "tbs_plan_set_stream", "tbs_green_tabulate", "tbs_green_import", "tbs_green_export",
    "tbs_potential", "tbs_solve", "tbs_harmonic_source", "tbs_harmonic_source_n", "tbs_adjoint", "tbs_misfit",
    "tbs_speed_gradient", "tbs_profile_enable", "tbs_profile_read", "tbs_plan_destroy",
    "tbs_last_error", "tbs_batch_create", "tbs_batch_solve", "tbs_batch_destroy",
    "tbs_batch_last_error", "tbs_plan_autotune", "tbs_green_periodic", "tbs_abl_profile",
    "tbs_kspace_coefficients", "tbs_density_contrast",
    "tbs_iterate", "tbs_batch_profile_enable", "tbs_batch_profile_read", "tbs_solve_noalloc",
    "tbs_harmonic_source_scaled", "tbs_batch_autotune",
)
PASS_KINDS = ("row_first", "row_mid", "row_last", "col_conv", "col_fwd", "col_inv")


class TBSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class TBSWarning(UserWarning):
    pass


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


_lib = None


def library() -> ctypes.CDLL:
    """Load libtbs.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python -m paper_2507_13754_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    c128p = ctypes.POINTER(c128)
    sig = {
        "tbs_version": (ctypes.c_int, []),
        "tbs_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "tbs_padded_length": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int, i64p]),
        "tbs_wavenumber": (ctypes.c_int, [ctypes.c_double] * 4 + [c128p]),
        "tbs_background_k0": (ctypes.c_int, [ctypes.c_double] * 5 + [c128p]),
        "tbs_hankel01": (ctypes.c_int, [c128, c128p, c128p]),
        "tbs_self_cell": (ctypes.c_int, [ctypes.c_int, c128, ctypes.c_double, c128p]),
        "tbs_plan_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, i64p, ctypes.c_double,
                                           c128, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]),
        "tbs_plan_info": (ctypes.c_int, [vp, i64p, i64p]),
        "tbs_plan_set_stream": (ctypes.c_int, [vp, vp]),
        "tbs_green_tabulate": (ctypes.c_int, [vp]),
        "tbs_green_import": (ctypes.c_int, [vp, vp]),
        "tbs_green_export": (ctypes.c_int, [vp, vp]),
        "tbs_potential": (ctypes.c_int, [vp, vp] + [ctypes.c_double] * 5 + [vp, vp]),
        "tbs_solve": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp, dp]),
        "tbs_solve_noalloc": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp, dp]),
        "tbs_harmonic_source_n": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p), vp,
                                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, vp]),
        "tbs_harmonic_source": (ctypes.c_int, [vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, vp]),
        "tbs_harmonic_source_scaled": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                                      ctypes.POINTER(ctypes.c_int), vp, ctypes.c_double,
                                                      ctypes.c_double, ctypes.c_double, vp,
                                                      ctypes.POINTER(ctypes.c_int)]),
        "tbs_adjoint": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp, vp, dp, ctypes.c_int]),
        "tbs_misfit": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp, vp, vp]),
        "tbs_speed_gradient": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int]),
        "tbs_plan_autotune": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "tbs_profile_enable": (ctypes.c_int, [vp, ctypes.c_int]),
        "tbs_profile_read": (ctypes.c_int, [vp, dp, i64p]),
        "tbs_plan_destroy": (None, [vp]),
        "tbs_batch_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int]),
        "tbs_batch_solve": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int,
                                           ctypes.POINTER(vp), dp]),
        "tbs_batch_destroy": (None, [vp]),
        "tbs_batch_autotune": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "tbs_batch_profile_enable": (ctypes.c_int, [vp, ctypes.c_int]),
        "tbs_batch_profile_read": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ctypes.c_int), i64p, dp, ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "tbs_batch_last_error": (ctypes.c_char_p, [vp]),
        "tbs_last_error": (ctypes.c_char_p, [vp]),
        "tbs_green_periodic": (ctypes.c_int, [vp, ctypes.c_double, vp]),
        "tbs_kspace_coefficients": (ctypes.c_int, [ctypes.c_double] * 4 + [vp]),
        "tbs_density_contrast": (ctypes.c_int, [vp, vp]),
        "tbs_abl_profile": (ctypes.c_int, [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, dp]),
        "tbs_iterate": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       vp, ctypes.POINTER(ctypes.c_int), dp, ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int, plan=None, what: str = "") -> int:
    if rc == TBS_OK:
        return rc
    L = library()
    msg = L.tbs_last_error(plan).decode() if plan is not None or rc < 0 else ""
    name = L.tbs_status_string(rc).decode()
    if rc < 0:
        raise TBSError(rc, f"{what}: {name}: {msg}")
    import warnings
    warnings.warn(f"{what}: {name}: {msg}", TBSWarning, stacklevel=3)
    return rc


# ------------------------------------------------------------- host helpers --

def padded_length(n: int, padding: int = 2) -> int:
    m = ctypes.c_int64()
    _check(library().tbs_padded_length(n, padding, ctypes.byref(m)), what="tbs_padded_length")
    return int(m.value)


def wavenumber(omega: float, c: float, alpha0: float, y: float) -> complex:
    k = c128()
    _check(library().tbs_wavenumber(omega, c, alpha0, y, ctypes.byref(k)), what="tbs_wavenumber")
    return complex(k.re, k.im)


def background_k0(omega: float, c0: float, alpha0: float, y: float, eps: float = 0.0) -> complex:
    k = c128()
    _check(library().tbs_background_k0(omega, c0, alpha0, y, eps, ctypes.byref(k)),
           what="tbs_background_k0")
    return complex(k.re, k.im)


def hankel01(z: complex) -> Tuple[complex, complex]:
    h0, h1 = c128(), c128()
    _check(library().tbs_hankel01(c128(z.real, z.imag), ctypes.byref(h0), ctypes.byref(h1)),
           what="tbs_hankel01")
    return complex(h0.re, h0.im), complex(h1.re, h1.im)


def self_cell(ndim: int, k0: complex, dx: float) -> complex:
    w = c128()
    _check(library().tbs_self_cell(ndim, c128(k0.real, k0.imag), dx, ctypes.byref(w)),
           what="tbs_self_cell")
    return complex(w.re, w.im)


# -------------------------------------------------------------------- plans --

def _torch():
    import torch
    return torch


def _ptr(t, dtype, shape: Optional[Sequence[int]] = None, name: str = "tensor"):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class KSpacePotential(ctypes.Structure):
    """Case II k-space potential VV = eta |p|^(nu+1) - i (tau omega |p|^nu + eps)."""
    _fields_ = [("tau", ctypes.c_double), ("eta", ctypes.c_double), ("nu", ctypes.c_double),
                ("omega", ctypes.c_double)]


def kspace_potential(alpha0: float, nu: float, c: float, omega: float) -> KSpacePotential:
    """Case II coefficients (tau, eta) of the power law alpha0 omega^nu at speed c."""
    out = KSpacePotential()
    _check(library().tbs_kspace_coefficients(float(alpha0), float(nu), float(c), float(omega),
                                             ctypes.byref(out)), what="tbs_kspace_coefficients")
    return out


def abl_profile(n: int, dx: float, zeta: float, mu_cells: float) -> np.ndarray:
    """The sigmoid absorbing-layer profile along one axis (host, float64)."""
    out = np.empty(int(n), dtype=np.float64)
    _check(library().tbs_abl_profile(int(n), float(dx), float(zeta), float(mu_cells),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           what="tbs_abl_profile")
    return out


class Plan:
    """Born-series plan for one grid, dx, background k0, precision and batch.

    ``shape``: C-order grid, (ny, nx) or (nz, ny, nx).  ``dtype``:
    torch.complex64 (FP32 with Kahan-compensated sums) or torch.complex128."""

    def __init__(self, shape: Sequence[int], dx: float, k0: complex, padding: int = 2,
                 dtype=None, batch: int = 1, stream=None):
        torch = _torch()
        L = library()
        self.dtype = dtype if dtype is not None else torch.complex64
        if self.dtype not in (torch.complex64, torch.complex128):
            raise TypeError("dtype must be torch.complex64 or torch.complex128")
        self.shape = tuple(int(s) for s in shape)
        if len(self.shape) not in (2, 3):
            raise ValueError("shape must be (ny, nx) or (nz, ny, nx)")
        self.ndim = len(self.shape)
        grid = list(reversed(self.shape)) + [1] * (3 - self.ndim)
        self.batch = int(batch)
        self.k0 = complex(k0)
        self.dx = float(dx)
        self._stream = stream
        h = ctypes.c_void_p()
        g = (ctypes.c_int64 * 3)(*grid)
        rc = L.tbs_plan_create(ctypes.byref(h), self.ndim, g, self.dx, c128(self.k0.real, self.k0.imag),
                               int(padding), TBS_C128 if self.dtype == torch.complex128 else TBS_C64,
                               self.batch, self._stream_handle())
        if rc != TBS_OK:
            msg = L.tbs_last_error(None).decode()
            raise TBSError(rc, f"tbs_plan_create: {L.tbs_status_string(rc).decode()}: {msg}")
        self._h = h
        pad = (ctypes.c_int64 * 3)()
        nbytes = ctypes.c_int64()
        L.tbs_plan_info(h, pad, ctypes.byref(nbytes))
        self.padded = tuple(pad[i] for i in range(3))        # (Mx, My, Mz)
        self.device_bytes = int(nbytes.value)

    def _stream_handle(self):
        torch = _torch()
        s = self._stream if self._stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def _sync_stream(self):
        library().tbs_plan_set_stream(self._h, self._stream_handle())

    @property
    def points(self) -> int:
        return int(np.prod(self.shape))

    def close(self):
        if getattr(self, "_h", None):
            library().tbs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- Green spectrum --
    def tabulate(self):
        self._sync_stream()
        _check(library().tbs_green_tabulate(self._h), self._h, "tbs_green_tabulate")
        return self

    def autotune(self):
        """Pick the fastest block shapes for this plan (bitwise-neutral);
        returns (rows per row-pass block, columns per convolution block)."""
        nr, nc = ctypes.c_int(), ctypes.c_int()
        self._sync_stream()
        _check(library().tbs_plan_autotune(self._h, ctypes.byref(nr), ctypes.byref(nc)), self._h,
               "tbs_plan_autotune")
        return nr.value, nc.value

    def import_spectrum(self, full: np.ndarray):
        Mx, My, Mz = self.padded
        want = (Mz, My, Mx) if self.ndim == 3 else (My, Mx)
        a = np.ascontiguousarray(full, dtype=np.complex128)
        if a.shape != want:
            raise ValueError(f"spectrum must have shape {want}")
        self._sync_stream()
        _check(library().tbs_green_import(self._h, a.ctypes.data_as(ctypes.c_void_p)), self._h,
               "tbs_green_import")
        return self

    def export_spectrum(self) -> np.ndarray:
        Mx, My, Mz = self.padded
        shp = (Mx // 2 + 1, My // 2 + 1) + ((Mz // 2 + 1,) if self.ndim == 3 else ())
        out = np.empty(shp, dtype=np.complex128)
        _check(library().tbs_green_export(self._h, out.ctypes.data_as(ctypes.c_void_p)), self._h,
               "tbs_green_export")
        return out

    # -- medium --
    def potential(self, c, omega: float, c0: float, alpha0: float, y: float, eps: float = 0.0,
                  with_derivative: bool = False):
        torch = _torch()
        cp = _ptr(c, torch.float64, self.shape, "c")
        V = torch.empty(self.shape, dtype=self.dtype, device=c.device)
        dV = torch.empty(self.shape, dtype=self.dtype, device=c.device) if with_derivative else None
        self._sync_stream()
        _check(library().tbs_potential(self._h, cp, omega, c0, alpha0, y, eps,
                                       ctypes.c_void_p(V.data_ptr()),
                                       ctypes.c_void_p(dV.data_ptr()) if dV is not None else None),
               self._h, "tbs_potential")
        return (V, dV) if with_derivative else V

    # -- series --
    def _bshape(self):
        return (self.batch,) + self.shape

    def solve(self, source, potential, nterms: int, out=None, residual: bool = False):
        torch = _torch()
        sp = _ptr(source, self.dtype, self._bshape(), "source")
        vp = _ptr(potential, self.dtype, self.shape, "potential")
        if out is None:
            out = torch.empty(self._bshape(), dtype=self.dtype, device=source.device)
        op = _ptr(out, self.dtype, self._bshape(), "out")
        res = np.empty((self.batch, nterms), dtype=np.float64) if residual else None
        self._sync_stream()
        rc = library().tbs_solve(self._h, sp, vp, int(nterms), op,
                                 res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if residual else None)
        _check(rc, self._h, "tbs_solve")
        return (out, res) if residual else out

    def solve_noalloc(self, source, potential, nterms: int, out, residual: bool = False):
        """solve() on the library's static workspace (tbs_solve_noalloc): no
        device allocation by the library or here, so `out` is required."""
        torch = _torch()
        sp = _ptr(source, self.dtype, self._bshape(), "source")
        vp = _ptr(potential, self.dtype, self.shape, "potential")
        op = _ptr(out, self.dtype, self._bshape(), "out")
        res = np.empty((self.batch, nterms), dtype=np.float64) if residual else None
        self._sync_stream()
        rc = library().tbs_solve_noalloc(self._h, sp, vp, int(nterms), op,
                                         res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if residual else None)
        _check(rc, self._h, "tbs_solve_noalloc")
        return (out, res) if residual else out

    def harmonic_source(self, p1, c, omega: float, rho: float, BA: float, out=None):
        torch = _torch()
        pp = _ptr(p1, self.dtype, self._bshape(), "p1")
        cp = _ptr(c, torch.float64, self.shape, "c")
        if out is None:
            out = torch.empty(self._bshape(), dtype=self.dtype, device=p1.device)
        op = _ptr(out, self.dtype, self._bshape(), "out")
        self._sync_stream()
        _check(library().tbs_harmonic_source(self._h, pp, cp, omega, rho, BA, op), self._h,
               "tbs_harmonic_source")
        return out

    def harmonic_source_n(self, n: int, fields, c, omega: float, rho: float, BA: float, out=None):
        """S_n from psi_1 .. psi_{n-1} (list of device tensors of the batch shape)."""
        torch = _torch()
        if len(fields) < n - 1:
            raise ValueError("harmonic_source_n needs psi_1 .. psi_{n-1}")
        ptrs = (ctypes.c_void_p * max(1, n - 1))(*[_ptr(f, self.dtype, self._bshape(), "field")
                                                   for f in fields[: n - 1]])
        cp = _ptr(c, torch.float64, self.shape, "c")
        if out is None:
            out = torch.empty(self._bshape(), dtype=self.dtype, device=fields[0].device)
        op = _ptr(out, self.dtype, self._bshape(), "out")
        self._sync_stream()
        _check(library().tbs_harmonic_source_n(self._h, int(n), ptrs, cp, omega, rho, BA, op), self._h,
               "tbs_harmonic_source_n")
        return out

    def harmonic_source_scaled(self, n: int, fields, exps, c, omega: float, rho: float, BA: float, out=None):
        """S_n * 2^e from fields psi_a * 2^exps[a-1] (a = 1 .. n-1); returns
        (S_out, e).  The solve driven by S_out yields psi_n * 2^e."""
        torch = _torch()
        if len(fields) < n - 1 or len(exps) < n - 1:
            raise ValueError("harmonic_source_scaled needs psi_1 .. psi_{n-1} and their exponents")
        ptrs = (ctypes.c_void_p * max(1, n - 1))(*[_ptr(f, self.dtype, self._bshape(), "field")
                                                   for f in fields[: n - 1]])
        ex = (ctypes.c_int * max(1, n - 1))(*[int(e) for e in exps[: n - 1]])
        cp = _ptr(c, torch.float64, self.shape, "c")
        if out is None:
            out = torch.empty(self._bshape(), dtype=self.dtype, device=fields[0].device)
        op = _ptr(out, self.dtype, self._bshape(), "out")
        e = ctypes.c_int()
        self._sync_stream()
        _check(library().tbs_harmonic_source_scaled(self._h, int(n), ptrs, ex, cp, omega, rho, BA, op,
                                                    ctypes.byref(e)), self._h, "tbs_harmonic_source_scaled")
        return out, e.value

    def density_contrast(self, gamma=None):
        """Attach (float64 device map, shape of the grid) or detach (None) the
        density-contrast term; the tensor is kept alive by the plan."""
        torch = _torch()
        gp = _ptr(gamma, torch.float64, self.shape, "gamma")
        _check(library().tbs_density_contrast(self._h, gp), self._h, "tbs_density_contrast")
        self._gamma = gamma
        return self

    # -- the paper's periodic scheme (plans made with padding=1) --
    def green_periodic(self, eps: float, vv: Optional[KSpacePotential] = None):
        self._sync_stream()
        _check(library().tbs_green_periodic(self._h, float(eps), ctypes.byref(vv) if vv is not None else None),
               self._h, "tbs_green_periodic")
        return self

    def iterate(self, source, potential=None, mask_x=None, mask_y=None, check_row: Optional[int] = None,
                tol: float = 1e-5, max_iter: int = 2000, out=None, cbs: bool = False):
        """Fixed-point iteration of the paper (cbs=True: the convergent Born
        series); returns (psi, iterations, errors)."""
        torch = _torch()
        sp = _ptr(source, self.dtype, self._bshape(), "source")
        vp = _ptr(potential, self.dtype, self.shape, "potential")
        mx = _ptr(mask_x, torch.float64, (self.shape[1],), "mask_x")
        my = _ptr(mask_y, torch.float64, (self.shape[0],), "mask_y")
        if out is None:
            out = torch.empty(self._bshape(), dtype=self.dtype, device=source.device)
        op = _ptr(out, self.dtype, self._bshape(), "out")
        errs = np.zeros(int(max_iter), dtype=np.float64)
        n = ctypes.c_int()
        row = self.shape[0] // 2 if check_row is None else int(check_row)
        self._sync_stream()
        _check(library().tbs_iterate(self._h, sp, vp, mx, my, row, float(tol), int(max_iter), op,
                                     ctypes.byref(n), errs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     TBS_ITER_CBS if cbs else TBS_ITER_PAPER),
               self._h, "tbs_iterate")
        return out, int(n.value), errs[: n.value].copy()

    def adjoint(self, source, potential, nterms: int, adj_source, out=None,
                flags: int = TBS_ADJ_STORE, residual: bool = False):
        torch = _torch()
        sp = _ptr(source, self.dtype, self._bshape(), "source")
        vp = _ptr(potential, self.dtype, self.shape, "potential")
        qp = _ptr(adj_source, self.dtype, self._bshape(), "adj_source")
        if out is None:
            out = torch.empty(self._bshape(), dtype=self.dtype, device=adj_source.device)
        op = _ptr(out, self.dtype, self._bshape(), "out")
        res = np.empty((self.batch, nterms), dtype=np.float64) if residual else None
        self._sync_stream()
        _check(library().tbs_adjoint(self._h, sp, vp, int(nterms), qp, op,
                                     res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if residual else None,
                                     int(flags)), self._h, "tbs_adjoint")
        return (out, res) if residual else out

    def misfit(self, p, rec_index, p_obs):
        """rec_index: CUDA int64 [R] flat spatial indices; p_obs [B][R]."""
        torch = _torch()
        pp = _ptr(p, self.dtype, self._bshape(), "p")
        rp = _ptr(rec_index, torch.int64, None, "rec_index")
        nrec = int(rec_index.numel())
        op = _ptr(p_obs, self.dtype, (self.batch, nrec), "p_obs")
        q = torch.empty(self._bshape(), dtype=self.dtype, device=p.device)
        J = torch.empty((1,), dtype=torch.float64, device=p.device)
        self._sync_stream()
        _check(library().tbs_misfit(self._h, pp, rp, nrec, op, ctypes.c_void_p(q.data_ptr()),
                                    ctypes.c_void_p(J.data_ptr())), self._h, "tbs_misfit")
        return q, J

    def profile(self, enable: bool = True):
        """Start (or stop) per-pass event timing on the plan's stream."""
        self._sync_stream()
        _check(library().tbs_profile_enable(self._h, int(enable)), self._h, "tbs_profile_enable")

    def profile_read(self):
        """{pass kind: (total ms, launches)} since profile(); resets."""
        ms = (ctypes.c_double * 6)()
        cnt = (ctypes.c_int64 * 6)()
        _check(library().tbs_profile_read(self._h, ms, cnt), self._h, "tbs_profile_read")
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(PASS_KINDS)}

    def speed_gradient(self, g, dVdc, out=None, accumulate: bool = False):
        torch = _torch()
        gp = _ptr(g, self.dtype, self._bshape(), "g")
        dp = _ptr(dVdc, self.dtype, self.shape, "dVdc")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=g.device)
            accumulate = False
        op = _ptr(out, torch.float64, self.shape, "out")
        self._sync_stream()
        _check(library().tbs_speed_gradient(self._h, gp, dp, op, int(accumulate)), self._h,
               "tbs_speed_gradient")
        return out


class Batch:
    """Several 2D plans solved together: passes of grids with equal padded
    lengths share one grouped launch per term, and the whole series is recorded
    once as a HIP graph and replayed for the same buffers."""

    def __init__(self, plans: Sequence[Plan]):
        L = library()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h for p in self.plans])
        h = ctypes.c_void_p()
        for p in self.plans:
            p._sync_stream()
        rc = L.tbs_batch_create(ctypes.byref(h), arr, len(self.plans))
        if rc != TBS_OK:
            raise TBSError(rc, f"tbs_batch_create: {L.tbs_last_error(None).decode()}")
        self._h = h

    def solve(self, sources, potentials, nterms: int, outs=None, residual: bool = False):
        torch = _torch()
        n = len(self.plans)
        if len(sources) != n or len(potentials) != n:
            raise ValueError("one source and one potential per plan")
        if outs is None:
            outs = [torch.empty((p.batch,) + p.shape, dtype=p.dtype, device=s.device)
                    for p, s in zip(self.plans, sources)]
        sp = [_ptr(s, p.dtype, (p.batch,) + p.shape, "source") for p, s in zip(self.plans, sources)]
        vp = [_ptr(v, p.dtype, p.shape, "potential") for p, v in zip(self.plans, potentials)]
        op = [_ptr(o, p.dtype, (p.batch,) + p.shape, "out") for p, o in zip(self.plans, outs)]
        A = ctypes.c_void_p * n
        rows = sum(p.batch for p in self.plans)
        self.plans[0]._sync_stream()     # the caller's stream the batch joins
        res = np.empty((rows, nterms), dtype=np.float64) if residual else None
        L = library()
        rc = L.tbs_batch_solve(self._h, A(*sp), A(*vp), int(nterms), A(*op),
                               res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if residual else None)
        if rc < 0:
            raise TBSError(rc, f"tbs_batch_solve: {L.tbs_batch_last_error(self._h).decode()}")
        if rc > 0:
            import warnings
            warnings.warn(f"tbs_batch_solve: {L.tbs_status_string(rc).decode()}: "
                          f"{L.tbs_batch_last_error(self._h).decode()}", TBSWarning, stacklevel=2)
        return (outs, res) if residual else outs

    def autotune(self, sources, potentials, outs):
        """Pick the grouped launches' block shapes by timing them on these
        buffers (bitwise-neutral; the contents of outs are undefined after)."""
        n = len(self.plans)
        sp = [_ptr(s, p.dtype, (p.batch,) + p.shape, "source") for p, s in zip(self.plans, sources)]
        vp = [_ptr(v, p.dtype, p.shape, "potential") for p, v in zip(self.plans, potentials)]
        op = [_ptr(o, p.dtype, (p.batch,) + p.shape, "out") for p, o in zip(self.plans, outs)]
        A = ctypes.c_void_p * n
        self.plans[0]._sync_stream()
        L = library()
        rc = L.tbs_batch_autotune(self._h, A(*sp), A(*vp), A(*op))
        if rc != TBS_OK:
            raise TBSError(rc, f"tbs_batch_autotune: {L.tbs_batch_last_error(self._h).decode()}")

    def profile(self, enable: bool = True):
        """Per-launch event timing of later solves (no graph replay meanwhile)."""
        L = library()
        rc = L.tbs_batch_profile_enable(self._h, 1 if enable else 0)
        if rc != TBS_OK:
            raise TBSError(rc, f"tbs_batch_profile_enable: {L.tbs_batch_last_error(self._h).decode()}")

    def profile_read(self):
        """Timing since the last read: a list of dicts (kind name, FFT length,
        launches, summed ms, member tiles as plan indices with their
        right-hand-side counts), one per grouped launch kind of every set."""
        L = library()
        ne = ctypes.c_int()
        ci = ctypes.c_int
        cap = 0
        while True:
            kind, length, shape, first = (ci * max(cap, 1))(), (ci * max(cap, 1))(), (ci * max(cap, 1))(), (ci * (cap + 1))()
            mcap = 4 * sum(p.batch for p in self.plans) + 8
            members, mrhs = (ci * mcap)(), (ci * mcap)()
            launches = (ctypes.c_int64 * max(cap, 1))()
            ms = (ctypes.c_double * max(cap, 1))()
            rc = L.tbs_batch_profile_read(self._h, cap, ctypes.byref(ne), kind, length, shape, launches, ms, first,
                                          members, mrhs)
            if rc == TBS_ERR_INVALID and ne.value > cap:
                cap = ne.value
                continue
            break
        if rc != TBS_OK:
            raise TBSError(rc, f"tbs_batch_profile_read: {L.tbs_batch_last_error(self._h).decode()}")
        out = []
        for e in range(ne.value):
            out.append({"kind": PASS_KINDS[kind[e]], "length": int(length[e]), "shape": int(shape[e]),
                        "launches": int(launches[e]), "ms": float(ms[e]),
                        "members": [int(members[i]) for i in range(first[e], first[e + 1])],
                        "member_rhs": [int(mrhs[i]) for i in range(first[e], first[e + 1])]})
        return out

    def close(self):
        if getattr(self, "_h", None):
            library().tbs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
