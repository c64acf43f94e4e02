"""FP64 CPU oracle of the traditional Born series (TBS) Helmholtz solver.

TEST INFRASTRUCTURE.  This module is the slow, plainly written reference the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
never does, and it shares no code with the GPU library (it uses numpy/scipy
only).  Everything is complex128/float64.

What it computes (citations are to the paper's sections and equations):

* wavenumber k(x) and potential V(x) = k(x)^2 - k0^2 of an absorbing,
  dispersive, heterogeneous medium (Sec. 2.1.2 Eqs. power_law_absorption and
  acoustic_waveequn_time_independent_absorbing_dispersion; Sec. 2.2
  Eq. acoustic_waveequn6; Sec. 2.3.3 Eq. TBS_equation_inhomogeneous);
* the free-space Green's function g (Sec. 2.2 Eqs. soln_greens_fn, greens_fn),
  its cell-sampled kernel W(m) and the discrete operator (G f)_i = sum_j
  W(i-j) f_j, both as a direct O(P^2) sum and through zero-padded FFTs
  (Sec. 2.2 Eq. TBS_1, G = F^-1 g~ F);
* the Born series u_0 = G s, u_n = G(V u_{n-1}), p_L = sum_{n<L} u_n
  (Sec. 2.2 Eqs. TBS_2, TBS_algorithm, TBS_input), with the relative-norm
  residual of each term (Sec. 3.1 Eq. Error, read as a whole-grid L2 norm);
* dense Lippmann-Schwinger solves and the spectral radius of G V
  (Sec. 2.2, convergence condition under Eq. TBS_2);
* the second-harmonic source -xi (2 omega)^2 p1^2 / 2 (Sec. 2.1.4
  Eq. nonlinear_waveeqn_shi2; Sec. 2.3.4 Eq. TBS_solution_shi_2) and the
  sum-frequency sources of harmonics 3..5 (Sec. 2.3.4,
  Eq. TBS_solution_nonlinear_shi_n);
* the paper's own periodic scheme (Sec. 2.2 Eq. of g~, Sec. 3.1 and
  Algorithm 1): g~(p) = 1/(|p|^2 - k^2 - i eps) on the unpadded grid, the
  spatial potential (Cases I, III, IV) or the k-space potential of the
  absorbing-dispersive medium (Case II, Sec. 2.3.2), the sigmoid absorbing
  layer applied after every iteration but the first (Eq. ABL_profile), and
  the centre-row relative L1 change as stopping error (Eq. Error), and the
  convergent Born series the paper names as its extension (gamma = i V / eps);
* the exact gradient of a receiver misfit of the truncated series with
  respect to the sound speed (the adjoint of the series; not in the paper);
* the density-contrast term div(gamma_rho grad psi) of Sec. 2.1.3 (which the
  paper drops for rho_s ~ rho_f) in conservative second-order differences,
  added to the potential of every term.

Readings where the paper is silent (each listed in the design notes):
the self-cell value W(0) is the integral of g over the disk (2D) or ball (3D)
of the cell's area/volume; off-diagonal cells are point samples; the
background wavenumber k0 is complex (absorption and dispersion included) and
the shift eps defaults to 0; first-order power-law dispersion
k = omega/c + alpha0 omega^y (i + tan(pi y / 2)) (y == 1: no dispersion term).
"""
from __future__ import annotations

import math
import os
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np
import scipy.fft
import scipy.linalg
import scipy.special

# scipy.fft threads: the host's cores, at most 16 (one GPU's share of a box)
WORKERS = max(1, min(os.cpu_count() or 1, 16))


# ---------------------------------------------------------------- medium ----

def wavenumber(omega: float, c, alpha0: float, y: float):
    """Complex wavenumber of a power-law absorbing, dispersive medium.

    The paper's absorption law is alpha = alpha0 omega^y (Sec. 2.1.2,
    Eq. power_law_absorption), and its frequency-domain operator adds
    -i tau omega (-lap)^{y/2} + eta (-lap)^{(y+1)/2} with
    tau = -2 alpha0 c^{y-1}, eta = 2 alpha0 c^y tan(pi y/2).  For a plane wave
    e^{iKx} that relation, solved to first order in alpha0 about omega/c, is
    K = omega/c + alpha0 omega^y (i + tan(pi y / 2)).  For y == 1 the
    dispersion coefficient is undefined (the paper requires y != 1), and only
    the absorption is kept: K = omega/c + i alpha0 omega."""
    c = np.asarray(c, dtype=np.float64)
    a = alpha0 * omega ** y
    if abs(y - 1.0) < 1e-12:
        return omega / c + 1j * a
    return omega / c + a * (1j + math.tan(math.pi * y / 2.0))


def background_k0(omega: float, c0: float, alpha0: float, y: float, eps: float = 0.0) -> complex:
    """Background wavenumber k0 with k0^2 = k(c0)^2 + i eps (Sec. 2.2,
    Eq. acoustic_waveequn6).  The principal root keeps Im k0 >= 0."""
    kb = complex(wavenumber(omega, c0, alpha0, y))
    return complex(np.sqrt(kb * kb + 1j * eps))


def potential(c, omega: float, c0: float, alpha0: float, y: float, eps: float = 0.0):
    """V(x) = k(x)^2 - k0^2 (Sec. 2.3.3, Eq. TBS_equation_inhomogeneous, with the
    absorption and dispersion of Sec. 2.1.2 carried by the complex k); V = -i eps
    in the background medium, 0 when eps = 0."""
    k = wavenumber(omega, c, alpha0, y)
    k0 = background_k0(omega, c0, alpha0, y, eps)
    return k * k - k0 * k0


def dpotential_dc(c, omega: float, alpha0: float, y: float):
    """dV/dc = 2 k dk/dc = -2 k omega / c^2 (k0 does not depend on c(x))."""
    c = np.asarray(c, dtype=np.float64)
    return -2.0 * wavenumber(omega, c, alpha0, y) * omega / (c * c)


# ------------------------------------------------------- Green's function ---

def green_point(k0: complex, r, ndim: int):
    """Free-space outgoing Green's function of lap g + k0^2 g = -delta
    (Sec. 2.2, Eq. greens_fn): (i/4) H0^(1)(k0 r) in 2D, e^{i k0 r}/(4 pi r) in 3D."""
    r = np.asarray(r, dtype=np.float64)
    if ndim == 2:
        return 0.25j * scipy.special.hankel1(0, k0 * r)
    if ndim == 3:
        return np.exp(1j * k0 * r) / (4.0 * np.pi * r)
    raise ValueError("ndim must be 2 or 3")


def self_cell(k0: complex, dx: float, ndim: int) -> complex:
    """W(0): the integral of g over a disk (2D) / ball (3D) with the cell's
    area / volume.  Closed forms of those integrals:
    2D, a = dx/sqrt(pi):      (i pi a / (2 k0)) H1^(1)(k0 a) - 1/k0^2,
    3D, a = dx (3/(4 pi))^(1/3): ((1 - i k0 a) e^{i k0 a} - 1) / k0^2."""
    if ndim == 2:
        a = dx / math.sqrt(math.pi)
        return complex(1j * math.pi * a / (2.0 * k0) * scipy.special.hankel1(1, k0 * a) - 1.0 / k0 ** 2)
    if ndim == 3:
        a = dx * (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
        return complex(((1.0 - 1j * k0 * a) * np.exp(1j * k0 * a) - 1.0) / k0 ** 2)
    raise ValueError("ndim must be 2 or 3")


def kernel_value(k0: complex, dx: float, offsets) -> np.ndarray:
    """W(m) = dx^d g(k0, |m| dx) for integer offsets m != 0 and the self-cell
    integral for m = 0.  ``offsets``: integer array [..., ndim]."""
    m = np.asarray(offsets, dtype=np.float64)
    ndim = m.shape[-1]
    r = dx * np.sqrt(np.sum(m * m, axis=-1))
    out = np.empty(r.shape, dtype=np.complex128)
    nz = r > 0
    out[nz] = dx ** ndim * green_point(k0, r[nz], ndim)
    out[~nz] = self_cell(k0, dx, ndim)
    return out


def smooth_size(n: int) -> int:
    """Smallest 2,3,5-smooth integer >= n."""
    m = max(int(n), 1)
    while True:
        k = m
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        if k == 1:
            return m
        m += 1


def padded_shape(grid: Sequence[int]) -> Tuple[int, ...]:
    """Zero-padded FFT sizes: smallest 5-smooth M >= 2N - 1 per axis, the
    least size for which the circular convolution equals the linear one."""
    return tuple(smooth_size(2 * n - 1) for n in grid)


def kernel_padded(k0: complex, dx: float, mshape: Sequence[int]) -> np.ndarray:
    """W on the padded periodic grid: index i of an axis of size M holds the
    offset m = i for i <= M/2 and m = i - M otherwise (so for even M the
    otherwise unused index M/2 holds W at offset M/2 and the array stays even
    in every axis)."""
    axes = []
    for M in mshape:
        i = np.arange(M)
        axes.append(np.where(i <= M // 2, i, i - M))
    mesh = np.meshgrid(*axes, indexing="ij")
    offs = np.stack(mesh, axis=-1)
    return kernel_value(k0, dx, offs)


def green_spectrum(k0: complex, dx: float, grid: Sequence[int],
                   mshape: Optional[Sequence[int]] = None) -> np.ndarray:
    """Unnormalised DFT of the padded kernel, fftn(W_pad): the discrete
    counterpart of g~(p) in G = F^-1 g~ F (Sec. 2.2, Eq. TBS_1)."""
    mshape = tuple(mshape) if mshape is not None else padded_shape(grid)
    return scipy.fft.fftn(kernel_padded(k0, dx, mshape), workers=WORKERS)


class GreenOperator:
    """(G f)_i = sum_j W(i - j) f_j on a fixed grid, evaluated as
    crop(ifftn(fftn(W_pad) * fftn(zeropad(f)))) (exact to rounding because the
    padded size is >= 2N - 1 in every axis)."""

    def __init__(self, k0: complex, dx: float, grid: Sequence[int],
                 mshape: Optional[Sequence[int]] = None):
        self.k0, self.dx, self.grid = complex(k0), float(dx), tuple(grid)
        self.mshape = tuple(mshape) if mshape is not None else padded_shape(grid)
        for n, m in zip(self.grid, self.mshape):
            if m < 2 * n - 1:
                raise ValueError("padded size must be >= 2N-1")
        self.ghat = green_spectrum(self.k0, self.dx, self.grid, self.mshape)

    def __call__(self, f: np.ndarray, adjoint: bool = False) -> np.ndarray:
        """Apply G (or G^H, whose spectrum is conj(ghat) since W is even)
        over the trailing ``ndim`` axes of ``f``."""
        nd = len(self.grid)
        axes = tuple(range(-nd, 0))
        F = scipy.fft.fftn(f, s=self.mshape, axes=axes, workers=WORKERS)
        F *= np.conj(self.ghat) if adjoint else self.ghat
        out = scipy.fft.ifftn(F, axes=axes, workers=WORKERS)
        sl = (Ellipsis,) + tuple(slice(0, n) for n in self.grid)
        return np.ascontiguousarray(out[sl])


def apply_green_direct(k0: complex, dx: float, f: np.ndarray) -> np.ndarray:
    """Brute-force (G f)_i = sum_j W(i - j) f_j over all grid pairs (tiny grids)."""
    grid = f.shape
    nd = len(grid)
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), axis=-1).reshape(-1, nd)
    fv = f.reshape(-1)
    out = np.zeros(fv.shape, dtype=np.complex128)
    for j in range(idx.shape[0]):
        if fv[j] == 0:
            continue
        out += kernel_value(k0, dx, idx - idx[j]) * fv[j]
    return out.reshape(grid)


def dense_operator(k0: complex, dx: float, grid: Sequence[int]) -> np.ndarray:
    """A = [W(i - j)] over the flattened grid (P x P)."""
    nd = len(grid)
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), axis=-1).reshape(-1, nd)
    return kernel_value(k0, dx, idx[:, None, :] - idx[None, :, :])


# ------------------------------------------------------------ the series ----

def born_series(apply_g: Callable[[np.ndarray], np.ndarray], s: np.ndarray, V: Optional[np.ndarray],
                nterms: int, ndim: Optional[int] = None, keep_partial_sums: bool = False):
    """Traditional Born series (Sec. 2.2, Eqs. TBS_2, TBS_input, TBS_algorithm):
    u_0 = G s, u_n = G(V u_{n-1}), p = sum_{n=0}^{L-1} u_n.

    ``s`` may carry leading batch axes; V (shared by all of them) fixes the
    number of grid axes, else ``ndim`` does (V = None means V = 0).
    Returns (p, residual) with residual[..., n] = ||u_n|| / ||sum_{m<=n} u_m||
    (L2 over the grid axes, per right-hand side), and also the partial sums
    [P_1, ..., P_{L-1}], P_K = sum_{j<K} u_j, when ``keep_partial_sums``."""
    if nterms < 1:
        raise ValueError("nterms >= 1")
    nd = V.ndim if V is not None else (ndim if ndim is not None else s.ndim)
    grid_axes = tuple(range(-nd, 0))

    def norm(a):
        return np.sqrt(np.sum(np.abs(a) ** 2, axis=grid_axes))

    u = apply_g(s)
    p = u.copy()
    res = [norm(u) / norm(p)]
    partial = [p.copy()] if keep_partial_sums else None
    for n in range(1, nterms):
        u = np.zeros_like(u) if V is None else apply_g(V * u)
        p = p + u
        res.append(norm(u) / norm(p))
        if keep_partial_sums and n < nterms - 1:
            partial.append(p.copy())
    residual = np.stack([np.asarray(r) for r in res], axis=-1)
    if keep_partial_sums:
        return p, residual, partial
    return p, residual


def solve(k0: complex, dx: float, s: np.ndarray, V: Optional[np.ndarray], nterms: int,
          ndim: Optional[int] = None, mshape: Optional[Sequence[int]] = None):
    """FFT-evaluated Born series; the grid is that of V (or the trailing
    ``ndim`` axes of s when V is None)."""
    nd = V.ndim if V is not None else (ndim if ndim is not None else s.ndim)
    G = GreenOperator(k0, dx, s.shape[-nd:], mshape)
    return born_series(G, s, V, nterms, ndim=nd)


def density_operator(gamma: np.ndarray, dx: float, u: np.ndarray) -> np.ndarray:
    """D(u) = div(gamma_rho grad u) on the physical 2D or 3D grid (the density
    term of Sec. 2.1.3, Eq. acoustic_waveequn_time_dependent_inhomogeneous,
    with gamma_rho = (rho_s - rho_f) / rho_s of Eq. mismatch_parameters), in
    conservative second-order differences: per axis
    (g_{+1/2} (u_{+1} - u) - g_{-1/2} (u - u_{-1})) / dx^2 with g at the
    half points the mean of the two cells; u and gamma are 0 outside the grid.
    The grid has gamma.ndim axes (the trailing axes of ``u``, which may carry
    leading batch axes); the axis terms are added x first, then y, then z."""
    nd = gamma.ndim
    g = np.pad(np.asarray(gamma, dtype=np.float64), 1)
    U = np.pad(u, [(0, 0)] * (u.ndim - nd) + [(1, 1)] * nd)
    inner = tuple([slice(1, -1)] * nd)

    def shifted(a, axis, k):
        # a (padded) moved by k cells along grid axis ``axis``, cropped to the grid
        sl = list(inner)
        sl[axis] = slice(1 + k, a.shape[a.ndim - nd + axis] - 1 + k)
        return a[(Ellipsis,) + tuple(sl)]

    c = U[(Ellipsis,) + inner]
    gc = g[inner]
    out = 0.0
    for axis in reversed(range(nd)):
        gp = 0.5 * (gc + shifted(g, axis, 1))
        gm = 0.5 * (gc + shifted(g, axis, -1))
        out = out + gp * (shifted(U, axis, 1) - c) - gm * (c - shifted(U, axis, -1))
    return out / (dx * dx)


def born_series_density(apply_g: Callable[[np.ndarray], np.ndarray], s: np.ndarray, V: np.ndarray,
                        gamma: np.ndarray, dx: float, nterms: int):
    """The series with a density contrast: the equation of Sec. 2.1.3 in the
    frequency domain, lap psi + k0^2 psi = -(s + V psi - div(gamma grad psi)),
    so u_0 = G s, u_n = G(V u_{n-1} - D(u_{n-1})), p = sum_{n<L} u_n, with the
    same residuals as born_series (2D or 3D: the grid axes of gamma)."""
    axes = tuple(range(-gamma.ndim, 0))

    def norm(a):
        return np.sqrt(np.sum(np.abs(a) ** 2, axis=axes))

    u = apply_g(s)
    p = u.copy()
    res = [norm(u) / norm(p)]
    for _ in range(1, nterms):
        u = apply_g(V * u - density_operator(gamma, dx, u))
        p = p + u
        res.append(norm(u) / norm(p))
    return p, np.stack([np.asarray(r) for r in res], axis=-1)


def solve_density(k0: complex, dx: float, s: np.ndarray, V: np.ndarray, gamma: np.ndarray, nterms: int):
    """FFT-evaluated series with a density contrast (2D or 3D)."""
    G = GreenOperator(k0, dx, V.shape)
    return born_series_density(G, s, V, gamma, dx, nterms)


def density_matrix(gamma: np.ndarray, dx: float) -> np.ndarray:
    """Dense matrix of density_operator on the grid of gamma (small grids)."""
    n = gamma.size
    eye = np.eye(n).reshape((n,) + gamma.shape)
    return density_operator(gamma, dx, eye).reshape(n, n).T


def dense_ls(A: np.ndarray, V: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Converged Lippmann-Schwinger field p = G V p + G s (Sec. 2.2, Eq. TBS_1)
    as the dense solve (I - A diag(V)) p = A s."""
    v = V.reshape(-1)
    P = v.size
    p = scipy.linalg.solve(np.eye(P) - A * v[None, :], A @ s.reshape(-1))
    return p.reshape(V.shape)


def spectral_radius(A: np.ndarray, V: np.ndarray) -> float:
    """max |eig(A diag(V))|: the series converges iff it is < 1
    (Sec. 2.2, the condition stated under Eq. TBS_2)."""
    return float(np.max(np.abs(scipy.linalg.eigvals(A * V.reshape(-1)[None, :]))))


# --------------------------------------------------------------- harmonic ---

def harmonic_source(p1: np.ndarray, c, omega: float, rho: float, BA: float) -> np.ndarray:
    """Source of the second-harmonic solve: S2 = -xi (2 omega)^2 p1^2 / 2 with
    xi = (1 + B/(2A)) / (rho c^4) (Sec. 2.1.4, Eq. acoustic_waveequn_time_dependent_nonlinear
    and Eq. nonlinear_waveeqn_shi2 keeping the sum term only; Sec. 2.3.4,
    Eq. TBS_solution_shi_2).  c is the local sound speed."""
    c = np.asarray(c, dtype=np.float64)
    xi = (1.0 + 0.5 * BA) / (rho * c ** 4)
    return -0.5 * xi * (2.0 * omega) ** 2 * p1 * p1


def harmonic_source_n(fields, n: int, c, omega: float, rho: float, BA: float) -> np.ndarray:
    """Source of the n-th harmonic solve (n >= 2) from the lower harmonics
    fields = [psi_1, ..., psi_{n-1}]: S_n = -xi (n omega)^2 * (1/2) sum over
    a + b = n (a, b >= 1, ordered pairs) of psi_a psi_b, i.e. the sum-frequency
    terms of Sec. 2.1.4 (Eqs. of the nonlinear wave equations with sum terms)
    and Sec. 2.3.4 (Eq. TBS_solution_nonlinear_shi_n): psi_1 psi_2 for n = 3,
    psi_2^2 / 2 + psi_1 psi_3 for n = 4, psi_2 psi_3 + psi_1 psi_4 for n = 5.
    xi = (1 + B/(2A)) / (rho c^4) with the local c; omega is the fundamental."""
    if n < 2 or len(fields) < n - 1:
        raise ValueError("need psi_1 .. psi_{n-1}")
    c = np.asarray(c, dtype=np.float64)
    xi = (1.0 + 0.5 * BA) / (rho * c ** 4)
    acc = np.zeros(np.broadcast(fields[0], c).shape, dtype=np.complex128)
    for a in range(1, n):
        b = n - a
        acc = acc + fields[a - 1] * fields[b - 1]
    return -xi * (n * omega) ** 2 * 0.5 * acc


# ------------------------------------------------- periodic (paper) mode ---

def periodic_green_spectrum(k: complex, eps: float, dx: float, shape: Sequence[int]) -> np.ndarray:
    """g~(p) = 1 / (|p|^2 - k^2 - i eps) on the FFT grid of ``shape`` (C order,
    last axis fastest) with p = 2 pi m / (n dx), m the signed FFT index
    (Sec. 2.2, the Fourier transform of g; Algorithm 1's table after its
    fftShift)."""
    axes = [2.0 * np.pi * np.fft.fftfreq(n, d=dx) for n in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    p2 = sum(g * g for g in grids)
    return 1.0 / (p2 - complex(k) ** 2 - 1j * eps)


def kspace_potential(dx: float, shape: Sequence[int], omega: float, tau: float, eta: float,
                     nu: float, eps: float) -> np.ndarray:
    """Case II potential in k-space, VV(p) = eta |p|^(nu+1) - i (tau omega
    |p|^nu + eps) (Sec. 2.3.2 Eq. TBS_solution_absorbing-dispersive; the
    fractional Laplacians become powers of |p|)."""
    axes = [2.0 * np.pi * np.fft.fftfreq(n, d=dx) for n in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    kmod = np.sqrt(sum(g * g for g in grids))
    return eta * kmod ** (nu + 1.0) - 1j * (tau * omega * kmod ** nu + eps)


def tau_eta(alpha0: float, nu: float, c: float) -> Tuple[float, float]:
    """tau = -2 alpha0 c^(nu-1), eta = 2 alpha0 c^nu tan(pi nu / 2) (Sec. 2.1.2,
    the absorption and dispersion proportionality coefficients)."""
    return -2.0 * alpha0 * c ** (nu - 1.0), 2.0 * alpha0 * c ** nu * math.tan(math.pi * nu / 2.0)


def abl_profile(n: int, dx: float, zeta_np_per_cm: float, mu_cells: float) -> np.ndarray:
    """Sigmoid absorbing layer along one axis (Sec. 3.1 Eq. ABL_profile):
    f = 1 / (1 + exp(-zeta (x - mu / 2))) inside a layer of width mu at either
    end, x the distance in cm of the cell from the nearer outer edge; 1
    elsewhere."""
    i = np.arange(n, dtype=np.float64)
    d_cm = np.minimum(i, n - 1 - i) * dx * 100.0
    mu_cm = mu_cells * dx * 100.0
    f = 1.0 / (1.0 + np.exp(-zeta_np_per_cm * (d_cm - 0.5 * mu_cm)))
    return np.where(d_cm < mu_cm, f, 1.0)


def abl_mask(shape: Sequence[int], dx: float, zeta_np_per_cm: float, mu_cells: float) -> np.ndarray:
    """Absorbing-layer mask on a 2D grid: the product of the per-axis profiles."""
    ny, nx = shape
    return np.outer(abl_profile(ny, dx, zeta_np_per_cm, mu_cells), abl_profile(nx, dx, zeta_np_per_cm, mu_cells))


def paper_iterate(gtilde: np.ndarray, s: np.ndarray, V: Optional[np.ndarray] = None,
                  VV: Optional[np.ndarray] = None, mask: Optional[np.ndarray] = None,
                  check_row: Optional[int] = None, tol: float = 1e-5, max_iter: int = 2000):
    """The paper's periodic TBS scheme for one right-hand side ``s``.

    The Lippmann-Schwinger equation psi = G(V psi + S), G = F^-1 g~ F
    (Sec. 2.2, Eq. TBS_1) is solved as a fixed-point iteration that starts
    from psi^0 = G S (Eq. TBS_input).  An update applies Eq. TBS_algorithm with
    the potential of the medium: a pointwise product with V in space (the
    lossless, inhomogeneous and nonlinear media, Eqs. TBS_solution_lossless and
    TBS_solution_inhomogeneous) or, for the absorbing-dispersive medium, a
    product with VV in k-space (Eq. TBS_solution_absorbing-dispersive).  Sec. 3.1
    multiplies every updated field by the sigmoid absorbing layer ``mask`` and
    stops once the relative L1 change of the field on the check row (Eq. Error)
    drops below ``tol``; ``max_iter`` bounds the count.
    Returns (psi, iterations, errors)."""
    S_hat = np.fft.fft2(s)
    row = s.shape[0] // 2 if check_row is None else check_row

    def green(f_hat):
        return np.fft.ifft2(gtilde * f_hat)

    def update(psi):
        if VV is not None:
            return green(VV * np.fft.fft2(psi) + S_hat)
        scattered = 0.0 if V is None else V * psi
        return green(np.fft.fft2(scattered + s))

    def change(new, old):
        return float(np.sum(np.abs(new[row] - old[row])) / np.sum(np.abs(old[row])))

    psi = green(S_hat)
    errs: List[float] = []
    while len(errs) < max_iter:
        new = update(psi)
        if mask is not None:
            new = new * mask
        errs.append(change(new, psi))
        psi = new
        if errs[-1] < tol:
            break
    return psi, len(errs), np.array(errs)


def cbs_iterate(gtilde: np.ndarray, s: np.ndarray, V: np.ndarray, eps: float,
                mask: Optional[np.ndarray] = None, check_row: Optional[int] = None,
                tol: float = 1e-5, max_iter: int = 2000):
    """The convergent Born series the paper names as its extension (Sec. 1 and
    Sec. 5; the preconditioned iteration of Osnabrugge et al., which the paper
    cites): gamma = (i / eps) V, starting from psi_1 = gamma G s, then
      psi_{l+1} = psi_l + gamma (G(V psi_l + s) - psi_l)   [* ABL],
    with G = F^-1 g~ F and V = k^2 - k0^2 - i eps; it converges for
    eps >= max |k^2 - k0^2| (the condition the paper quotes).  Same stopping
    error and return values as paper_iterate (iterations count the updates
    after psi_1)."""
    gamma = 1j * V / eps
    S = np.fft.fft2(s)
    psi = gamma * np.fft.ifft2(gtilde * S)
    c = s.shape[0] // 2 if check_row is None else check_row
    errs = []
    for it in range(1, max_iter + 1):
        new = psi + gamma * (np.fft.ifft2(gtilde * np.fft.fft2(V * psi + s)) - psi)
        if mask is not None:
            new = new * mask
        err = float(np.sum(np.abs(new[c] - psi[c])) / np.sum(np.abs(psi[c])))
        errs.append(err)
        psi = new
        if err < tol:
            return psi, it, np.array(errs)
    return psi, max_iter, np.array(errs)


def periodic_helmholtz_dense(k2: np.ndarray, dx: float, s: np.ndarray) -> np.ndarray:
    """Direct solve of -lap psi - k(x)^2 psi = s on the periodic grid with the
    spectral Laplacian (|p|^2 in k-space): the equation the periodic
    iterations converge to (Sec. 2.2 Eq. acoustic_waveequn5 with U = k^2 - k_f^2).
    Dense, for grids of a few hundred points."""
    ny, nx = s.shape
    n = nx * ny
    px = 2.0 * np.pi * np.fft.fftfreq(nx, d=dx)
    py = 2.0 * np.pi * np.fft.fftfreq(ny, d=dx)
    P2 = (py[:, None] ** 2 + px[None, :] ** 2).ravel()
    eye = np.eye(n).reshape(n, ny, nx)
    lap = np.fft.ifft2(np.fft.fft2(eye) * P2.reshape(ny, nx)[None]).reshape(n, n).T
    A = lap - np.diag(np.asarray(k2).ravel())
    return np.linalg.solve(A, s.ravel()).reshape(ny, nx)


# ---------------------------------------------------------------- adjoint ---

def receiver_misfit(p: np.ndarray, receivers: np.ndarray, p_obs: np.ndarray):
    """J = 1/2 sum |R p - p_obs|^2 and the adjoint source q = R^H (R p - p_obs).
    ``p``: [S][...grid]; ``receivers``: [R][ndim] cell indices; ``p_obs``: [S][R]."""
    rr = tuple(receivers.T)
    r = p[(slice(None),) + rr] - p_obs
    J = 0.5 * float(np.sum(np.abs(r) ** 2))
    q = np.zeros_like(p)
    for b in range(p.shape[0]):
        np.add.at(q[b], rr, r[b])
    return J, q


def adjoint_series_gradient(G: GreenOperator, s: np.ndarray, V: np.ndarray, nterms: int,
                            q: np.ndarray) -> np.ndarray:
    """Gradient of Re<q, p_L> with respect to V for the L-term series:
    g_V = sum_{m=0}^{L-2} conj(w_m) * P_{L-1-m}, with w_0 = G^H q,
    w_m = G^H(conj(V) w_{m-1}) and P_K = sum_{j<K} u_j, so that
    d Re<q, p_L> = Re sum dV * g_V.  (Zero for L = 1.)"""
    _, _, partial = born_series(G, s, V, nterms, keep_partial_sums=True)
    g = np.zeros(V.shape, dtype=np.complex128)
    w = G(q, adjoint=True)
    for m in range(0, nterms - 1):
        g += np.conj(w) * partial[nterms - 2 - m]          # P_{L-1-m} = partial[L-2-m]
        w = G(np.conj(V) * w, adjoint=True)
    return g


def misfit_gradient(c: np.ndarray, freqs: Sequence[float], dx: float, c0: float, alpha0: float,
                    y: float, sources: np.ndarray, receivers: np.ndarray,
                    p_obs: Sequence[np.ndarray], nterms: int):
    """J(c) = 1/2 sum_{f,s} ||R p_{f,s}(c) - p_obs_{f,s}||^2 and dJ/dc(x) =
    sum_{f,s} Re(g_V(x) dV/dc(x)).  ``p_obs[f]`` is [S][R]."""
    J = 0.0
    grad = np.zeros(c.shape)
    for fi, f in enumerate(freqs):
        omega = 2.0 * math.pi * f
        k0 = background_k0(omega, c0, alpha0, y)
        V = potential(c, omega, c0, alpha0, y)
        G = GreenOperator(k0, dx, c.shape)
        p, _ = born_series(G, sources, V, nterms)
        Jf, q = receiver_misfit(p, receivers, p_obs[fi])
        J += Jf
        gV = np.zeros(c.shape, dtype=np.complex128)
        for b in range(sources.shape[0]):
            gV += adjoint_series_gradient(G, sources[b], V, nterms, q[b])
        grad += np.real(gV * dpotential_dc(c, omega, alpha0, y))
    return J, grad
