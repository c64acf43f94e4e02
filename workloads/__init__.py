"""Seeded synthetic workloads for the Born-series Helmholtz solver.

This module only *describes and synthesises inputs*: grids, sound-speed maps,
absorption laws (converted to SI units) and dense source arrays.  It holds none
of the solver's arithmetic (no wavenumber, potential, Green's function, FFT
convolution or series).  Both the FP64 oracle (``oracle/``) and the GPU library
(``paper_2507_13754_amd``) consume what it produces, each computing the method
independently.

Every array is float64/complex128, C order, x fastest: 2D arrays are ``[y][x]``,
3D arrays are ``[z][y][x]``.  A grid cell with integer index ``i`` sits at
physical position ``i*dx``.

The five workloads follow the transducer-field setups of the paper (a line array
of point elements in tissue-like media, power-law absorption, weak speed
contrast; Sec. 3.1) at the sizes of the measurement plan:

1. ``plain2d``     256^2, 1 MHz, Gaussian random field c(x), 16 terms.
2. ``absorb2d``    2048^2, 5 MHz, blob medium, power law y=1.5, 30 terms.
3. ``broadband``   48 frequencies 2-8 MHz on their own grids, 16 steering
                   angles each, 25 terms.
4. ``harmonic3d``  256^3, 3 MHz fundamental + 6 MHz second harmonic, 24 terms.
5. ``adjoint2d``   1024^2, 16 frequencies x 8 sources, 128 receivers, 25 terms.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

C0 = 1540.0          # background sound speed used by every workload [m/s]
RHO0 = 1000.0        # density [kg/m^3]
DB_PER_NP = 20.0 / math.log(10.0)   # 8.6859 dB per neper


def alpha0_si(alpha_db_cm_mhz: float, y: float) -> float:
    """Convert a power-law absorption prefactor from dB/(MHz^y cm) to
    Np m^-1 (rad/s)^-y, the units of the power law alpha = alpha0 * omega^y
    (Sec. 2.1.2, Eq. power_law_absorption)."""
    np_per_m = alpha_db_cm_mhz * 100.0 / DB_PER_NP       # at 1 MHz
    return np_per_m / (2.0 * math.pi * 1.0e6) ** y


def gaussian_random_field(shape: Sequence[int], ell_cells: float, seed: int) -> np.ndarray:
    """Zero-mean, unit-sample-std periodic Gaussian random field.

    White N(0,1) noise (PCG64 ``seed``) filtered in Fourier space by
    exp(-|kappa|^2 ell^2 / 8), which gives the covariance exp(-r^2/ell^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal(tuple(shape))
    kap2 = np.zeros(tuple(shape))
    for ax, n in enumerate(shape):
        k = 2.0 * np.pi * np.fft.fftfreq(n)              # rad per cell
        sh = [1] * len(shape)
        sh[ax] = n
        kap2 = kap2 + (k.reshape(sh)) ** 2
    filt = np.exp(-kap2 * ell_cells ** 2 / 8.0)
    g = np.real(np.fft.ifftn(np.fft.fftn(white) * filt))
    g -= g.mean()
    g /= g.std()
    return g


@dataclasses.dataclass(frozen=True)
class Blobs:
    """Analytic sum of Gaussian blobs, amp_b * exp(-|x - x_b|^2 / r_b^2),
    clipped to [-clip, clip].  Positions and radii in metres."""
    centres: np.ndarray      # [nb][ndim], (x, y[, z]) order
    radii: np.ndarray        # [nb]
    amps: np.ndarray         # [nb]
    clip: float

    def evaluate(self, shape: Sequence[int], dx: float) -> np.ndarray:
        """Field on the cell centres of a grid with the given ``shape``
        (C order, x fastest) and spacing ``dx``."""
        ndim = len(shape)
        axes = [np.arange(n) * dx for n in reversed(shape)]          # x, y, z
        out = np.zeros(tuple(shape))
        for c, r, a in zip(self.centres, self.radii, self.amps):
            d2 = np.zeros(tuple(shape))
            for ax in range(ndim):
                sh = [1] * ndim
                sh[ndim - 1 - ax] = shape[ndim - 1 - ax]
                d2 = d2 + ((axes[ax] - c[ax]) ** 2).reshape(sh)
            out += a * np.exp(-d2 / (r * r))
        return np.clip(out, -self.clip, self.clip)


def random_blobs(ndim: int, extent: float, count: int, seed: int,
                 radius=(1e-3, 4e-3), amp=0.03, clip=None) -> Blobs:
    """``count`` blobs with centres uniform in [0, extent)^ndim, radii uniform in
    ``radius`` and amplitudes uniform in [-amp, amp]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.0, extent, size=(count, ndim))
    radii = rng.uniform(radius[0], radius[1], size=count)
    amps = rng.uniform(-amp, amp, size=count)
    return Blobs(centres, radii, amps, amp if clip is None else clip)


@dataclasses.dataclass
class Case:
    """One single-frequency solve: everything a solver needs besides the method.

    ``sources``: complex128 ``[B][...grid]`` dense source densities (one cell per
    array element holding ``a_e / dx^ndim``).  ``c``: float64 sound speed on the
    grid.  ``alpha0``/``y``: power law in SI units (y == 1 means no dispersion)."""
    name: str
    grid: Tuple[int, ...]            # C order (z, y, x) / (y, x)
    dx: float
    freq: float
    c0: float
    alpha0: float
    y: float
    nterms: int
    c: np.ndarray
    sources: np.ndarray
    rho: float = RHO0
    BA: float = 7.0

    @property
    def ndim(self) -> int:
        return len(self.grid)

    @property
    def omega(self) -> float:
        return 2.0 * math.pi * self.freq

    @property
    def points(self) -> int:
        return int(np.prod(self.grid))


def element_sources(grid: Sequence[int], dx: float, cells: Sequence[Tuple[int, ...]],
                    amps: np.ndarray) -> np.ndarray:
    """Dense source arrays ``[B][...grid]``: element e of RHS b puts
    ``amps[b, e] / dx^ndim`` on cell ``cells[e]`` (C-order index tuple).  Two
    elements on one cell add."""
    amps = np.atleast_2d(np.asarray(amps, dtype=np.complex128))
    ndim = len(grid)
    s = np.zeros((amps.shape[0],) + tuple(grid), dtype=np.complex128)
    for e, cell in enumerate(cells):
        s[(slice(None),) + tuple(cell)] += amps[:, e] / dx ** ndim
    return s


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def plain2d(n: int = 256, nterms: int = 16, seed: int = 1, nrhs: int = 1) -> Case:
    """256^2 grid, dx = lambda/8 at 1 MHz, c = c0 (1 + 0.01 g) with g a unit
    Gaussian random field of correlation length 2 lambda; 0.5 dB/cm/MHz, y = 1;
    32 elements on row 8, columns 64 + 4e (pitch lambda/2), unit amplitude."""
    f = 1.0e6
    lam = C0 / f
    dx = lam / 8.0
    g = gaussian_random_field((n, n), ell_cells=2.0 * lam / dx, seed=seed)
    c = C0 * (1.0 + 0.01 * g)
    nel = 32
    x0 = n // 4
    cells = [(min(8, n - 1), min(x0 + 4 * e, n - 1)) for e in range(nel)]
    amps = np.ones((nrhs, nel), dtype=np.complex128)
    if nrhs > 1:   # extra RHS: deterministic apodisations
        for b in range(1, nrhs):
            amps[b] = np.exp(1j * 0.1 * b * np.arange(nel))
    return Case("plain2d", (n, n), dx, f, C0, alpha0_si(0.5, 1.0), 1.0, nterms, c,
                element_sources((n, n), dx, cells, amps))


def absorb2d(n: int = 2048, nterms: int = 30, seed: int = 2, nrhs: int = 1) -> Case:
    """2048^2 grid at dx = lambda/6, 5 MHz; blobs (1 per cm^2, radius 1-4 mm,
    +-3 %, clipped to +-3 %); 0.75 dB/(MHz^1.5 cm), y = 1.5; 64 elements on
    row 8 at pitch 3 dx, centred."""
    f = 5.0e6
    dx = C0 / f / 6.0
    extent = n * dx
    count = max(1, int(round(extent * extent * 1e4)))
    blobs = random_blobs(2, extent, count, seed)
    c = C0 * (1.0 + blobs.evaluate((n, n), dx))
    nel = 64
    x0 = n // 2 - (nel * 3) // 2
    cells = [(min(8, n - 1), min(max(x0 + 3 * e, 0), n - 1)) for e in range(nel)]
    amps = np.ones((nrhs, nel), dtype=np.complex128)
    for b in range(1, nrhs):
        amps[b] = np.exp(1j * 0.05 * b * np.arange(nel))
    return Case("absorb2d", (n, n), dx, f, C0, alpha0_si(0.75, 1.5), 1.5, nterms, c,
                element_sources((n, n), dx, cells, amps))


BROADBAND_FREQS = [2.0e6 + 6.0e6 * i / 47.0 for i in range(48)]
BROADBAND_ANGLES = [math.radians(-30.0 + 4.0 * j) for j in range(16)]


def broadband(freq_index: int, nangles: int = 16, nterms: int = 25, seed: int = 3,
              extent: float = 0.04) -> Case:
    """One frequency of the broadband workload: 48 frequencies 2-8 MHz, each
    on its own grid at dx = lambda/6 over a 4 x 4 cm domain; one analytic blob
    medium (16 blobs, seed 3) sampled per grid; 64 elements at pitch 0.154 mm,
    0.4 mm from the edge, nearest cell; ``nangles`` steering angles."""
    f = BROADBAND_FREQS[freq_index]
    dx = C0 / f / 6.0
    n = int(round(extent / dx))
    blobs = random_blobs(2, extent, 16, seed)
    c = C0 * (1.0 + blobs.evaluate((n, n), dx))
    nel = 64
    pitch = 0.154e-3
    xs = extent / 2.0 + (np.arange(nel) - (nel - 1) / 2.0) * pitch
    row = int(round(0.4e-3 / dx))
    cells = [(row, int(round(x / dx))) for x in xs]
    xc = extent / 2.0
    omega = 2.0 * math.pi * f
    amps = np.array([[np.exp(1j * omega * (xe - xc) * math.sin(th) / C0) for xe in xs]
                     for th in BROADBAND_ANGLES[:nangles]])
    return Case(f"broadband[{freq_index}]", (n, n), dx, f, C0, alpha0_si(0.75, 1.5), 1.5,
                nterms, c, element_sources((n, n), dx, cells, amps))


def harmonic3d(n: int = 256, nterms: int = 24, seed: int = 4) -> Case:
    """256^3 grid at dx = lambda/6 at 3 MHz; 3D blobs (1 per cm^3, +-2 %);
    config-2 absorption law; rho = 1000, B/A = 7; 64 elements along x at pitch
    3 dx, y = N/2, z = 8.  The case is the fundamental; the harmonic solve uses
    ``2*freq`` on the same grid."""
    f = 3.0e6
    dx = C0 / f / 6.0
    extent = n * dx
    count = max(1, int(round(extent ** 3 * 1e6)))
    blobs = random_blobs(3, extent, count, seed, amp=0.02)
    c = C0 * (1.0 + blobs.evaluate((n, n, n), dx))
    nel = min(64, max(1, n // 3))
    x0 = n // 2 - (nel * 3) // 2
    cells = [(min(8, n - 1), n // 2, x0 + 3 * e) for e in range(nel)]
    amps = np.ones((1, nel), dtype=np.complex128)
    return Case("harmonic3d", (n, n, n), dx, f, C0, alpha0_si(0.75, 1.5), 1.5, nterms, c,
                element_sources((n, n, n), dx, cells, amps), rho=RHO0, BA=7.0)


ADJOINT_FREQS = [2.0e6 + 4.0e6 * i / 15.0 for i in range(16)]


@dataclasses.dataclass
class AdjointProblem:
    """Sound-speed misfit problem: model map, true map, point sources,
    receivers, frequencies.  ``receivers`` are (row, col) cells."""
    grid: Tuple[int, int]
    dx: float
    freqs: List[float]
    c_model: np.ndarray
    c_true: np.ndarray
    sources: np.ndarray          # [S][Ny][Nx] complex128
    receivers: np.ndarray        # [R][2] int64 (row, col)
    alpha0: float
    y: float
    nterms: int
    fd_pixels: np.ndarray        # [64][2] int64 (row, col)


def adjoint2d(n: int = 1024, nfreq: int = 16, nsrc: int = 8, nrec: int = 128,
              nterms: int = 25, seed: int = 5) -> AdjointProblem:
    """1024^2 grid at dx = lambda/6 at 6 MHz; model map blobs +-3 % (seed 5);
    true map = model * (1 + 0.02 h), h a clipped blob field (seed 50); 8 point
    sources on row 8, columns 64 + 128 s; 128 receivers on row N-9, columns
    4 + 8 r; 64 FD pixels (seed 55).  Grid positions scale with ``n``
    (receivers that would share a cell after scaling are merged)."""
    dx = C0 / 6.0e6 / 6.0
    extent = n * dx
    scale = n / 1024.0
    count = max(1, int(round(extent * extent * 1e4)))
    c_model = C0 * (1.0 + random_blobs(2, extent, count, seed).evaluate((n, n), dx))
    h = random_blobs(2, extent, count, seed * 10, amp=1.0).evaluate((n, n), dx)
    c_true = c_model * (1.0 + 0.02 * h)
    src_cells = [(min(8, n - 1), min(int(round((64 + 128 * s) * scale)), n - 1)) for s in range(nsrc)]
    s = np.zeros((nsrc, n, n), dtype=np.complex128)
    for i, cell in enumerate(src_cells):
        s[(i,) + cell] = 1.0 / dx ** 2
    cols = sorted({min(int(round((4 + 8 * r) * scale)), n - 1) for r in range(nrec)})
    rec = np.array([(n - 9, col) for col in cols], dtype=np.int64)   # distinct cells
    rng = np.random.Generator(np.random.PCG64(seed * 11))
    lo, hi = int(0.2 * n), int(0.8 * n)
    fd = np.stack([rng.integers(lo, hi, 64), rng.integers(lo, hi, 64)], axis=1).astype(np.int64)
    freqs = [ADJOINT_FREQS[int(round(i * 15 / max(nfreq - 1, 1)))] for i in range(nfreq)] \
        if nfreq < 16 else list(ADJOINT_FREQS)
    return AdjointProblem((n, n), dx, freqs, c_model, c_true, s, rec,
                          alpha0_si(0.75, 1.5), 1.5, nterms, fd)


def random_field(shape: Sequence[int], seed: int, dtype=np.complex128) -> np.ndarray:
    """Seeded standard-normal (complex: independent re/im) test field."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if np.dtype(dtype).kind == "c":
        return (rng.standard_normal(tuple(shape)) + 1j * rng.standard_normal(tuple(shape))).astype(dtype)
    return rng.standard_normal(tuple(shape)).astype(dtype)


def small_medium(grid: Sequence[int], dx: float, contrast: float, seed: int) -> np.ndarray:
    """Sound speed c0 (1 + contrast * g) with g a smooth unit GRF (correlation
    length 4 cells); for parity tests on small ragged grids."""
    return C0 * (1.0 + contrast * gaussian_random_field(grid, 4.0, seed))


# --------------------------------------------------- the paper's own setups --

@dataclasses.dataclass
class PeriodicCase:
    """Inputs of the paper's periodic scheme (Sec. 3.1, Algorithm 1)."""
    name: str
    n: int
    dx: float
    c0: float
    omega: float
    eps_factor: float          # eps = eps_factor * (omega / c0)^2
    c: np.ndarray              # sound speed map [n][n] (scatterer inside)
    sources: np.ndarray        # [1][n][n] complex grid values of S
    alpha0: float              # Case II power law (0: no k-space potential)
    nu: float
    dispersion: bool           # Case II: keep the dispersion (eta) term
    zeta: float                # absorbing layer, Np/cm
    mu_cells: float            # absorbing layer width in cells
    check_row: int
    tol: float = 1e-5
    max_iter: int = 2000


def paper_periodic(case: str = "homogeneous", n: int = 4096, vs: float = 1650.0) -> PeriodicCase:
    """The paper's 2D transducer setup scaled to n cells per side (n = 4096:
    the paper's grid): dx = 20 um, v_f = 1500 m/s, f = 55 v_f / (4096 dx)
    = 1007080 Hz, eps = 0.8 k_f^2, a line of 501 (scaled: 501 n / 4096, odd)
    point sources of value -1e6 i at column 675 (scaled) centred on the
    middle row, the absorbing layer zeta = 21.48 Np/cm over 450 cells
    (scaled), the stopping row = the middle row, tol 1e-5, 2000 iterations
    at most.  case: "homogeneous" (Case I, lossless), "absorbing" (Case II
    with alpha0 = 5.5e-10, nu = 1.5 and the dispersion term dropped),
    "absorbing-dispersive" (Case II with both terms), "inhomogeneous"
    (Case III: a disk of radius 50 cells (scaled) and speed vs at the domain
    centre)."""
    if case not in ("homogeneous", "absorbing", "absorbing-dispersive", "inhomogeneous"):
        raise ValueError(case)
    dx, c0 = 20e-6, 1500.0
    f = 55.0 * c0 / (4096 * dx)
    s = n / 4096.0
    c = np.full((n, n), c0)
    if case == "inhomogeneous":
        r = max(2.0, 50.0 * s)
        yy, xx = np.mgrid[0:n, 0:n]
        c[(yy - n // 2) ** 2 + (xx - n // 2) ** 2 <= r * r] = vs
    src = np.zeros((1, n, n), np.complex128)
    half = max(1, int(round(250 * s)))
    col = max(1, int(round(675 * s)) - 1)
    src[0, n // 2 - half: n // 2 + half + 1, col] = -1e6j
    a0 = 5.5e-10 if case in ("absorbing", "absorbing-dispersive") else 0.0
    return PeriodicCase(name=f"paper-{case}-{n}", n=n, dx=dx, c0=c0, omega=2 * math.pi * f,
                        eps_factor=0.8, c=c, sources=src, alpha0=a0, nu=1.5,
                        dispersion=case == "absorbing-dispersive", zeta=21.48,
                        mu_cells=max(2.0, 450.0 * s), check_row=n // 2)
