"""Pins of the FP64 oracle against facts other than itself (CPU only).

Each test checks the oracle against something the paper or the mathematics
fixes: a brute-force sum, the PDE the Green's function solves, an independent
quadrature, a textbook dense solve, an invariant, a printed constant, or a
finite difference.  A dropped term, a wrong sign/factor, a transposed operand
or a wrong pad/crop in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.special

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# ---------------------------------------------------------------- P1 --------

@pytest.mark.parametrize("grid,mshapes", [
    ((13, 10), [None, (25, 19), (26, 20), (32, 27)]),
    ((7, 9), [None, (14, 18), (13, 17)]),
])
def test_direct_sum_equals_fft_2d(grid, mshapes):
    """Brute-force sum_j W(i-j) f_j equals the zero-padded FFT evaluation for
    every admissible padded size (pins padding, crop, index wrap, scaling)."""
    k0 = 2 * np.pi / 6.0 * (1 + 0.03j)
    dx = 1.0
    f = workloads.random_field(grid, seed=11)
    ref = oracle.apply_green_direct(k0, dx, f)
    for ms in mshapes:
        G = oracle.GreenOperator(k0, dx, grid, ms)
        assert rel(G(f), ref) < 1e-13, ms


def test_direct_sum_equals_fft_3d():
    grid = (6, 5, 7)
    k0 = 2 * np.pi / 5.0 * (1 + 0.02j)
    dx = 0.7
    f = workloads.random_field(grid, seed=12)
    ref = oracle.apply_green_direct(k0, dx, f)
    for ms in [None, (12, 10, 14), (16, 9, 15)]:
        G = oracle.GreenOperator(k0, dx, grid, ms)
        assert rel(G(f), ref) < 1e-13, ms


def test_padding_below_linear_size_rejected():
    with pytest.raises(ValueError):
        oracle.GreenOperator(1.0, 1.0, (8, 8), (14, 16))


# ------------------------------------------------- Green's function (PDE) ---

def _helmholtz_residual(ndim, ppw, extent):
    lam = 1.0
    k0 = 2 * np.pi / lam * (1 + 0.02j)
    dx = lam / ppw
    n = int(round(extent / dx))
    grid = (n,) * ndim
    axes = np.meshgrid(*[np.arange(n) * dx for _ in range(ndim)], indexing="ij")
    xc = (n // 2) * dx
    sig = 0.35
    f = np.exp(-sum((a - xc) ** 2 for a in axes) / sig ** 2).astype(np.complex128)
    u = oracle.GreenOperator(k0, dx, grid)(f)
    lap = np.zeros_like(u)
    for ax in range(ndim):
        r = lambda s: np.roll(u, s, axis=ax)  # noqa: E731
        lap += (-r(2) + 16 * r(1) - 30 * u + 16 * r(-1) - r(-2)) / (12 * dx * dx)
    res = lap + k0 * k0 * u + f
    inner = tuple(slice(3, n - 3) for _ in range(ndim))
    return float(np.linalg.norm(res[inner]) / np.linalg.norm(f[inner]))


@pytest.mark.parametrize("ndim,ppws,extent", [(2, (16, 32), 3.0), (3, (8, 16), 2.0)])
def test_green_operator_solves_helmholtz(ndim, ppws, extent):
    """u = G f satisfies lap u + k0^2 u = -f (Sec. 2.2, Eqs. soln_greens_fn and
    greens_fn) up to the O(dx^2) cell-quadrature error: the residual is small
    and falls about 4x when dx halves.  A wrong Green's-function constant,
    sign, Hankel kind, dx^d factor or self-cell value leaves an O(1) residual."""
    r1 = _helmholtz_residual(ndim, ppws[0], extent)
    r2 = _helmholtz_residual(ndim, ppws[1], extent)
    assert r2 < (3e-3 if ndim == 2 else 1.5e-2), (r1, r2)
    assert 2.8 < r1 / r2 < 6.0, (r1, r2)


@pytest.mark.parametrize("k0", [2 * np.pi / 6 * (1 + 0.004j), 0.9 + 0.2j, 2.5 + 0.0j])
def test_self_cell_matches_quadrature(k0):
    """W(0) equals the integral of g over the equal-area disk / equal-volume
    ball computed by adaptive quadrature."""
    dx = 1.0
    a2 = dx / math.sqrt(math.pi)
    f2 = lambda r, part: part(0.25j * scipy.special.hankel1(0, k0 * r) * 2 * np.pi * r)  # noqa: E731
    q2 = (scipy.integrate.quad(f2, 0, a2, args=(np.real,), epsabs=0, epsrel=1e-13, limit=200)[0]
          + 1j * scipy.integrate.quad(f2, 0, a2, args=(np.imag,), epsabs=0, epsrel=1e-13, limit=200)[0])
    assert abs(oracle.self_cell(k0, dx, 2) - q2) < 1e-12 * abs(q2)
    a3 = dx * (3 / (4 * math.pi)) ** (1 / 3)
    f3 = lambda r, part: part(np.exp(1j * k0 * r) / (4 * np.pi * r) * 4 * np.pi * r * r)  # noqa: E731
    q3 = (scipy.integrate.quad(f3, 0, a3, args=(np.real,), epsabs=0, epsrel=1e-13)[0]
          + 1j * scipy.integrate.quad(f3, 0, a3, args=(np.imag,), epsabs=0, epsrel=1e-13)[0])
    assert abs(oracle.self_cell(k0, dx, 3) - q3) < 1e-12 * abs(q3)


@pytest.mark.parametrize("ndim", [2, 3])
def test_point_source_gives_green_function(ndim):
    """A unit point source (density 1/dx^d on one cell) with V = 0 gives
    u_0(x) = g(k0, |x - x0|) off the source cell."""
    grid = (11, 9) if ndim == 2 else (7, 6, 5)
    dx = 0.25
    k0 = 2 * np.pi * (1 + 0.01j)
    src = tuple(n // 3 for n in grid)
    s = np.zeros(grid, dtype=np.complex128)
    s[src] = 1.0 / dx ** ndim
    p, res = oracle.solve(k0, dx, s, None, 1, ndim=ndim)
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), axis=-1)
    r = dx * np.sqrt(np.sum((idx - np.array(src)) ** 2, axis=-1))
    mask = r > 0
    if ndim == 2:
        g = 0.25j * scipy.special.hankel1(0, k0 * r[mask])
    else:
        g = np.exp(1j * k0 * r[mask]) / (4 * np.pi * r[mask])
    assert rel(p[mask], g) < 1e-12


# ---------------------------------------------------------------- series ----

def test_zero_potential_gives_first_term_only():
    """V = 0: every u_n (n >= 1) is exactly zero and p = u_0."""
    grid = (12, 10)
    k0 = 1.3 + 0.05j
    s = workloads.random_field(grid, 3)
    G = oracle.GreenOperator(k0, 0.5, grid)
    p, res = oracle.born_series(G, s, np.zeros(grid, np.complex128), 5)
    assert np.array_equal(p, G(s))
    assert res[0] == 1.0 and np.all(res[1:] == 0.0)


def _small_problem(rho_target, n=12, seed=4):
    grid = (n, n)
    dx = 1.0
    k0 = 2 * np.pi / 6.0 * (1 + 0.01j)
    V = workloads.random_field(grid, seed) * np.exp(-((np.arange(n)[:, None] - n / 2) ** 2
                                                      + (np.arange(n)[None, :] - n / 2) ** 2) / 9.0)
    A = oracle.dense_operator(k0, dx, grid)
    rho = oracle.spectral_radius(A, V)
    V = V * (rho_target / rho)
    s = np.zeros(grid, np.complex128)
    s[1, 3] = 1.0
    s[1, 7] = -0.5j
    return k0, dx, grid, A, V, s


def test_series_converges_to_dense_ls_when_radius_below_one():
    """rho(GV) < 1: partial sums approach the dense Lippmann-Schwinger solution
    (Sec. 2.2, Eq. TBS_1) geometrically at rate rho (the condition stated under
    Eq. TBS_2)."""
    k0, dx, grid, A, V, s = _small_problem(0.5)
    assert abs(oracle.spectral_radius(A, V) - 0.5) < 1e-10
    p_inf = oracle.dense_ls(A, V, s)
    G = oracle.GreenOperator(k0, dx, grid)
    errs = [rel(oracle.born_series(G, s, V, L)[0], p_inf) for L in (10, 20, 40)]
    assert errs[2] < 1e-9
    assert errs[1] < errs[0] * 0.5 ** 10 * 30
    assert errs[1] > errs[0] * 0.5 ** 10 / 30


def test_series_diverges_when_radius_above_one():
    k0, dx, grid, A, V, s = _small_problem(1.3)
    G = oracle.GreenOperator(k0, dx, grid)
    _, res = oracle.born_series(G, s, V, 60)
    # ||u_n|| / ||p_{n+1}|| tends to a nonzero limit (terms outgrow the sum's
    # convergence), while for rho < 1 it tends to 0.
    assert res[-1] > 0.1
    _, res_ok = oracle.born_series(G, s, V * (0.5 / 1.3), 60)
    assert res_ok[-1] < 1e-12


def test_partial_sum_ls_residual_is_next_term():
    """p_L - G(V p_L) - G s = -u_L for every L (the recursion under
    Eq. TBS_1)."""
    k0, dx, grid, A, V, s = _small_problem(0.7)
    G = oracle.GreenOperator(k0, dx, grid)
    for L in (1, 2, 5):
        pL, _ = oracle.born_series(G, s, V, L)
        pL1, _ = oracle.born_series(G, s, V, L + 1)
        uL = pL1 - pL
        lhs = pL - G(V * pL) - G(s)
        assert rel(lhs, -uL) < 1e-12


def test_dense_operator_matches_fft_operator():
    k0, dx, grid, A, V, s = _small_problem(0.5, n=9)
    f = workloads.random_field(grid, 8)
    assert rel(oracle.GreenOperator(k0, dx, grid)(f), (A @ f.ravel()).reshape(grid)) < 1e-13


@pytest.mark.parametrize("L", [1, 3, 8])
def test_reciprocity(L):
    """W is even, so every truncated term operator (GV)^n G is complex
    symmetric: the field at B from a point source at A equals the field at A
    from B, for any V and L."""
    grid = (14, 11)
    dx = 1.0
    k0 = 2 * np.pi / 5 * (1 + 0.02j)
    V = 0.05 * workloads.random_field(grid, 21)
    a, b = (2, 3), (11, 8)
    s = np.zeros((2,) + grid, np.complex128)
    s[(0,) + a] = 1.0
    s[(1,) + b] = 1.0
    p, _ = oracle.solve(k0, dx, s, V, L)
    assert abs(p[(0,) + b] - p[(1,) + a]) < 1e-13 * abs(p[(0,) + b])


def test_batch_is_linear_and_matches_single():
    grid = (10, 12)
    k0 = 1.1 + 0.1j
    V = 0.2 * workloads.random_field(grid, 5)
    s = workloads.random_field((3,) + grid, 6)
    pb, rb = oracle.solve(k0, 0.8, s, V, 6)
    for b in range(3):
        p1, r1 = oracle.solve(k0, 0.8, s[b], V, 6)
        assert rel(pb[b], p1) < 1e-14 and np.allclose(rb[b], r1, rtol=1e-13)
    pc, _ = oracle.solve(k0, 0.8, 2.0 * s[0] - 1j * s[1], V, 6)
    assert rel(pc, 2.0 * pb[0] - 1j * pb[1]) < 1e-13


def test_residual_definition():
    grid = (8, 8)
    k0 = 1.1 + 0.1j
    V = 0.2 * workloads.random_field(grid, 5)
    s = workloads.random_field(grid, 6)
    G = oracle.GreenOperator(k0, 1.0, grid)
    p3, r3 = oracle.born_series(G, s, V, 3)
    p2, _ = oracle.born_series(G, s, V, 2)
    assert r3[0] == pytest.approx(1.0)
    assert r3[2] == pytest.approx(np.linalg.norm(p3 - p2) / np.linalg.norm(p3), rel=1e-13)


# ----------------------------------------------------------- medium model ---

def test_paper_constants():
    """Scalars the paper prints (golden file with citations)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    prm = g["params"]
    f = prm["multiple"] * prm["v_f"] / (prm["n_grid"] * prm["dx"])
    assert f == pytest.approx(g["frequency_hz"]["value"], rel=g["frequency_hz"]["rtol"])
    kf = 2 * np.pi * g["frequency_hz"]["value"] / prm["v_f"]
    assert kf * prm["a"] == pytest.approx(g["kf_a"]["value"], rel=g["kf_a"]["rtol"])
    tau, eta = oracle.tau_eta(prm["alpha0"], prm["nu"], prm["v_f"])
    assert tau == pytest.approx(g["tau"]["value"], rel=g["tau"]["rtol"])
    assert eta == pytest.approx(g["eta"]["value"], rel=g["eta"]["rtol"])
    assert workloads.alpha0_si(0.75, 1.5) == pytest.approx(g["alpha0_si"]["value"], rel=g["alpha0_si"]["rtol"])


def test_wavenumber_solves_paper_dispersion_relation_to_first_order():
    """K from ``oracle.wavenumber`` makes the plane-wave symbol of the paper's
    absorbing-dispersive Helmholtz operator (Sec. 2.1.2, Eq.
    acoustic_waveequn_time_independent_absorbing_dispersion),
    -K^2 + k_f^2 - i tau omega K^y + eta K^(y+1), vanish to first order in
    alpha0: the symbol falls as alpha0^2 (a wrong sign or factor in the
    absorption or dispersion term leaves an O(alpha0) symbol)."""
    omega, c, y = 2 * np.pi * 5e6, 1540.0, 1.5
    kf = omega / c
    sym = []
    for a0 in (5.5e-10, 5.5e-11):
        K = complex(oracle.wavenumber(omega, c, a0, y))
        tau = -2 * a0 * c ** (y - 1)
        eta = 2 * a0 * c ** y * math.tan(math.pi * y / 2)
        sym.append(abs(-K * K + kf * kf - 1j * tau * omega * K ** y + eta * K ** (y + 1)))
    first_order = abs(2 * kf * 5.5e-10 * omega ** y)
    assert sym[0] < 5e-2 * first_order
    assert 70 < sym[0] / sym[1] < 130


@pytest.mark.parametrize("y", [1.0, 1.5, 1.1])
def test_wavenumber_absorption_is_power_law(y):
    """Im k = alpha0 omega^y (Sec. 2.1.2, Eq. power_law_absorption)."""
    omega, a0 = 2 * np.pi * 3e6, 3e-10
    k = oracle.wavenumber(omega, np.array([1400.0, 1600.0]), a0, y)
    assert np.allclose(k.imag, a0 * omega ** y, rtol=1e-14)
    assert np.allclose(oracle.potential(np.array([1540.0]), omega, 1540.0, a0, y), 0.0, atol=1e-9)


def _plane_wave_wavenumber(mult, n):
    """Wavenumber of the outgoing wave of a point source on a long periodic
    line in the Case II medium (Sec. 2.3.2): the fixed point of the iteration
    of Eq. TBS_solution_absorbing-dispersive, psi^ = g~ (VV psi^ + S^), i.e.
    psi^ = g~ S^ / (1 - g~ VV), with alpha0 = mult x the paper's tissue value.
    Returns (K fitted from the phase and log-amplitude of psi between two
    distances, K of oracle.wavenumber)."""
    f, c, nu = 1.0e6, 1500.0, 1.5
    om = 2 * np.pi * f
    dx = c / f / 20
    k = om / c
    eps = 0.8 * k * k
    a0 = mult * 5.5e-10
    tau, eta = oracle.tau_eta(a0, nu, c)
    g = oracle.periodic_green_spectrum(k, eps, dx, (n,))
    VV = oracle.kspace_potential(dx, (n,), om, tau, eta, nu, eps)
    s = np.zeros(n, np.complex128)
    s[0] = 1.0 / dx
    psi = np.fft.ifft(g * np.fft.fft(s) / (1.0 - g * VV))
    K1 = complex(oracle.wavenumber(om, c, a0, nu))
    # fit over 0.5 .. 5 decay lengths of the first-order wave
    i1, i2 = int(0.5 / K1.imag / dx), int(5.0 / K1.imag / dx)
    x = np.arange(i1, i2) * dx
    A = np.vstack([x, np.ones_like(x)]).T
    kr = np.linalg.lstsq(A, np.unwrap(np.angle(psi[i1:i2])), rcond=None)[0][0]
    ki = -np.linalg.lstsq(A, np.log(np.abs(psi[i1:i2])), rcond=None)[0][0]
    return complex(kr, ki), K1, k


def test_kspace_potential_plane_wave_matches_wavenumber():
    """Pins the Case II k-space potential VV, tau and eta (Sec. 2.1.2 and
    Sec. 2.3.2, Eq. TBS_solution_absorbing-dispersive) through the physics of
    the converged iteration: the eps shift cancels at the fixed point, and the
    field of a point source is an outgoing wave whose phase advance (Re K,
    dispersion from eta) and decay (Im K, absorption from tau) equal the
    plane-wave wavenumber of ``oracle.wavenumber`` (pinned separately by the
    dispersion relation) up to its first-order error, which falls as alpha0^2.
    A flipped sign or a missing factor on the tau, eta or eps term changes K
    at first order."""
    Ka, K1a, k = _plane_wave_wavenumber(3, 16384)
    Kb, K1b, _ = _plane_wave_wavenumber(10, 8192)
    # measured absorption and dispersion agree with the first-order law ...
    assert abs(Ka.imag - K1a.imag) < 0.03 * K1a.imag
    assert abs((Ka.real - k) - (K1a.real - k)) < 0.03 * abs(K1a.real - k)
    # ... and the difference is the second-order remainder
    ratio = abs(Kb - K1b) / abs(Ka - K1a)
    assert 8.0 < ratio < 15.0, ratio      # (10/3)^2 = 11.1


def _eps_helmholtz_residual(ppw, eps_frac):
    """Converged (dense Lippmann-Schwinger) field of a smooth source in a
    smooth absorbing medium, with k0^2 = k(c0)^2 + i eps and V = k^2 - k0^2,
    checked against the Helmholtz equation with the physical k(x) only."""
    om, c0, a0, y = 2 * np.pi, 1.0, 0.02, 1.0
    dx = 1.0 / ppw
    n = int(round(2.0 / dx))
    ax = np.meshgrid(*[np.arange(n) * dx] * 2, indexing="ij")
    xc = (n // 2) * dx
    f = np.exp(-sum((a - xc) ** 2 for a in ax) / 0.3 ** 2).astype(np.complex128)
    cmap = c0 * (1 + 0.05 * np.exp(-sum((a - xc - 0.2) ** 2 for a in ax) / 0.4 ** 2))
    eps = eps_frac * (om / c0) ** 2
    k0 = oracle.background_k0(om, c0, a0, y, eps)
    V = oracle.potential(cmap, om, c0, a0, y, eps)
    p = oracle.dense_ls(oracle.dense_operator(k0, dx, (n, n)), V, f)
    k = oracle.wavenumber(om, cmap, a0, y)
    lap = np.zeros_like(p)
    for axis in range(2):
        r = lambda s: np.roll(p, s, axis=axis)  # noqa: E731
        lap += (-r(2) + 16 * r(1) - 30 * p + 16 * r(-1) - r(-2)) / (12 * dx * dx)
    res = lap + k * k * p + f
    inner = (slice(3, n - 3),) * 2
    return float(np.linalg.norm(res[inner]) / np.linalg.norm(f[inner]))


def test_potential_eps_shift():
    """The eps shift of Sec. 2.2 (k0^2 = k_f^2 + i eps) only moves a term
    between the two sides of the equation: in the background medium the
    potential is exactly -i eps (Sec. 2.3.1, Eq. TBS_equation_lossless), and the
    converged field with eps > 0 satisfies the Helmholtz equation of the
    physical medium (lap p + k(x)^2 p = -f) to O(dx^2), as with eps = 0.  A
    wrong sign of i eps in either background_k0 or potential leaves an O(1)
    residual that does not fall with dx."""
    om, c0, a0, y = 2 * np.pi * 3e6, 1540.0, 2e-10, 1.5
    kb = complex(oracle.wavenumber(om, c0, a0, y))
    for eps_frac in (0.3, 0.8):
        eps = eps_frac * abs(kb) ** 2
        v = oracle.potential(np.array([c0, c0]), om, c0, a0, y, eps)
        assert np.all(np.abs(v - (-1j * eps)) <= 1e-13 * abs(kb) ** 2)
        k0 = oracle.background_k0(om, c0, a0, y, eps)
        assert k0.imag > kb.imag
    r1, r2 = _eps_helmholtz_residual(12, 0.5), _eps_helmholtz_residual(24, 0.5)
    assert r2 < 6e-3 and 3.0 < r1 / r2 < 5.5, (r1, r2)


# --------------------------------------------------------------- harmonic ---

def test_harmonic_source_from_time_domain():
    """The second-harmonic source equals the 2 omega Fourier component of the
    time-domain nonlinear term, moved to the right-hand side in the paper's
    form lap psi + k^2 psi = -S (Sec. 2.1.4, Eq.
    acoustic_waveequn_time_dependent_nonlinear: + xi d^2(Psi^2)/dt^2 on the
    left).  Computed numerically from sampled Psi(t) = Re(p1 e^{-i omega t})."""
    omega, rho, BA = 2 * np.pi * 3e6, 1000.0, 7.0
    c = np.array([1500.0, 1540.0, 1600.0])
    p1 = np.array([1.0 + 2.0j, -0.3 + 0.1j, 2.0 - 1.0j]) * 1e5
    nt = 64
    t = np.arange(nt) * (2 * np.pi / omega) / nt
    Psi = np.real(p1[:, None] * np.exp(-1j * omega * t[None, :]))
    xi = (1 + BA / 2) / (rho * c ** 4)
    # xi * d^2(Psi^2)/dt^2 through its exact Fourier series in time
    spec = np.fft.fft(Psi ** 2, axis=1) / nt
    # complex amplitude X of the term Re(X e^{-2 i omega t}): component of e^{-2 i omega t}
    X2 = 2 * spec[:, nt - 2]                       # e^{-2i w t} is fft bin -2
    term = xi * (-(2 * omega) ** 2) * X2          # d^2/dt^2 -> -(2 omega)^2
    # lap psi2 + k2^2 psi2 + term = 0  =>  lap psi2 + k2^2 psi2 = -S2 with S2 = term
    S2 = oracle.harmonic_source(p1, c, omega, rho, BA)
    assert rel(S2, term) < 1e-12


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_harmonic_source_n_from_time_domain(n):
    """S_n equals the n omega Fourier component of xi d^2(Psi^2)/dt^2 for
    Psi(t) = sum_{k<n} Re(psi_k e^{-i k omega t}) (no difference-frequency term
    can reach n omega from harmonics below n), in the form lap psi + k^2 psi = -S."""
    omega, rho, BA = 2 * np.pi * 1e6, 1000.0, 5.0
    rng = np.random.default_rng(70 + n)
    c = np.array([1480.0, 1500.0, 1575.0, 1620.0])
    fields = [(rng.standard_normal(4) + 1j * rng.standard_normal(4)) * 10 ** (5 - k) for k in range(n - 1)]
    nt = 64
    t = np.arange(nt) * (2 * np.pi / omega) / nt
    Psi = sum(np.real(f[:, None] * np.exp(-1j * (k + 1) * omega * t[None, :])) for k, f in enumerate(fields))
    xi = (1 + BA / 2) / (rho * c ** 4)
    spec = np.fft.fft(Psi ** 2, axis=1) / nt
    Xn = 2 * spec[:, nt - n]                      # amplitude of e^{-i n omega t}
    term = xi * (-(n * omega) ** 2) * Xn
    S = oracle.harmonic_source_n(fields, n, c, omega, rho, BA)
    assert rel(S, term) < 1e-12
    if n == 2:
        assert rel(S, oracle.harmonic_source(fields[0], c, omega, rho, BA)) < 1e-15


# ---------------------------------------------------- periodic (paper) mode --

def test_periodic_green_kernel_is_the_lossy_hankel_function():
    """ifft(g~)/dx^2 on a large periodic grid approaches the free-space 2D
    Green's function (i/4) H0(kappa r), kappa^2 = k^2 + i eps (the eps-lossy
    equation of Sec. 2.2), with second-order convergence in dx: pins the sign
    and the normalisation of g~ and the p-grid."""
    import scipy.special
    lam = 1.0
    k = 2 * np.pi / lam
    eps = 0.8 * k * k
    kap = np.sqrt(k * k + 1j * eps)
    errs = []
    for ppw in (10, 20, 40):
        dx = lam / ppw
        n = 32 * ppw // 10 * 8
        ker = np.fft.ifft2(oracle.periodic_green_spectrum(k, eps, dx, (n, n))) / dx ** 2
        cells = [int(round(r * ppw)) for r in (0.4, 0.8)]   # r = 0.4 and 0.8 wavelengths
        e = max(abs(ker[0, m] - 0.25j * scipy.special.hankel1(0, kap * m * dx)) /
                abs(0.25j * scipy.special.hankel1(0, kap * m * dx)) for m in cells)
        errs.append(e)
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1], errs
    assert errs[2] < 3e-3, errs


def _periodic_case(n=24, seed=3):
    dx = 1.0
    k = 2 * np.pi / 6.3       # between grid wavenumbers
    eps = 0.8 * k * k
    s = workloads.random_field((n, n), seed)
    return dx, k, eps, s


@pytest.mark.parametrize("L", [1, 2, 7])
def test_paper_iteration_constant_potential_closed_form(L):
    """Case I with a constant V and no absorbing layer: the iteration is
    diagonal in k-space, psi^L = ifft(g~ S (1 - (g~ V)^(L+1)) / (1 - g~ V))
    (the geometric partial sum of the series, Sec. 2.2 Eq. TBS_2)."""
    dx, k, eps, s = _periodic_case()
    g = oracle.periodic_green_spectrum(k, eps, dx, s.shape)
    V = -1j * eps + 0.1 * k * k
    psi, it, errs = oracle.paper_iterate(g, s, V=np.full(s.shape, V), tol=0.0, max_iter=L)
    q = g * V
    ref = np.fft.ifft2(g * np.fft.fft2(s) * (1 - q ** (L + 1)) / (1 - q))
    assert it == L and len(errs) == L
    assert rel(psi, ref) < 1e-12


def test_paper_iteration_kspace_potential_closed_form():
    """Case II: psi^L = ifft(g~ S (1 - (g~ VV)^(L+1)) / (1 - g~ VV)) with the
    k-space potential of the absorbing-dispersive medium."""
    dx, k, eps, s = _periodic_case(seed=5)
    g = oracle.periodic_green_spectrum(k, eps, dx, s.shape)
    tau, eta = oracle.tau_eta(5.5e-10, 1.5, 1500.0)
    # a medium 1e3 times more lossy than tissue keeps the test sensitive to VV
    VV = oracle.kspace_potential(dx, s.shape, 2 * np.pi * 1e6, 1e3 * tau, 1e3 * eta, 1.5, eps)
    psi, it, _ = oracle.paper_iterate(g, s, VV=VV, tol=0.0, max_iter=5)
    q = g * VV
    ref = np.fft.ifft2(g * np.fft.fft2(s) * (1 - q ** 6) / (1 - q))
    assert rel(psi, ref) < 1e-12


def test_paper_iteration_converges_to_lossless_periodic_solution():
    """With V = -i eps the eps-shift cancels at convergence: psi solves the
    lossless periodic Helmholtz equation, psi^ = S^ / (|p|^2 - k^2)
    (Sec. 2.3.1 Eq. TBS_solution_lossless)."""
    dx, k, eps, s = _periodic_case(n=16, seed=7)
    g = oracle.periodic_green_spectrum(k, eps, dx, s.shape)
    # the homogeneous lossless medium's potential with the eps shift
    omega = k * 1500.0
    V = oracle.potential(np.full(s.shape, 1500.0), omega, 1500.0, 0.0, 1.0, eps)
    psi, it, errs = oracle.paper_iterate(g, s, V=V, tol=1e-13, max_iter=20000)
    axes = [2 * np.pi * np.fft.fftfreq(n, d=dx) for n in s.shape]
    P2 = axes[0][:, None] ** 2 + axes[1][None, :] ** 2
    ref = np.fft.ifft2(np.fft.fft2(s) / (P2 - k * k))
    assert it < 20000 and rel(psi, ref) < 1e-9


def test_abl_profile_shape():
    """Eq. ABL_profile with the paper's zeta = 21.48 Np/cm and mu = 450 dx at
    dx = 20 um: 1/2 at mu/2 from the edge, rising through the layer, 1
    beyond it, and the 2D mask is the product of the axis profiles."""
    dx, zeta, mu = 20e-6, 21.48, 450
    n = 1200
    f = oracle.abl_profile(n, dx, zeta, mu)
    assert f[225] == pytest.approx(0.5, abs=1e-15)
    assert f[n - 1 - 225] == pytest.approx(0.5, abs=1e-15)
    assert np.all(np.diff(f[:450]) > 0)
    assert np.all(f[450:n - 450] == 1.0)
    assert f[0] == pytest.approx(1.0 / (1.0 + math.exp(zeta * 0.45)), rel=1e-12)
    m = oracle.abl_mask((n, 1000), dx, zeta, mu)
    assert m[225, 500] == pytest.approx(0.5) and m[600, 450] == 1.0
    assert m[225, 225] == pytest.approx(0.25)


def _strong_scatterer(n=16, seed=9, contrast=0.6):
    dx = 1.0
    k0 = 2 * np.pi / 6.0
    blob = np.exp(-(((np.arange(n) - n / 2)[:, None] ** 2 + (np.arange(n) - n / 2)[None, :] ** 2) / 8.0))
    k = k0 * (1 + contrast * blob) + 0.02j * k0
    k2 = k * k
    s = np.zeros((n, n), np.complex128)
    s[3, 5] = 1.0
    s[n - 4, 2] = 0.5j
    return dx, k0, k2, s


def test_periodic_dense_solve_is_the_helmholtz_solution():
    """The dense periodic solve satisfies the equation through an independent
    route (the spectral Laplacian applied by FFTs to the solution)."""
    dx, k0, k2, s = _strong_scatterer()
    psi = oracle.periodic_helmholtz_dense(k2, dx, s)
    px = 2 * np.pi * np.fft.fftfreq(s.shape[1], d=dx)
    py = 2 * np.pi * np.fft.fftfreq(s.shape[0], d=dx)
    lap_psi = -np.fft.ifft2(np.fft.fft2(psi) * (py[:, None] ** 2 + px[None, :] ** 2))
    assert rel(-lap_psi - k2 * psi, s) < 1e-12


def test_cbs_converges_where_tbs_diverges():
    """Strong scatterer (60 % speed contrast): the paper's series diverges
    (spectral radius of G V above 1), the convergent Born series with
    eps = max |k^2 - k0^2| reaches the dense periodic Helmholtz solution."""
    dx, k0, k2, s = _strong_scatterer()
    dV = k2 - k0 * k0
    eps = 1.01 * np.max(np.abs(dV))
    g = oracle.periodic_green_spectrum(k0, eps, dx, s.shape)
    V = dV - 1j * eps
    exact = oracle.periodic_helmholtz_dense(k2, dx, s)
    # TBS (paper iteration) on the same potential: the change grows
    _, _, e_tbs = oracle.paper_iterate(g, s, V=V, tol=0.0, max_iter=60)
    assert e_tbs[-1] > e_tbs[20]
    psi, it, errs = oracle.cbs_iterate(g, s, V, eps, tol=1e-12, max_iter=20000)
    assert it < 20000
    assert rel(psi, exact) < 1e-9


def test_cbs_weak_scatterer_agrees_with_tbs_limit():
    """Weak medium: CBS and the paper's iteration converge to the same field."""
    dx, k0, k2, s = _strong_scatterer(contrast=0.02)
    dV = k2 - k0 * k0
    eps = 0.8 * k0 * k0
    g = oracle.periodic_green_spectrum(k0, eps, dx, s.shape)
    V = dV - 1j * eps
    a, _, _ = oracle.paper_iterate(g, s, V=V, tol=1e-13, max_iter=20000)
    b, _, _ = oracle.cbs_iterate(g, s, V, eps, tol=1e-13, max_iter=20000)
    assert rel(a, b) < 1e-9
    assert rel(b, oracle.periodic_helmholtz_dense(k2, dx, s)) < 1e-9


# ------------------------------------------------------- density contrast --

def test_density_operator_discrete_symbol():
    """On a constant gamma, D acts on sin(a x) sin(b y) at interior cells as
    gamma times the discrete Laplacian symbol -(4/dx^2)(sin^2(a dx/2) +
    sin^2(b dx/2)) (a closed form), which tends to -gamma (a^2 + b^2)."""
    n, dx, gam = 40, 0.3, 0.7
    a, b = 0.9, 1.7
    y, x = np.mgrid[0:n, 0:n] * dx
    u = np.sin(a * x) * np.sin(b * y)
    D = oracle.density_operator(np.full((n, n), gam), dx, u)
    sym = -(4.0 / dx ** 2) * (np.sin(a * dx / 2) ** 2 + np.sin(b * dx / 2) ** 2)
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose(D[inner], gam * sym * u[inner], rtol=0, atol=1e-12)


def test_density_operator_second_order_variable_coefficient():
    """Smooth gamma and u: D(u) converges to div(gamma grad u) (analytic) at
    second order in dx."""
    errs = []
    for n in (32, 64, 128):
        dx = 4.0 / n
        y, x = np.mgrid[0:n, 0:n] * dx + dx / 2
        gam = 0.3 * np.exp(-((x - 2) ** 2 + (y - 2) ** 2))
        u = np.exp(1j * (1.3 * x + 0.4 * y)) * np.exp(-((x - 2) ** 2 + (y - 2) ** 2) / 2)
        # analytic div(gamma grad u) with complex u (symbolic derivatives written out)
        gx = gam * (-2 * (x - 2)); gy = gam * (-2 * (y - 2))
        ux = u * (1.3j - (x - 2)); uy = u * (0.4j - (y - 2))
        uxx = ux * (1.3j - (x - 2)) - u; uyy = uy * (0.4j - (y - 2)) - u
        exact = gx * ux + gy * uy + gam * (uxx + uyy)
        D = oracle.density_operator(gam, dx, u)
        inner = (slice(n // 8, -n // 8), slice(n // 8, -n // 8))
        errs.append(np.max(np.abs(D[inner] - exact[inner])) / np.max(np.abs(exact[inner])))
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1], errs


def test_density_operator_symmetric_negative():
    """Summation by parts: the matrix of D is real symmetric and negative
    semidefinite for gamma >= 0 (the term is self-adjoint)."""
    rng = np.random.default_rng(4)
    gam = rng.uniform(0, 0.4, (7, 9))
    Dm = oracle.density_matrix(gam, 0.5)
    assert np.allclose(Dm, Dm.T, atol=1e-14)
    assert np.max(np.linalg.eigvalsh(Dm)) < 1e-12


def test_density_operator_discrete_symbol_3d():
    """3D: on a constant gamma, D acts on sin(a x) sin(b y) sin(c z) at interior
    cells as gamma times -(4/dx^2)(sin^2(a dx/2) + sin^2(b dx/2) + sin^2(c dx/2))."""
    n, dx, gam = 14, 0.4, 0.3
    a, b, c = 0.8, 1.3, 2.1
    z, y, x = np.mgrid[0:n, 0:n, 0:n] * dx
    u = np.sin(a * x) * np.sin(b * y) * np.sin(c * z)
    D = oracle.density_operator(np.full((n, n, n), gam), dx, u)
    sym = -(4.0 / dx ** 2) * (np.sin(a * dx / 2) ** 2 + np.sin(b * dx / 2) ** 2 + np.sin(c * dx / 2) ** 2)
    inner = (slice(1, -1),) * 3
    assert np.allclose(D[inner], gam * sym * u[inner], rtol=0, atol=1e-12)
    # each axis enters: a function of z alone sees only the z part of the symbol
    uz = np.broadcast_to(np.sin(c * z[:, :1, :1]), (n, n, n)).copy()
    Dz = oracle.density_operator(np.full((n, n, n), gam), dx, uz)
    symz = -(4.0 / dx ** 2) * np.sin(c * dx / 2) ** 2
    assert np.allclose(Dz[inner], gam * symz * uz[inner], rtol=0, atol=1e-12)


def test_density_operator_second_order_3d():
    """3D, smooth gamma and u: D(u) converges to the analytic div(gamma grad u)
    at second order in dx."""
    errs = []
    for n in (16, 32, 64):
        dx = 4.0 / n
        z, y, x = np.mgrid[0:n, 0:n, 0:n] * dx + dx / 2
        r2 = (x - 2) ** 2 + (y - 2) ** 2 + (z - 2) ** 2
        gam = 0.3 * np.exp(-r2)
        u = np.exp(1j * (1.1 * x + 0.4 * y - 0.7 * z)) * np.exp(-r2 / 2)
        gx, gy, gz = gam * (-2 * (x - 2)), gam * (-2 * (y - 2)), gam * (-2 * (z - 2))
        ux, uy, uz = u * (1.1j - (x - 2)), u * (0.4j - (y - 2)), u * (-0.7j - (z - 2))
        uxx = ux * (1.1j - (x - 2)) - u
        uyy = uy * (0.4j - (y - 2)) - u
        uzz = uz * (-0.7j - (z - 2)) - u
        exact = gx * ux + gy * uy + gz * uz + gam * (uxx + uyy + uzz)
        D = oracle.density_operator(gam, dx, u)
        inner = (slice(n // 8, -n // 8),) * 3
        errs.append(np.max(np.abs(D[inner] - exact[inner])) / np.max(np.abs(exact[inner])))
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1], errs


def test_density_operator_symmetric_negative_3d():
    rng = np.random.default_rng(5)
    gam = rng.uniform(0, 0.4, (4, 5, 6))
    Dm = oracle.density_matrix(gam, 0.5)
    assert np.allclose(Dm, Dm.T, atol=1e-14)
    assert np.max(np.linalg.eigvalsh(Dm)) < 1e-12


def test_density_series_converges_to_dense_solve_3d():
    grid = (5, 6, 7)
    dx = 1.0
    k0 = 2 * np.pi / 6 * (1 + 0.03j)
    V = 0.05 * (k0 * k0).real * workloads.random_field(grid, 23).real
    zz, yy, xx = np.mgrid[0:grid[0], 0:grid[1], 0:grid[2]]
    gam = 0.06 * np.exp(-((zz - 2) ** 2 + (yy - 3) ** 2 + (xx - 3) ** 2) / 4.0)
    s = workloads.random_field(grid, 24)
    A = oracle.dense_operator(k0, dx, grid)
    Dm = oracle.density_matrix(gam, dx)
    K = A @ (np.diag(V.ravel()) - Dm)
    exact = np.linalg.solve(np.eye(K.shape[0]) - K, A @ s.ravel()).reshape(grid)
    assert np.max(np.abs(np.linalg.eigvals(K))) < 0.6
    p, res = oracle.solve_density(k0, dx, s, V, gam, 60)
    assert rel(p, exact) < 1e-9
    assert res[-1] < 1e-9


def test_density_series_converges_to_dense_solve():
    """With a weak density and speed contrast the series converges to the
    dense solution of p = G (V - D) p + G s."""
    grid = (10, 11)
    dx = 1.0
    k0 = 2 * np.pi / 6 * (1 + 0.03j)
    V = 0.05 * (k0 * k0).real * workloads.random_field(grid, 21).real
    yy, xx = np.mgrid[0:grid[0], 0:grid[1]]
    gam = 0.06 * np.exp(-((yy - 5) ** 2 + (xx - 5) ** 2) / 6.0)
    s = workloads.random_field(grid, 22)
    A = oracle.dense_operator(k0, dx, grid)
    Dm = oracle.density_matrix(gam, dx)
    K = A @ (np.diag(V.ravel()) - Dm)
    exact = np.linalg.solve(np.eye(K.shape[0]) - K, A @ s.ravel()).reshape(grid)
    rho = np.max(np.abs(np.linalg.eigvals(K)))
    assert rho < 0.6
    p, res = oracle.solve_density(k0, dx, s, V, gam, 60)
    assert rel(p, exact) < 1e-9
    assert res[-1] < 1e-9


# ---------------------------------------------------------------- adjoint ---

def test_adjoint_green_operator_dot_product():
    grid = (9, 13)
    G = oracle.GreenOperator(1.3 + 0.07j, 0.6, grid)
    f = workloads.random_field(grid, 1)
    h = workloads.random_field(grid, 2)
    lhs = np.vdot(h, G(f))
    rhs = np.vdot(G(h, adjoint=True), f)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_adjoint_series_dot_product():
    """d Re<q, p_L> along a direction dV equals Re sum dV g_V (directional
    derivative by complex-step-free central difference in FP64)."""
    grid = (10, 9)
    k0 = 2 * np.pi / 6 * (1 + 0.02j)
    G = oracle.GreenOperator(k0, 1.0, grid)
    V = 0.05 * workloads.random_field(grid, 3)
    s = workloads.random_field(grid, 4)
    q = workloads.random_field(grid, 5)
    dV = workloads.random_field(grid, 6)
    L = 6
    g = oracle.adjoint_series_gradient(G, s, V, L, q)
    h = 1e-6
    fp = np.vdot(q, oracle.born_series(G, s, V + h * dV, L)[0]).real
    fm = np.vdot(q, oracle.born_series(G, s, V - h * dV, L)[0]).real
    fd = (fp - fm) / (2 * h)
    assert abs(fd - np.sum(dV * g).real) < 1e-7 * abs(fd)
    assert np.all(oracle.adjoint_series_gradient(G, s, V, 1, q) == 0)


def test_misfit_gradient_matches_finite_differences():
    """dJ/dc from the adjoint series equals central FD (h = 1e-6 c0) at sampled
    pixels, in FP64, on a small grid."""
    prob = workloads.adjoint2d(n=24, nfreq=2, nsrc=2, nrec=8, nterms=5)
    rec = prob.receivers.copy()
    p_obs = []
    for f in prob.freqs:
        om = 2 * np.pi * f
        k0 = oracle.background_k0(om, workloads.C0, prob.alpha0, prob.y)
        V = oracle.potential(prob.c_true, om, workloads.C0, prob.alpha0, prob.y)
        p, _ = oracle.solve(k0, prob.dx, prob.sources, V, prob.nterms)
        p_obs.append(p[(slice(None),) + tuple(rec.T)])
    J, grad = oracle.misfit_gradient(prob.c_model, prob.freqs, prob.dx, workloads.C0, prob.alpha0,
                                     prob.y, prob.sources, rec, p_obs, prob.nterms)
    assert J > 0
    h = 1e-6 * workloads.C0
    for (iy, ix) in [(12, 12), (8, 15), (16, 5)]:
        cp = prob.c_model.copy(); cp[iy, ix] += h
        cm = prob.c_model.copy(); cm[iy, ix] -= h
        Jp, _ = oracle.misfit_gradient(cp, prob.freqs, prob.dx, workloads.C0, prob.alpha0, prob.y,
                                       prob.sources, rec, p_obs, prob.nterms)
        Jm, _ = oracle.misfit_gradient(cm, prob.freqs, prob.dx, workloads.C0, prob.alpha0, prob.y,
                                       prob.sources, rec, p_obs, prob.nterms)
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - grad[iy, ix]) < 1e-6 * np.max(np.abs(grad)), (iy, ix, fd, grad[iy, ix])
