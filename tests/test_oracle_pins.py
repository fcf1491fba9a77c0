"""Pins of the FP64 oracle against closed forms, identities and invariances.

Each test fixes a property that the paper's method (Section 2.2: the
discretised Rybicki-Lightman / Lienard-Wiechert spectral integral) must have,
computed by means independent of the oracle's own arithmetic:

* straight motion radiates nothing (the integrand vanishes identically);
* a driven oscillator seen from any direction in the plane of drift and
  observer has kappa constant and a geometric-series closed form for the
  discrete sum (Doppler-shifted line at w0 / (1 - beta_d cos theta));
* for uniformly spaced retarded times the discrete sum obeys an exact
  Parseval identity;
* uniform circular motion at integer harmonics equals the Bessel closed form
  m^2 beta^2 J'_m(m beta)^2 (Jacobi-Anger) in the orbit plane and Schott's
  angular distribution out of it, with its in-plane K_{2/3} asymptotics and,
  integrated over solid angle, the synchrotron x int K_{5/3} form;
* the solid-angle and frequency integral of a smooth orbit equals the
  Lienard (relativistic Larmor) energy;
* rotations, time shifts, translations, charge sign, weights, permutations,
  splitting the trajectory in time and sharding the particles.
"""
import numpy as np
import pytest
import scipy.special as sp

import oracle
from workloads import Batch, orbits
from workloads.configs import log_grid, synchrotron_setup

FOUR_PI2 = 4 * np.pi**2


def spectrum_of(batch, dirs, omega):
    return oracle.spectrum(batch, dirs, omega, n_species=1)[0]


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("beta", [[0.9, 0.0, 0.0], [0.3, -0.5, 0.7], [0.0, 0.0, -0.999]])
def test_straight_motion_radiates_nothing(beta):
    b = orbits.straight(beta, [1.0, -2.0, 0.5], 300, 0.01)
    dirs = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [-1, 0.2, 0.3]], dtype=float)
    S = spectrum_of(b, dirs, log_grid(0.1, 1e4, 40))
    assert np.all(S == 0.0)


# ---------------------------------------------------------------- P2
def _oscillator_closed_form(beta_d, beta1, w0, n, dt, t0, theta, omega):
    """A_x of the driven oscillator seen along n = (0, sin th, cos th).

    kappa = 1 - beta_d cos th is constant, the retarded time is kappa t and the
    integrand is x-directed with magnitude beta1 w0 sin(w0 t) / kappa, so the
    sum is two geometric series.
    """
    kap = 1 - beta_d * np.cos(theta)
    Om = omega * kap

    def G(x):
        x = np.asarray(x, dtype=np.float64)
        num = 1 - np.exp(1j * x * n * dt)
        den = 1 - np.exp(1j * x * dt)
        out = np.where(np.abs(den) > 1e-300, num / np.where(den == 0, 1, den), n)
        return np.exp(1j * x * t0) * out

    return (beta1 * w0 * dt / kap) / 2j * (G(Om + w0) - G(Om - w0)), kap


@pytest.mark.parametrize("theta_deg", [0.0, 30.0, 90.0, 150.0, 180.0])
def test_driven_oscillator_geometric_series(theta_deg):
    beta_d, beta1, w0, n, dt, t0 = 0.6, 0.3, 2.0, 1000, 0.0137, 0.37
    th = np.radians(theta_deg)
    b = orbits.driven_oscillator(beta_d, beta1, w0, n, dt, t0=t0)
    om = np.linspace(0.05, 25.0, 97)
    A = oracle.amplitude(b, 0, [0.0, np.sin(th), np.cos(th)], om)
    Ax, kap = _oscillator_closed_form(beta_d, beta1, w0, n, dt, t0, th, om)
    scale = np.max(np.abs(Ax))
    assert np.max(np.abs(A[:, 0] - Ax)) <= 1e-12 * scale
    assert np.max(np.abs(A[:, 1:])) <= 1e-12 * scale


def test_doppler_shifted_line_position_and_height():
    """Whole periods: the line sits at w0/kappa and its centre value is beta1^2 N_per^2 / (4 kappa^2).

    At the line centre the discrete sum of the counter-rotating part vanishes
    exactly (a full set of roots of unity), so the centre value is exact.
    """
    beta_d, beta1, w0 = 0.5, 0.05, 1.0
    per, spp = 20, 64  # periods, samples per period
    n, dt = per * spp, 2 * np.pi / w0 / spp
    b = orbits.driven_oscillator(beta_d, beta1, w0, n, dt)
    kap = 1 - beta_d
    om = np.linspace(0.8, 1.2, 4001) * w0 / kap
    S = spectrum_of(b, [[0, 0, 1]], om)[0]
    assert abs(om[np.argmax(S)] * kap / w0 - 1) < 1e-3  # main lobe half-width is 1/per = 5e-2
    centre = spectrum_of(b, [[0, 0, 1]], [w0 / kap])[0, 0]
    assert abs(centre / (beta1**2 * per**2 / (4 * kap**2)) - 1) < 1e-12


# ---------------------------------------------------------------- P3
def test_discrete_parseval_uniform_retarded_time():
    beta_d, beta1, w0, n, dt = 0.7, 0.2, 3.0, 257, 0.021
    b = orbits.driven_oscillator(beta_d, beta1, w0, n, dt, t0=-1.3)
    kap = 1 - beta_d
    M = 2 * n + 3
    om = np.linspace(0.0, np.pi / (kap * dt), M + 1)
    S = spectrum_of(b, [[0, 0, 1]], om)[0]
    lhs = np.trapezoid(S, om)
    t = b.t0[0] + np.arange(n) * dt
    g2 = (beta1 * w0 * np.sin(w0 * t) / kap) ** 2
    rhs = dt * g2.sum() / (4 * np.pi * kap)
    assert abs(lhs / rhs - 1) < 1e-12


# ---------------------------------------------------------------- P5
def test_synchrotron_harmonics_config_step():
    """Config grid (dt = T/2000): exact Bessel values at harmonics well below the sampling rate."""
    cfg = synchrotron_setup()
    b = orbits.circular(cfg["gamma"], 1.0, cfg["n"], cfg["dt"])
    beta = np.sqrt(1 - 1 / cfg["gamma"] ** 2)
    m = np.array([1, 2, 3, 7, 10, 31, 100, 250, 500], dtype=float)
    S = spectrum_of(b, [[1, 0, 0]], m)[0]
    exact = m**2 * beta**2 * sp.jvp(m, m * beta) ** 2
    np.testing.assert_allclose(S, exact, rtol=1e-11)


@pytest.mark.slow
def test_synchrotron_harmonics_fine_step():
    g = 10.0
    n = 100_000
    b = orbits.circular(g, 1.0, n, 2 * np.pi / n)
    beta = np.sqrt(1 - 1 / g**2)
    m = np.array([1000, 1508, 3000, 6000, 15000], dtype=float)
    S = spectrum_of(b, [[1, 0, 0]], m)[0]
    exact = m**2 * beta**2 * sp.jvp(m, m * beta) ** 2
    np.testing.assert_allclose(S, exact, rtol=1e-9)


def test_synchrotron_harmonics_other_gamma_and_phase():
    """Same closed form for gamma = 3, another start phase and a different omega0."""
    g, w0 = 3.0, 2.5
    n = 4000
    b = orbits.circular(g, w0, n, 2 * np.pi / w0 / n, phase0=1.234, charge=+1.0, weight=2.0)
    beta = np.sqrt(1 - 1 / g**2)
    m = np.array([1, 2, 5, 9, 20, 40], dtype=float)
    S = spectrum_of(b, [[0, -1, 0]], m * w0)[0]
    exact = 2.0 * m**2 * beta**2 * sp.jvp(m, m * beta) ** 2
    np.testing.assert_allclose(S, exact, rtol=1e-11)


def test_synchrotron_in_plane_k23_asymptotics():
    """Between harmonics the time-averaged in-plane spectrum approaches the K_{2/3} form.

    Averaging S over one harmonic spacing at omega ~ m omega0 gives the per-period
    line strength; the continuum form (Jackson 14.79 at theta = 0) predicts
    (1/3 pi^2) (omega rho)^2 gamma^-4 K_{2/3}^2(omega rho / 3 gamma^3) per unit omega per period,
    i.e. the line value at omega = m omega0 within the O(1/gamma^2) corrections of the asymptotics.
    """
    cfg = synchrotron_setup()
    g = cfg["gamma"]
    beta = np.sqrt(1 - 1 / g**2)
    b = orbits.circular(g, 1.0, cfg["n"], cfg["dt"])
    wc = cfg["omega_c"]
    m = np.round(np.array([0.01, 0.03, 0.1, 0.3]) * wc)
    S = spectrum_of(b, [[1, 0, 0]], m)[0]
    rho = beta
    xi = m * rho / (3 * g**3)
    asym = (m * rho) ** 2 / (3 * np.pi**2) / g**4 * sp.kv(2 / 3, xi) ** 2
    ratio = S / asym
    assert np.all(np.abs(ratio - 1) < 0.08), ratio


def _circular_fine(gamma=10.0, n=100_000):
    """One period of the config-1 orbit on a fine step (T / 1e5): the discrete sum equals
    the continuous integral to ~1e-9 at the harmonics used below."""
    return orbits.circular(gamma, 1.0, n, 2 * np.pi / n)


def _elevated(psi):
    """Unit directions at elevation psi above the orbit plane (x-y), azimuth 0."""
    psi = np.atleast_1d(psi)
    return np.stack([np.cos(psi), np.zeros_like(psi), np.sin(psi)], 1)


def test_synchrotron_harmonics_out_of_plane_schott():
    """Every elevation, not only the orbit plane: at harmonic m of one period the spectrum is
    m^2 [cot^2(th) J_m(m beta sin th)^2 + beta^2 J'_m(m beta sin th)^2] (Schott's angular
    distribution of the harmonics; th the polar angle from the orbit normal), exact."""
    g = 10.0
    b = _circular_fine(g)
    beta = np.sqrt(1 - 1 / g**2)
    psi = np.array([-0.9, -0.3, -0.05, 0.0, 0.02, 0.1, 0.45, 1.2])
    th = np.pi / 2 - psi
    m = np.array([1.0, 3.0, 10.0, 40.0, 150.0, 600.0])
    S = spectrum_of(b, _elevated(psi), m)
    for i, t in enumerate(th):
        x = m * beta * np.sin(t)
        exact = m**2 * ((np.cos(t) / np.sin(t)) ** 2 * sp.jv(m, x) ** 2 + beta**2 * sp.jvp(m, x) ** 2)
        big = exact >= 1e-12 * exact.max()
        np.testing.assert_allclose(S[i][big], exact[big], rtol=1e-8)


def _synchrotron_F(x):
    """F(x) = x int_x^inf K_{5/3}(s) ds, by adaptive quadrature of scipy's K_nu."""
    from scipy.integrate import quad

    return x * quad(lambda s: sp.kv(5.0 / 3.0, s), x, np.inf, limit=200)[0]


def test_synchrotron_function_integral():
    """int_0^inf F(x) dx = 8 pi / (9 sqrt 3), which fixes the total of the x int K_{5/3} form
    (per revolution (8 pi / 9) gamma omega_c, the Larmor energy up to O(1/gamma^2))."""
    from scipy.integrate import quad

    total = quad(_synchrotron_F, 0.0, 1.0, limit=200)[0] + quad(_synchrotron_F, 1.0, 60.0, limit=200)[0]
    assert abs(total / (8 * np.pi / (9 * np.sqrt(3))) - 1) < 1e-7


def _angle_integrated(gamma, n, ratio_x):
    """2 pi int cos(psi) S(psi) dpsi over |psi| <= 8 / gamma (96-node Gauss-Legendre) at the
    harmonics nearest ratio_x * w_c, and sqrt(3) gamma F(w / w_c) there."""
    b = orbits.circular(gamma, 1.0, n, 2 * np.pi / n)
    beta = np.sqrt(1 - 1 / gamma**2)
    wc = 1.5 * gamma**3 / beta
    xg, wg = np.polynomial.legendre.leggauss(96)
    half = 8.0 / gamma
    psi = half * xg
    m = np.round(np.asarray(ratio_x) * wc)
    S = spectrum_of(b, _elevated(psi), m)
    dW = 2 * np.pi * half * np.sum((wg * np.cos(psi))[:, None] * S, axis=0)
    form = np.array([np.sqrt(3) * gamma * _synchrotron_F(w / wc) for w in m])
    return dW, form


def test_synchrotron_angle_integrated_x_int_k53():
    """Solid-angle integral of one period's spectrum against the synchrotron form.

    The harmonics of a whole period do not depend on azimuth, so the solid-angle integral is
    2 pi int cos(psi) S(psi) dpsi over the elevation psi.  At harmonics w = m w0 near
    0.1 ... 2 w_c it must equal sqrt(3) gamma F(w / w_c), w_c = (3/2) gamma^3 w0 / beta
    (Rybicki-Lightman; Jackson 14.91), up to the O(1/gamma^2) corrections of that
    ultra-relativistic form: at most 2.5 % at gamma = 10 (the config-1 orbit) and 0.4 % at
    gamma = 30, and the deviation must shrink by at least 5x between the two (1/gamma^2
    predicts 9x).  A wrong power of kappa, prefactor, cross product or phase in the oracle
    moves these ratios by far more."""
    x = np.array([0.1, 0.3, 1.0, 2.0])
    dw10, f10 = _angle_integrated(10.0, 100_000, x)
    dw30, f30 = _angle_integrated(30.0, 400_000, x)
    r10, r30 = dw10 / f10, dw30 / f30
    assert np.all(np.abs(r10 - 1) < 0.025), r10
    assert np.all(np.abs(r30 - 1) < 0.004), r30
    assert np.all(np.abs(r10 - 1) > 5 * np.abs(r30 - 1)), (r10, r30)


# ---------------------------------------------------------------- P4 / P6
def _gauss_orbit(beta_d=0.5, amp=0.05, w0=1.0, sigma=6.0, n=1500, dt=0.06):
    return orbits.gaussian_oscillator(amp, w0, sigma, beta_d, n, dt)


def test_continuous_parseval_oblique_direction():
    """int_0^inf S dw = (1/4pi) int |n x ((n - beta) x betadot)|^2 / kappa^5 dt for a band-limited orbit."""
    b = _gauss_orbit()
    for th in (0.0, 0.7, 1.9):
        nvec = np.array([np.sin(th) * np.cos(0.3), np.sin(th) * np.sin(0.3), np.cos(th)])
        om = np.linspace(0.0, 12.0, 2401)
        S = spectrum_of(b, [nvec], om)[0]
        lhs = np.trapezoid(S, om)
        # right side on a 4x finer analytic grid
        fb = orbits.gaussian_oscillator(0.05, 1.0, 6.0, 0.5, 4 * 1500, 0.015)
        beta = np.stack([fb.bx, fb.by, fb.bz], 1)
        bdot = np.stack([fb.ax, fb.ay, fb.az], 1)
        kap = 1 - beta @ nvec
        v = np.cross(nvec, np.cross(nvec[None, :] - beta, bdot))
        rhs = np.trapezoid((v**2).sum(1) / kap**5, dx=0.015) / (4 * np.pi)
        assert abs(lhs / rhs - 1) < 1e-6, (th, lhs, rhs)


@pytest.mark.slow
def test_lienard_total_energy_over_sphere():
    """Solid-angle and frequency integral equals the Lienard energy (2/3) int gamma^6 (bdot^2 - |b x bdot|^2) dt."""
    b = _gauss_orbit(beta_d=0.5, amp=0.05, n=1000, dt=0.09)
    xg, wg = np.polynomial.legendre.leggauss(40)
    nphi = 16
    phis = 2 * np.pi * (np.arange(nphi) + 0.5) / nphi
    dirs, wts = [], []
    for c, w in zip(xg, wg):
        s = np.sqrt(1 - c * c)
        for ph in phis:
            dirs.append([s * np.cos(ph), s * np.sin(ph), c])
            wts.append(w * 2 * np.pi / nphi)
    dirs, wts = np.array(dirs), np.array(wts)
    om = np.linspace(0.0, 10.0, 801)
    S = spectrum_of(b, dirs, om)
    total = np.sum(wts * np.trapezoid(S, om, axis=1))
    fb = orbits.gaussian_oscillator(0.05, 1.0, 6.0, 0.5, 8000, 0.01125)
    beta = np.stack([fb.bx, fb.by, fb.bz], 1)
    bdot = np.stack([fb.ax, fb.ay, fb.az], 1)
    gam2 = 1 / (1 - (beta**2).sum(1))
    p = (2 / 3) * gam2**3 * ((bdot**2).sum(1) - (np.cross(beta, bdot) ** 2).sum(1))
    energy = np.trapezoid(p, dx=0.01125)
    assert abs(total / energy - 1) < 1e-5, (total, energy)


# ---------------------------------------------------------------- P7
def _small_ensemble():
    parts = [orbits.circular(4.0, 1.3, 300, 0.02, phase0=0.4),
             orbits.driven_oscillator(0.4, 0.3, 2.0, 257, 0.03, t0=0.1, charge=1.0, weight=0.5),
             _gauss_orbit(n=200, dt=0.3)]
    return Batch.concat(parts)


def test_rotation_invariance():
    b = _small_ensemble()
    dirs = np.array([[1, 0, 0], [0.3, 0.4, -0.5], [0, 0, 1]], dtype=float)
    om = log_grid(0.1, 50, 33)
    S0 = spectrum_of(b, dirs, om)
    ang = 0.77
    Rz = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(1.1), -np.sin(1.1)], [0, np.sin(1.1), np.cos(1.1)]])
    R = Rx @ Rz
    S1 = spectrum_of(orbits.rotate(b, R), (R @ dirs.T).T, om)
    np.testing.assert_allclose(S1, S0, rtol=1e-10, atol=1e-14 * S0.max())


def test_time_shift_translation_charge_sign_weight():
    b = _small_ensemble()
    dirs = np.array([[1, 0, 0], [0.3, 0.4, -0.5]], dtype=float)
    om = log_grid(0.1, 50, 29)
    S0 = spectrum_of(b, dirs, om)
    c = Batch.concat([b.select([i]) for i in range(b.n_particles)])
    c.t0 = c.t0 + 17.5
    c.x = c.x + 3.0
    c.y = c.y - 1.0
    c.charge = -c.charge
    np.testing.assert_allclose(spectrum_of(c, dirs, om), S0, rtol=1e-9, atol=1e-13 * S0.max())
    w = b.select(range(b.n_particles))
    w.weight = w.weight * 3.0
    np.testing.assert_allclose(spectrum_of(w, dirs, om), 3.0 * S0, rtol=1e-12)


def test_permutation_and_sharding():
    b = _small_ensemble()
    dirs = np.array([[0, 1, 0], [1, 1, 0]], dtype=float)
    om = log_grid(0.1, 50, 21)
    S0 = spectrum_of(b, dirs, om)
    perm = b.select([2, 0, 1])
    np.testing.assert_allclose(spectrum_of(perm, dirs, om), S0, rtol=1e-13)
    shard = spectrum_of(b.select([0, 2]), dirs, om) + spectrum_of(b.select([1]), dirs, om)
    np.testing.assert_allclose(shard, S0, rtol=1e-13)


def test_time_chunks_add_in_amplitude():
    b = orbits.circular(5.0, 1.0, 1000, 0.01)
    om = log_grid(0.5, 300, 17)
    n = [0.2, 0.9, -0.1]
    A = oracle.amplitude(b, 0, n, om)
    m = 377
    first = b.select([0])
    first.offsets = np.array([0, m])
    second = Batch(offsets=np.array([0, 1000 - m]), x=b.x[m:], y=b.y[m:], z=b.z[m:], bx=b.bx[m:],
                   by=b.by[m:], bz=b.bz[m:], ax=b.ax[m:], ay=b.ay[m:], az=b.az[m:],
                   t0=b.t0 + m * b.dt, dt=b.dt, charge=b.charge, weight=b.weight, species=b.species)
    A2 = oracle.amplitude(first, 0, n, om) + oracle.amplitude(second, 0, n, om)
    np.testing.assert_allclose(A2, A, rtol=1e-11, atol=1e-13 * np.abs(A).max())


def test_species_reduction_and_per_particle_terms():
    b = _small_ensemble()
    b.species = np.array([1, 0, 1], dtype=np.int32)
    dirs = np.array([[0, 0, 1]], dtype=float)
    om = log_grid(0.2, 20, 11)
    S, pp = oracle.spectrum(b, dirs, om, n_species=2, per_particle=True)
    np.testing.assert_allclose(S[0], pp[1], rtol=1e-15)
    np.testing.assert_allclose(S[1], pp[0] + pp[2], rtol=1e-15)
    single = []
    for i in range(3):
        one = b.select([i])
        one.species = np.zeros(1, dtype=np.int32)
        single.append(spectrum_of(one, dirs, om))
    for i in range(3):
        np.testing.assert_allclose(pp[i], single[i], rtol=1e-15)


# ---------------------------------------------------------------- P8 (extended precision)
def test_terms_against_50_digit_arithmetic():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    b = orbits.circular(8.0, 1.0, 12, 0.05, phase0=0.3)
    nvec = np.array([0.6, 0.0, 0.8])
    om = np.array([3.0, 250.0, 4000.0])
    A = oracle.amplitude(b, 0, nvec, om)
    for j, w in enumerate(om):
        acc = [mp.mpc(0)] * 3
        for k in range(12):
            beta = [mp.mpf(float(v)) for v in (b.bx[k], b.by[k], b.bz[k])]
            bd = [mp.mpf(float(v)) for v in (b.ax[k], b.ay[k], b.az[k])]
            r = [mp.mpf(float(v)) for v in (b.x[k], b.y[k], b.z[k])]
            nn = [mp.mpf(float(v)) for v in nvec]
            kap = 1 - sum(nn[i] * beta[i] for i in range(3))
            u = [nn[i] - beta[i] for i in range(3)]
            c1 = [u[1] * bd[2] - u[2] * bd[1], u[2] * bd[0] - u[0] * bd[2], u[0] * bd[1] - u[1] * bd[0]]
            c2 = [nn[1] * c1[2] - nn[2] * c1[1], nn[2] * c1[0] - nn[0] * c1[2],
                  nn[0] * c1[1] - nn[1] * c1[0]]
            tau = mp.mpf(float(b.t0[0])) + k * mp.mpf(float(b.dt[0])) - sum(nn[i] * r[i] for i in range(3))
            ph = mp.expj(mp.mpf(float(w)) * tau) * mp.mpf(float(b.dt[0]))
            for i in range(3):
                acc[i] += c2[i] / kap**2 * ph
        ref = np.array([complex(a) for a in acc])
        assert np.max(np.abs(A[j] - ref)) <= 1e-12 * np.max(np.abs(ref))


# ---------------------------------------------------------------- error behaviour
def test_superluminal_and_bad_direction_rejected():
    b = Batch.concat([orbits.circular(3.0, 1.0, 50, 0.01), orbits.straight([0.5, 0, 0], [0, 0, 0], 40, 0.1)])
    b.bx[60] = 1.0  # |beta| = 1 in particle 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.spectrum(b, [[1, 0, 0]], [1.0, 2.0])
    assert e.value.status == oracle.LWO_ERANGE and e.value.where == 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.spectrum(b.select([0]), [[0, 0, 0]], [1.0])
    assert e.value.status == oracle.LWO_EINVAL


def test_empty_particle_contributes_nothing():
    b = Batch.concat([orbits.circular(3.0, 1.0, 50, 0.01), orbits.circular(3.0, 1.0, 0, 0.01)])
    S, pp = oracle.spectrum(b, [[1, 0, 0]], [1.0, 5.0], per_particle=True)
    assert np.all(pp[1] == 0)
    assert np.all(S[0] == pp[0])


def test_sampled_bins_equal_the_full_spectrum():
    """The sampled-bin routine (used on the full workloads) agrees with lwo_spectrum bin by bin."""
    b = _small_ensemble()
    b.species = np.array([0, 1, 0], dtype=np.int32)
    dirs = np.array([[1, 0, 0], [0.3, 0.4, -0.5], [0, 0, 1]], dtype=float)
    om = log_grid(0.1, 50, 13)
    S = oracle.spectrum(b, dirs, om, n_species=2)
    picks = [(0, 0), (1, 5), (2, 12), (1, 7)]
    d_, w_ = dirs[[d for d, _ in picks]], om[[j for _, j in picks]]
    got_all = oracle.sampled_bins(b, d_, w_)
    got_s1 = oracle.sampled_bins(b, d_, w_, species=1)
    for i, (d, j) in enumerate(picks):
        assert abs(got_all[i] - (S[0, d, j] + S[1, d, j])) <= 1e-13 * got_all[i]
        assert abs(got_s1[i] - S[1, d, j]) <= 1e-13 * max(got_s1[i], 1e-300)
