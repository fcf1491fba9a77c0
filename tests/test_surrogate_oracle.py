"""Pins of the FP64 surrogate-network reference and of the feature reference (CPU)."""
import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import features as feat
from workloads import orbits

SHAPE = (5, 7, 2, 4)


def test_gelu_closed_form():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 1.0, 2.0])
    np.testing.assert_allclose(oracle.mlp_gelu(z), z * 0.5 * (1 + sp.erf(z / np.sqrt(2))), rtol=1e-15)
    assert abs(oracle.mlp_gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def test_param_count_of_the_spectrum_network():
    # 16 -> 256 -> 256 -> 256 -> 256
    assert oracle.mlp_num_params(16, 256, 3, 256) == 16 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 256 + 256


def test_linear_network_reduces_to_matrix_product():
    # no hidden layer: y = W x + b
    rng = np.random.default_rng(1)
    W = rng.normal(size=(3, 4))
    b = rng.normal(size=3)
    x = rng.normal(size=(6, 4))
    out = oracle.mlp_forward_backward((4, 1, 0, 3), np.concatenate([W.ravel(), b]), x)
    np.testing.assert_allclose(out["y"], x @ W.T + b, rtol=1e-14)


def test_gradient_against_central_differences():
    rng = np.random.default_rng(2)
    n = oracle.mlp_num_params(*SHAPE)
    p = rng.normal(scale=0.5, size=n)
    x = rng.normal(size=(9, SHAPE[0]))
    t = rng.normal(size=(9, SHAPE[3]))
    g = oracle.mlp_forward_backward(SHAPE, p, x, t, want_grad=True)["grad"]
    h = 1e-6
    for i in rng.choice(n, 25, replace=False):
        e = np.zeros(n)
        e[i] = h
        fd = (oracle.mlp_forward_backward(SHAPE, p + e, x, t)["loss"] -
              oracle.mlp_forward_backward(SHAPE, p - e, x, t)["loss"]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_features_of_uniform_circular_motion():
    """gamma constant, |a_perp| = beta omega0 exactly, no force along beta."""
    g, w0, n, dt = 5.0, 2.0, 4000, 2 * np.pi / 2.0 / 4000
    b = orbits.circular(g, w0, n, dt)
    beta = np.sqrt(1 - 1 / g**2)
    f = feat.features(b, [[0.0, 0.0, 1.0]])[0, 0]
    assert abs(f[0] - np.log(g)) < 1e-12
    assert f[1] < 1e-12
    assert abs(f[2] - np.log(beta * w0)) < 1e-9
    assert abs(f[4] - np.log(beta * w0)) < 1e-9
    assert abs(f[5] - 1.0) < 1e-9
    assert abs(f[10] - np.log(n * dt)) < 1e-12
    # observer along the orbit axis: kappa = 1 everywhere, never inside the 1/gamma cone
    assert abs(f[13]) < 1e-12 and abs(f[14]) < 1e-12 and f[15] == 0.0


def test_features_of_straight_motion():
    b = orbits.straight([0.6, 0.0, 0.0], [0, 0, 0], 100, 0.01)
    f = feat.features(b, [[1.0, 0.0, 0.0]])[0, 0]
    assert f[2] == np.log(feat.EPS) and f[8] == 0.0 and f[6] == 0.0
    assert abs(f[13] - np.log(0.4)) < 1e-12 and f[15] == 1.0  # looking down the velocity


def test_energy_feature_is_the_frequency_integral_of_the_spectrum():
    """exp(feature 11) = int_0^inf S dw (Parseval) for a band-limited orbit, checked
    against the spectral oracle integrated over a fine linear frequency grid."""
    b = orbits.gaussian_oscillator(0.05, 1.0, 6.0, 0.5, 1500, 0.06)
    for th in (0.0, 0.7, 1.9):
        nvec = np.array([np.sin(th) * np.cos(0.3), np.sin(th) * np.sin(0.3), np.cos(th)])
        f = feat.features(b, [nvec])[0, 0]
        om = np.linspace(0.0, 12.0, 2401)
        S = oracle.spectrum(b, [nvec], om, n_species=1)[0, 0]
        assert abs(np.exp(f[11]) / np.trapezoid(S, om) - 1) < 1e-6


def test_energy_feature_of_straight_motion_is_zero():
    b = orbits.straight([0.3, 0.4, 0.0], [0, 0, 0], 50, 0.1)
    f = feat.features(b, [[0.0, 0.0, 1.0], [0.6, 0.8, 0.0]])[0]
    assert np.all(f[:, 11] == np.log(1e-30))


# ---------------------------------------------------------------- features 3, 6, 7, 8, 9, 12
# A constant-speed zigzag, beta = beta0 (cos phi, sin phi, 0) with phi = phi_m sin(W t), fixes
# these features in closed form: gamma is constant, |a_perp| = beta0 |phi'| exactly, over
# whole periods the mean unit velocity is x and the deflection angle is |phi|, and the force
# reverses at every zero of cos(W t).
ZZ_BETA, ZZ_PHI, ZZ_W = 0.8, 0.3, 2.0


def _zigzag(periods, spp, t0_frac):
    dt = 2 * np.pi / ZZ_W / spp
    return orbits.zigzag(ZZ_BETA, ZZ_PHI, ZZ_W, periods * spp, dt, t0=t0_frac * dt), dt


def test_feature_rms_aperp_and_deflection_of_a_zigzag():
    """Samples at t_k = k T / spp over whole periods (spp divisible by 4): the discrete means
    of cos^2 and sin^2 are exactly 1/2 and a sample sits on each turning point, so
    rms |a_perp| = beta0 phi_m W / sqrt 2, gamma theta_rms = gamma phi_m / sqrt 2 and
    gamma theta_max = gamma phi_m."""
    b, dt = _zigzag(periods=5, spp=400, t0_frac=0.0)
    g = 1 / np.sqrt(1 - ZZ_BETA**2)
    f = feat.features(b, [[0.0, 0.0, 1.0]])[0, 0]
    assert abs(f[0] - np.log(g)) < 1e-12
    assert abs(f[3] - np.log(ZZ_BETA * ZZ_PHI * ZZ_W / np.sqrt(2) + feat.EPS)) < 1e-10
    assert abs(f[6] - g * ZZ_PHI / np.sqrt(2)) < 1e-10
    assert abs(f[7] - g * ZZ_PHI) < 1e-10


@pytest.mark.parametrize("periods,spp", [(3, 500), (7, 130)])
def test_feature_reversal_rate_of_a_zigzag(periods, spp):
    """With the first sample a third of a step after t = 0, no sample sits on a zero of
    cos(W t) and every one of the 2 P zeros inside the record falls between two samples:
    exactly 2 P reversals, so rate = 2 P / (N dt) (per unit time, not per sample) and
    feature 9 = ln(gamma^2 rate + 1e-6)."""
    b, dt = _zigzag(periods, spp, t0_frac=1.0 / 3.0)
    n = periods * spp
    g = 1 / np.sqrt(1 - ZZ_BETA**2)
    f = feat.features(b, [[1.0, 0.0, 0.0]])[0, 0]
    rate = 2 * periods / (n * dt)
    assert abs(f[8] / rate - 1) < 1e-13
    assert abs(f[9] - np.log(g * g * rate + 1e-6)) < 1e-12
    # circular motion never reverses the force (consecutive accelerations turn by w0 dt)
    c = feat.features(orbits.circular(3.0, 1.0, 800, 0.01), [[1.0, 0.0, 0.0]])[0, 0]
    assert c[8] == 0.0 and c[9] == np.log(1e-6)


@pytest.mark.parametrize("alpha", [0.0, 0.05, 0.4, 1.3, np.pi - 0.2])
def test_feature_observer_angle_to_the_mean_beam(alpha):
    """Feature 12 is gamma times the angle between n and the mean beam direction (x here),
    not a mean of the angles between n and the instantaneous velocity: with n tilted by
    alpha out of the plane of the swing it is gamma alpha exactly, while the velocity itself
    is never at angle alpha from n except at the zero crossings of phi."""
    b, _ = _zigzag(periods=4, spp=400, t0_frac=0.0)
    g = 1 / np.sqrt(1 - ZZ_BETA**2)
    n = [np.cos(alpha), 0.0, np.sin(alpha)]
    f = feat.features(b, [n])[0, 0]
    assert abs(f[12] - g * alpha) < 1e-10
    # straight motion: the mean direction is the velocity itself
    s = feat.features(orbits.straight([0.6 * np.cos(0.7), 0.6 * np.sin(0.7), 0.0], [0, 0, 0], 20, 0.1),
                      [[1.0, 0.0, 0.0]])[0, 0]
    assert abs(s[12] - 1.25 * 0.7) < 1e-12


def test_feature_gamma_spread_of_a_two_speed_record():
    """Feature 1 (std / mean of gamma) of a record spending equal numbers of samples at
    gamma1 and gamma2 is |gamma2 - gamma1| / (gamma2 + gamma1)."""
    n = 200
    beta = np.zeros((n, 3))
    beta[: n // 2, 0] = 0.6   # gamma 1.25
    beta[n // 2:, 0] = 0.8    # gamma 5/3
    bdot = np.zeros((n, 3))
    bdot[:, 1] = 0.01
    f = feat.features_one(beta, bdot, 0.05, [0.0, 1.0, 0.0])
    g1, g2 = 1.25, 5.0 / 3.0
    assert abs(f[1] - (g2 - g1) / (g2 + g1)) < 1e-13
    assert abs(f[0] - np.log(0.5 * (g1 + g2))) < 1e-13
