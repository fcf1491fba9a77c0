"""Pins of the spectral-diagnostics oracle (CPU): closed forms the definitions must reproduce."""
import numpy as np

from oracle import diagnostics as dg

W = np.exp(np.linspace(np.log(0.1), np.log(1e3), 401))  # log grid, step h in ln w
H = np.log(W[1] / W[0])


def _broken(a, b, kb):
    x = np.log(W / W[kb])
    return np.exp(np.where(x < 0, a * x, b * x))


def test_broken_power_law_slopes_and_kink_peak():
    a, b, kb = 1.0, -1.5, 200
    r = dg.row_diagnostics(_broken(a, b, kb), W)
    assert r[0] == kb and r[1] == W[kb] and r[3] == 1.0
    assert abs(r[4] - a) < 1e-12 and abs(r[6] - b) < 1e-12
    # the parabola through a kink of slopes a, b on a uniform ln-grid has its vertex at
    # h (a + b) / (2 (a - b)) from the kink
    assert abs(np.log(r[2] / W[kb]) - H * (a + b) / (2 * (a - b))) < 1e-12
    # bin counts: w in [0.01, 0.3] w_k and [3, 30] w_k on the grid
    lw = np.log(W / W[kb])
    assert r[5] == np.sum((lw >= np.log(0.01) - 1e-12) & (lw <= np.log(0.3) + 1e-12))
    assert r[7] == np.sum((lw >= np.log(3.0) - 1e-12) & (lw <= np.log(30.0) + 1e-12))


def test_log_gaussian_peak_is_found_between_grid_points():
    x0 = np.log(3.7)  # not a grid point
    S = 5.0 * np.exp(-(np.log(W) - x0) ** 2 / (2 * 0.4**2))
    r = dg.row_diagnostics(S, W)
    assert abs(np.log(r[2]) - x0) < 1e-10
    assert W[int(r[0]) - 1] < 3.7 < W[int(r[0]) + 1]


def test_edge_peak_zero_row_and_ties():
    r = dg.row_diagnostics(W ** -2.0, W)  # falling everywhere: peak at the first bin
    assert r[0] == 0 and r[2] == W[0] and np.isnan(r[4]) and r[5] == 0
    assert abs(r[6] + 2.0) < 1e-12
    z = dg.row_diagnostics(np.zeros(W.size), W)
    assert z[0] == 0 and z[3] == 0 and np.isnan(z[4]) and np.isnan(z[6]) and z[5] == 0 and z[7] == 0
    S = np.ones(W.size)
    S[[50, 300]] = 2.0
    t = dg.row_diagnostics(S, W)
    assert t[0] == 50
    # a flat top does not bend down: the peak stays on the grid
    assert t[2] == W[50] or abs(np.log(t[2] / W[50])) <= H


def test_observer_average_weights():
    f = _broken(1.0, -1.0, 100)
    S = np.stack([(d + 1) * f for d in range(6)])[None]
    a = np.array([0.0, 1.0, 2.0, 0.5, 0.0, 3.0])
    avg, diag = dg.spectral_diagnostics(S, W, weights=a)
    np.testing.assert_allclose(avg[0], np.dot(a, np.arange(1, 7)) / a.sum() * f, rtol=1e-14)
    avg1, _ = dg.spectral_diagnostics(S, W)
    np.testing.assert_allclose(avg1[0], 3.5 * f, rtol=1e-14)
    # every row has the same shape, so the same peak and slopes
    assert np.all(diag[0, :, 0] == 100)
    np.testing.assert_allclose(diag[0, :, 4], 1.0, atol=1e-12)
    np.testing.assert_allclose(diag[0, :, 6], -1.0, atol=1e-12)
