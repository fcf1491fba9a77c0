"""Checks of the seeded input generators (not of the method)."""
import os

import numpy as np

import workloads
from workloads import configs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert rows
    for r in rows:
        v = [int(h, 16) for h in r]
        out = workloads.philox4x32_10(v[0:4], v[4:6])
        assert list(out) == v[6:10]


def test_slices_regenerate_bitwise():
    r = configs.jitter_recipe(steps=64)
    a = workloads.generate(r, 0, 8)
    b = workloads.generate(r, 5, 3)
    sub = a.select([5, 6, 7])
    for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az", "t0", "dt", "charge", "species"):
        assert np.array_equal(getattr(sub, k), getattr(b, k)), k


def test_field_rms_and_deflection_parameter():
    r = configs.jitter_recipe(steps=16)
    n_modes, brms, kbar = workloads.field_info(r)
    assert 380 <= n_modes <= 420
    assert abs(brms / kbar - r.delta) < 1e-12
    g = np.arange(64) * (r.box / 64)
    X, Z = np.meshgrid(g, g, indexing="ij")
    B = workloads.field_eval(r, X.ravel(), Z.ravel())
    # discrete orthogonality on a 64 x 64 grid over one period: mean B^2 = sum a^2 / 2 exactly
    assert abs(np.sqrt(np.mean(B**2)) / brms - 1) < 1e-10
    assert abs(np.mean(B)) < 1e-10 * brms


def test_beams_speed_and_sampling_rules():
    r = configs.jitter_recipe(steps=512)
    b = workloads.generate(r, 0, 16)
    beta2 = b.bx**2 + b.by**2 + b.bz**2
    assert np.all(beta2 < 1)
    for p in range(16):
        s = slice(b.offsets[p], b.offsets[p + 1])
        # the magnetic push conserves the speed; midpoint velocities stay near it
        sp_ = np.sqrt(beta2[s])
        assert sp_.max() - sp_.min() < 1e-3
        gam = 1 / np.sqrt(1 - sp_.max() ** 2)
        assert 2.2 < gam < 4.2  # gamma0 = 3 boosted from a kT = 0.01 rest-frame spread
        # beams: even ids along +x, odd along -x
        assert np.sign(b.bx[s].mean()) == (1 if p % 2 == 0 else -1)
        # positions advance by the half-step velocity: r_{k+1} - r_k = beta^{k+1/2} dt,
        # and beta_k averages consecutive half-step velocities
        dx = np.diff(b.x[s]) / r.dt
        mid = 0.5 * (dx[:-1] + dx[1:])
        assert np.max(np.abs(mid - b.bx[s][1:-1])) < 1e-12
        acc = np.diff(dx) / r.dt
        assert np.max(np.abs(acc - b.ax[s][1:-1])) < 1e-6 * max(1.0, np.abs(acc).max())


def test_no_field_gives_straight_lines():
    r = workloads.make_recipe(7, steps=100, delta=0.0)
    b = workloads.generate(r, 0, 4)
    assert np.all(b.ax == 0) and np.all(b.ay == 0) and np.all(b.az == 0)


def test_uneven_population_mix():
    r = configs.uneven_recipe()
    lens, spec, g0, q, m = workloads.particle_meta(r, 0, 20000)
    assert lens.min() >= 256 and lens.max() <= 8192
    frac = np.bincount(spec, minlength=3) / spec.size
    assert abs(frac[0] - 0.475) < 0.02 and abs(frac[1] - 0.475) < 0.02 and abs(frac[2] - 0.05) < 0.01
    assert set(np.unique(g0)) == {2.0, 5.0, 15.0}
    assert np.all(q[spec == 0] == -1) and np.all(q[spec > 0] == 1)
    assert np.all(m[spec == 2] == 16) and np.all(m[spec < 2] == 1)


def test_direction_sets():
    for d, n in ((configs.dirs_jitter(), 4), (configs.dirs_wide(), 16), (configs.dirs_equal_area(), 64)):
        assert d.shape == (n, 3)
        np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, rtol=1e-15)
    ea = configs.dirs_equal_area()
    assert np.abs(ea.sum(0)).max() < 1e-12  # symmetric cell centres


def test_two_d_motion_stays_in_the_field_plane():
    """2D2V: no y momentum and y = 0 at start; B along y keeps every sample in the x-z plane."""
    from workloads import configs

    b = workloads.generate(configs.jitter_2d_recipe(steps=600), 0, 8)
    assert np.all(b.y == 0.0) and np.all(b.by == 0.0) and np.all(b.ay == 0.0)
    assert np.all(np.abs(b.bx[b.offsets[:-1]]) > 0.9)  # they start in the counter-streaming beams
    b3 = workloads.generate(configs.jitter_recipe(steps=600), 0, 8)
    assert np.any(b3.by != 0.0)  # the 3D recipe is unchanged


def test_two_d_radiation_has_no_out_of_plane_field_in_plane():
    """In-plane motion seen from an in-plane observer radiates no field along y."""
    import oracle
    from workloads import configs

    b = workloads.generate(configs.jitter_2d_recipe(steps=300), 0, 3)
    dirs = configs.dirs_paper(two_d=True)
    assert np.all(dirs[:, 1] == 0.0)
    _, A = oracle.coherent_spectrum(b, dirs, configs.log_grid(0.1, 100.0, 64), n_species=1,
                                    with_amplitude=True)
    assert np.all(A[..., 1] == 0.0) and np.abs(A).max() > 0
