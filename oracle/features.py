"""Reference (NumPy, FP64) of the 16 per-(particle, direction) features of the surrogate.

TEST INFRASTRUCTURE: the GPU feature kernel is checked against this.  The
features summarise what sets a particle's spectrum in the jitter regime:
Lorentz factor, the transverse acceleration and its moments, the deflection
angle measured in units of the beaming angle 1/gamma, the rate at which the
force reverses (filament crossings), and the observer's position relative to
the beam (kappa statistics).  EPS keeps logarithms finite.

 0 ln <gamma>                 8  force reversals per unit time (rate)
 1 std(gamma) / <gamma>       9  ln(<gamma>^2 rate + 1e-6)
 2 ln(<|a_perp|> + EPS)      10  ln T, T = N dt
 3 ln(rms |a_perp| + EPS)    11  ln(E + 1e-30), E the radiated energy per unit solid angle
 4 ln(max |a_perp| + EPS)    12  <gamma> angle(n, mean beam direction)
 5 <a_perp^4> / <a_perp^2>^2 13  ln <kappa>
 6 <gamma> theta_rms          14  ln min kappa
 7 <gamma> theta_max          15  fraction of samples with angle(n, beta) < 1/gamma

a_perp is the part of d(beta)/dt perpendicular to beta; theta the angle of
beta to the mean unit velocity; a force reversal is a sample whose d(beta)/dt
has a negative dot product with the previous sample's.  E is the Riemann sum
over the samples of |n x ((n - beta) x betadot)|^2 / kappa^5 dt / (4 pi), the
energy per unit solid angle radiated towards n (Jackson, eq. 14.38), which by
Parseval's theorem is the frequency integral of the spectrum in direction n.
"""
import numpy as np

N_FEATURES = 16
EPS = 1e-12


def features_one(beta, bdot, dt, n):
    beta = np.asarray(beta, dtype=np.float64)
    bdot = np.asarray(bdot, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64) / np.linalg.norm(n)
    N = beta.shape[0]
    b2 = np.einsum("ij,ij->i", beta, beta)
    gam = 1.0 / np.sqrt(1.0 - b2)
    bn = np.sqrt(b2)
    bhat = beta / np.where(bn > 0, bn, 1.0)[:, None]
    apar = np.einsum("ij,ij->i", bdot, bhat)
    aperp_v = bdot - apar[:, None] * bhat
    aperp = np.sqrt(np.einsum("ij,ij->i", aperp_v, aperp_v))
    g = gam.mean()
    m2 = np.mean(aperp**2)
    mean_dir = bhat.mean(axis=0)
    e = mean_dir / max(np.linalg.norm(mean_dir), 1e-300)
    cosang = np.clip(bhat @ e, -1.0, 1.0)
    sinang = np.linalg.norm(np.cross(bhat, e), axis=1)
    theta = np.arctan2(sinang, cosang)
    rev = np.count_nonzero(np.einsum("ij,ij->i", bdot[1:], bdot[:-1]) < 0) if N > 1 else 0
    T = N * dt
    rate = rev / T
    kap = 1.0 - beta @ n
    ang_n = np.arctan2(np.linalg.norm(np.cross(bhat, n[None, :]), axis=1), bhat @ n)
    ang_ne = np.arctan2(np.linalg.norm(np.cross(e, n)), e @ n)
    v = np.cross(n[None, :], np.cross(n[None, :] - beta, bdot))
    energy = np.sum(np.einsum("ij,ij->i", v, v) / kap**5) * dt / (4.0 * np.pi)
    return np.array([
        np.log(g),
        gam.std() / g,
        np.log(aperp.mean() + EPS),
        np.log(np.sqrt(m2) + EPS),
        np.log(aperp.max() + EPS),
        np.mean(aperp**4) / (m2 * m2) if m2 > 0 else 0.0,
        g * np.sqrt(np.mean(theta**2)),
        g * theta.max(),
        rate,
        np.log(g * g * rate + 1e-6),
        np.log(T),
        np.log(energy + 1e-30),
        g * ang_ne,
        np.log(kap.mean()),
        np.log(kap.min()),
        np.mean(ang_n < 1.0 / gam),
    ])


def features(batch, dirs):
    """[P][nd][16] features of every particle of a workloads.Batch for every direction."""
    dirs = np.atleast_2d(dirs)
    out = np.zeros((batch.n_particles, dirs.shape[0], N_FEATURES))
    for p in range(batch.n_particles):
        s = slice(batch.offsets[p], batch.offsets[p + 1])
        beta = np.stack([batch.bx[s], batch.by[s], batch.bz[s]], 1)
        bdot = np.stack([batch.ax[s], batch.ay[s], batch.az[s]], 1).astype(np.float64)
        for d, n in enumerate(dirs):
            out[p, d] = features_one(beta, bdot, float(batch.dt[p]), n)
    return out
