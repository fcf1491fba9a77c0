"""Reference (NumPy, FP64) of the pitch-cone selection (Section 3.2).

TEST INFRASTRUCTURE: the GPU pitch-cone kernel is checked against this.

The paper compares subsets of the ensemble whose momenta lie in a narrow cone of half
width dtheta = 1/Gamma_bulk around inclinations theta_m = m pi / 8 from the streaming
direction, against the whole ensemble, as histograms in gamma^2.  Its figure reports the
relative deviation from isotropy: the subset's share of each gamma^2 bin divided by the
share an isotropic distribution would put in the cone (1 = isotropic, 4 = three times more
than isotropic).  Readings:

* the pitch angle is theta = angle(p, streaming axis) folded to [0, pi/2], i.e.
  cos theta = |p . a| / |p| (the printed arctan of p_par / |p_perp| would put a particle
  moving along the stream at 90 degrees, against the text's "theta_C = 0 is head-on");
* a particle is in cone m when theta_lo <= theta <= theta_hi, with theta_lo =
  max(0, theta_m - dtheta) and theta_hi = min(pi/2, theta_m + dtheta), decided as
  cos theta_hi <= cos theta <= cos theta_lo (bounds from the C library's cos);
* an isotropic distribution puts cos theta_lo - cos theta_hi of its particles in the cone
  (the folded angle has density sin theta on [0, pi/2]);
* gamma^2 = 1 + |u|^2 (u = gamma beta) is binned into [edge_i, edge_{i+1}); particles
  outside the edges are not counted.

Outputs: counts [n_cones + 1][n_bins] (row n_cones: all particles), deviation
[n_cones][n_bins] = (counts_m / counts_all) / (cos theta_lo - cos theta_hi) (NaN where a
bin is empty), membership [P] (the first cone that holds the particle, -1 for none).
"""
import math

import numpy as np


def cone_bounds(theta_c, dtheta):
    """(cos theta_hi, cos theta_lo) per cone, with the C library's cos."""
    out = []
    for t in theta_c:
        lo = max(0.0, t - dtheta)
        hi = min(0.5 * math.pi, t + dtheta)
        out.append((math.cos(hi), math.cos(lo)))
    return np.array(out)


def pitch_cones(ux, uy, uz, axis, theta_c, dtheta, edges):
    ux, uy, uz = (np.asarray(v, dtype=np.float64) for v in (ux, uy, uz))
    a = np.asarray(axis, dtype=np.float64)
    a = a / math.sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2])
    u2 = ux * ux + uy * uy + uz * uz
    upar = np.abs(ux * a[0] + uy * a[1] + uz * a[2])
    with np.errstate(invalid="ignore", divide="ignore"):
        c = np.where(u2 > 0, upar / np.sqrt(u2), 1.0)  # a particle at rest counts as on-axis
    g2 = 1.0 + u2
    edges = np.asarray(edges, dtype=np.float64)
    nb = edges.size - 1
    b = np.searchsorted(edges, g2, side="right") - 1  # edges[b] <= g2 < edges[b + 1]
    inside = (b >= 0) & (b < nb)
    bounds = cone_bounds(theta_c, dtheta)
    nc = len(theta_c)
    counts = np.zeros((nc + 1, nb), dtype=np.int64)
    member = np.full(ux.size, -1, dtype=np.int32)
    np.add.at(counts[nc], b[inside], 1)
    for m in range(nc):
        sel = (c >= bounds[m, 0]) & (c <= bounds[m, 1])
        member[(member < 0) & sel] = m
        np.add.at(counts[m], b[inside & sel], 1)
    frac = bounds[:, 1] - bounds[:, 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        dev = (counts[:nc] / counts[nc][None, :]) / frac[:, None]
    dev[:, counts[nc] == 0] = np.nan
    return counts, dev, member
