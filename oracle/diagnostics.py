"""Reference (NumPy, FP64) of the spectral diagnostics.

TEST INFRASTRUCTURE: the GPU diagnostics kernel is checked against this.  Only
tests, the smoke check and the CPU leg of the benchmark may use it.

The results section (Section 3.3 and the captions of its spectrum figures)
characterises each observer's spectrum by its peak frequency omega_peak and by
low- and high-frequency power-law indices alpha and beta, S ~ omega^alpha below
the peak and S ~ omega^beta above it, and also shows a spectrum averaged over
the six observers spread in inclination (Section 2.2).  The paper reads these
off its plots; the definitions below are the plain quantitative ones:

* observer average: S_avg(w) = sum_d a_d S_d(w) / sum_d a_d, caller weights
  a_d >= 0 (equal weights by default);
* peak: k = the first index of the largest S; refined omega_peak = exp(vertex)
  of the parabola through (ln w, ln S) at k-1, k, k+1 (kept within
  [ln w_{k-1}, ln w_{k+1}]), or w_k itself at an edge of the grid, where a
  neighbour is not positive, or where the three points do not bend down;
* slopes: ordinary least squares of ln S on ln w over the bins with S > 0 and
  alpha_lo w_k <= w <= alpha_hi w_k (alpha), beta_lo w_k <= w <= beta_hi w_k
  (beta); NaN when fewer than two bins qualify.

Each row gives [k, w_k, omega_peak, S_k, alpha, n_alpha, beta, n_beta].
"""
import numpy as np

N_DIAG = 8


def observer_average(S, weights=None):
    """S [..., nd, nw] -> [..., nw]."""
    S = np.asarray(S, dtype=np.float64)
    nd = S.shape[-2]
    a = np.ones(nd) if weights is None else np.asarray(weights, dtype=np.float64)
    assert a.shape == (nd,) and np.all(a >= 0)
    # observers are summed one after another (a rounding order the peak decision can rely on)
    total, acc = 0.0, np.zeros(S.shape[:-2] + S.shape[-1:])
    for d in range(nd):
        total += float(a[d])
        acc = acc + a[d] * S[..., d, :]
    assert total > 0
    return acc / total


def _parabola_vertex(x, y):
    """Vertex abscissa of the parabola through three points, or None if it does not open downwards."""
    (x0, x1, x2), (y0, y1, y2) = x, y
    d = (x0 - x1) * (x0 - x2) * (x1 - x2)
    A = (x2 * (y1 - y0) + x1 * (y0 - y2) + x0 * (y2 - y1)) / d
    B = (x2 * x2 * (y0 - y1) + x1 * x1 * (y2 - y0) + x0 * x0 * (y1 - y2)) / d
    if not A < 0.0:
        return None
    return min(max(-B / (2.0 * A), x0), x2)


def _slope(lw, ls):
    n = lw.size
    if n < 2:
        return np.nan, n
    xm, ym = lw.mean(), ls.mean()
    sxx = np.sum((lw - xm) ** 2)
    if sxx == 0.0:
        return np.nan, n
    return float(np.sum((lw - xm) * (ls - ym)) / sxx), n


def row_diagnostics(S, omega, alpha_range=(1e-2, 0.3), beta_range=(3.0, 30.0)):
    S = np.asarray(S, dtype=np.float64)
    w = np.asarray(omega, dtype=np.float64)
    k = int(np.argmax(S))  # first of equal maxima
    wk, sk = w[k], S[k]
    wpeak = wk
    if 0 < k < w.size - 1 and S[k - 1] > 0 and S[k + 1] > 0 and sk > 0:
        v = _parabola_vertex(np.log(w[k - 1:k + 2]), np.log(S[k - 1:k + 2]))
        if v is not None:
            wpeak = float(np.exp(v))
    out = [float(k), wk, wpeak, sk]
    for lo, hi in (alpha_range, beta_range):
        m = (S > 0) & (w >= lo * wk) & (w <= hi * wk)
        slope, n = _slope(np.log(w[m]), np.log(S[m]))
        out += [slope, float(n)]
    return np.array(out)


def spectral_diagnostics(S, omega, weights=None, alpha_range=(1e-2, 0.3), beta_range=(3.0, 30.0)):
    """S [ns, nd, nw] -> (average [ns, nw], diagnostics [ns, nd + 1, N_DIAG]); row nd is the average's."""
    S = np.asarray(S, dtype=np.float64)
    ns, nd, nw = S.shape
    avg = observer_average(S, weights)
    diag = np.zeros((ns, nd + 1, N_DIAG))
    for s in range(ns):
        for d in range(nd):
            diag[s, d] = row_diagnostics(S[s, d], omega, alpha_range, beta_range)
        diag[s, nd] = row_diagnostics(avg[s], omega, alpha_range, beta_range)
    return avg, diag
