"""CPU emulation of the spreading kernel's index logic (no GPU).

The matrix-core path spreads each (particle, direction, band) column's samples onto a uniform
grid: sample s adds its W tap values to grid points lo_s .. lo_s + W - 1.  One work-group
walks a particle's samples for a group of up to two bands, in chunks of up to 256 samples
loaded once: a chunk takes the samples whose taps stay within kWin points of the oldest
unwritten point in every band of the group (and leaves its last sample to the next chunk, so
that the next first tap is known).  Per band, a table gives the first sample reaching each
point of the chunk; each pair of adjacent points (x0 = 2 y, x0 + 1) is summed over the samples
reaching either, reading taps x0 - lo and x0 + 1 - lo from rows padded with a zero tap on each
side; a point below the next chunk's first tap is final and is written; the points at or above
it (fewer than W) are carried to the next chunk in a W-entry buffer (two, used in turn) and
added there to the first W points; points no sample reaches are written as zeros.  This module
re-states that logic step by step, with the kernel's clamps and sizes, and checks on random
first-tap sequences -- dense, sparse (3 to 7 points per sample), gapped, co-located -- at
windows of 512 (the kernel's), 768 and 1024, for one band and for two bands sharing the walk,
that

* every index stays inside its buffer (first-sample table, padded tap rows, carry, column),
* every carried sum lands on a point of the next chunk's window,
* every grid point below Q is written exactly once and equals the brute-force sum of the taps
  that land on it,

and that on disordered data (which the kernel reports as a data error) the walk still ends in
bounds.
"""
import numpy as np
import pytest

CHUNK = 256


def emulate_group(los, vals_list, Qs, W, k_win, strict=True):
    """Index logic of one work-group (one column per band, bands walked together): returns
    [(F, write counts)] per band.  vals[s, i] is sample s's value on tap i (one component
    stands for the four of the kernel)."""
    nb = len(los)
    n = len(los[0])
    F = [np.zeros(Q) for Q in Qs]
    writes = [np.zeros(Q, dtype=int) for Q in Qs]
    # tap rows as the kernel keeps them: a zero before tap 0 and after tap W - 1
    wpad = []
    for vals in vals_list:
        w = np.zeros((n, W + 2))
        w[:, 1:W + 1] = vals
        wpad.append(w)
    carry = [[np.zeros(W), np.zeros(W)] for _ in range(nb)]
    qdone, cbase, par = [0] * nb, [0] * nb, [0] * nb

    def clamp(v, a, b):
        return min(max(v, a), b)

    kc, guard = 0, 0
    while kc < n:
        guard += 1
        assert guard < 10 * n + 10, "chunk walk does not end"
        cnt = min(CHUNK, n - kc)
        more = kc + cnt < n
        # __syncthreads_count: threads whose sample fits in every band (a prefix on valid data)
        fits = sum(1 for t in range(cnt)
                   if all(los[b][kc + t] - qdone[b] <= k_win - W for b in range(nb)))
        take = max(min(fits, cnt - 1 if more else cnt), 1)
        last = kc + take >= n
        for b in range(nb):
            lo = los[b][kc:kc + cnt]
            Q = Qs[b]
            base = lo[0]
            top = lo[take - 1] + W - 1
            G = min(top - base + 1, k_win)
            qfin = Q if last else min(Q, lo[take] if take < cnt else top + 1)
            first = np.full(k_win + W + 1, -12345)
            for t in range(take):
                prev = base - 1 if t == 0 else lo[t - 1] + W - 1
                mine = lo[t] + W - 1
                for x in range(max(prev + 1, base) - base, min(mine - base, G - 1) + 1):
                    assert 0 <= x < len(first)
                    first[x] = t
            for t in range(W + 1):
                assert 0 <= max(G, 0) + t < len(first)
                first[max(G, 0) + t] = take
            cin = carry[b][par[b]]
            cout = carry[b][par[b] ^ 1]
            cout[:] = 0.0
            used = np.zeros(W, dtype=bool)
            for y in range((G + 1) // 2):
                x0 = 2 * y
                q0 = base + x0
                assert 0 <= x0 + 1 + W < len(first)
                sb = clamp(first[x0], 0, take)
                se = clamp(first[x0 + 1 + W], sb, take)
                acc = [0.0, 0.0]
                for s in range(sb, se):
                    assert 0 <= s < CHUNK
                    r = clamp(q0 - lo[s], -1, W - 1) + 1
                    assert 0 <= r and r + 1 <= W + 1
                    acc[0] += wpad[b][kc + s, r]
                    acc[1] += wpad[b][kc + s, r + 1]
                for j in range(2):
                    x = x0 + j
                    if x >= G:
                        continue
                    q = base + x
                    v = acc[j]
                    ci = q - cbase[b]
                    if 0 <= ci < W:
                        v += cin[ci]
                        used[ci] = True
                    if q < qfin:
                        assert 0 <= q < Q
                        F[b][q] = v
                        writes[b][q] += 1
                    else:
                        co = q - qfin
                        if strict and q < Q:  # points past the column are never written
                            assert 0 <= co < W, f"open point {q} is {co} past the final ones"
                        if 0 <= co < W:
                            cout[co] = v
            if strict:
                # every sum carried in for a point of the column is read by this chunk
                inside = cbase[b] + np.arange(W) < Q
                assert np.all(cin[~used & inside] == 0.0), "a carried sum fell outside the next chunk"
            for q in range(qdone[b], min(base, qfin)):
                F[b][q] = 0.0
                writes[b][q] += 1
            for q in range(max(base + G, qdone[b]), qfin):
                F[b][q] = 0.0
                writes[b][q] += 1
            qdone[b] = max(qdone[b], qfin)
            cbase[b] = qfin
            par[b] ^= 1
        kc += take
    return list(zip(F, writes))


def emulate(lo_all, vals, Q, W, k_win, strict=True):
    """One band alone."""
    return emulate_group([lo_all], [vals], [Q], W, k_win, strict)[0]


def brute(lo, vals, Q, W):
    F = np.zeros(Q)
    for s, l in enumerate(lo):
        for i in range(W):
            if l + i < Q:
                F[l + i] += vals[s, i]
    return F


def ordered_case(rng, n, spacing, W):
    """First taps of n samples with the given per-sample spacing generator, from lo = 1 (the
    smallest first tap the kernel produces), and the column length the kernel would use."""
    steps = spacing(rng, n)
    lo = 1 + np.concatenate([[0], np.cumsum(steps[1:])]).astype(int)
    Q = int(lo[-1] + W + 1 + rng.integers(0, 3))
    return lo, Q


SPACINGS = {
    "dense": lambda rng, n: (rng.random(n) < 0.2).astype(int),
    "sparse_3_7": lambda rng, n: rng.integers(3, 8, n),
    "mixed": lambda rng, n: np.where(rng.random(n) < 0.5, rng.integers(0, 2, n), rng.integers(2, 6, n)),
    "gapped": lambda rng, n: np.where(rng.random(n) < 0.01, rng.integers(900, 3000, n), rng.integers(0, 3, n)),
    "co_located": lambda rng, n: np.zeros(n, dtype=int),
}


@pytest.mark.parametrize("W", [8, 10])
@pytest.mark.parametrize("k_win", [512, 768, 1024])
@pytest.mark.parametrize("kind", sorted(SPACINGS))
def test_every_point_written_once_and_equal_to_brute_force(kind, k_win, W):
    rng = np.random.default_rng(sum(map(ord, kind)) * 7919 + k_win * 31 + W)
    for n in (1, 2, 255, 256, 257, 700):
        lo, Q = ordered_case(rng, n, SPACINGS[kind], W)
        vals = rng.normal(size=(n, W))
        F, writes = emulate(lo, vals, Q, W, k_win)
        assert np.all(writes == 1), (kind, n, np.flatnonzero(writes != 1)[:10])
        np.testing.assert_allclose(F, brute(lo, vals, Q, W), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("W", [8, 10])
def test_column_clipped_by_the_plan(W):
    """A span past the plan: first taps pile up at qmax + 1 (the kernel clamps the grid
    coordinate), Q = qmax; points below Q are still written once."""
    rng = np.random.default_rng(5)
    lo, _ = ordered_case(rng, 600, SPACINGS["sparse_3_7"], W)
    qmax = int(lo[300])
    lo = np.minimum(lo, qmax + 1)
    vals = rng.normal(size=(600, W))
    F, writes = emulate(lo, vals, qmax, W, 512)
    assert np.all(writes == 1)
    np.testing.assert_allclose(F, brute(lo, vals, qmax, W), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_disordered_data_ends_in_bounds(seed):
    """Out-of-order first taps (invalid samples are put at lo = 1, other orders come from
    inconsistent positions): the walk ends and indices stay in their buffers (asserted
    inside); values and write counts are not checked (the kernel reports such data)."""
    rng = np.random.default_rng(seed)
    W = 10
    lo = rng.integers(1, 3000, 700)
    lo[rng.random(700) < 0.3] = 1
    Q = 3000 + W + 1
    vals = rng.normal(size=(700, W))
    emulate(lo, vals, Q, W, 512, strict=False)


def test_sparse_first_chunk_spanning_the_window():
    """Spacings of 3 to 7 points, so that a first chunk's taps reach past point kWin while
    point 0 is still unwritten (windows of 512 and 768): the chunk stops short of them."""
    rng = np.random.default_rng(12)
    for k_win in (512, 768):
        hit = 0
        for _ in range(40):
            lo, Q = ordered_case(rng, 600, SPACINGS["sparse_3_7"], 10)
            hit += int(lo[min(254, len(lo) - 1)] + 9 >= k_win)
            vals = rng.normal(size=(600, 10))
            F, writes = emulate(lo, vals, Q, 10, k_win)
            assert np.all(writes == 1)
            np.testing.assert_allclose(F, brute(lo, vals, Q, 10), rtol=1e-12, atol=1e-12)
        assert hit > 0


@pytest.mark.parametrize("W", [8, 10])
@pytest.mark.parametrize("kind", sorted(SPACINGS))
@pytest.mark.parametrize("ratio", [1, 3, 9, 40])
def test_two_bands_share_the_walk(kind, ratio, W):
    """Two bands of one work-group: the second band's grid is `ratio` times coarser (as a
    lower frequency band is), so its first taps advance more slowly; the chunks are common and
    each band's column is still written once and equals its brute-force sum.  A ratio below one
    (the coarse band first) is the same walk with the bands swapped."""
    rng = np.random.default_rng(sum(map(ord, kind)) * 131 + ratio * 7 + W)
    for n in (1, 255, 256, 257, 700):
        lo_a, Q_a = ordered_case(rng, n, SPACINGS[kind], W)
        lo_b = 1 + (lo_a - 1) // ratio
        Q_b = int(lo_b[-1] + W + 1)
        vals_a, vals_b = rng.normal(size=(n, W)), rng.normal(size=(n, W))
        for order in ((0, 1), (1, 0)):
            los = [(lo_a, lo_b)[i] for i in order]
            vals = [(vals_a, vals_b)[i] for i in order]
            Qs = [(Q_a, Q_b)[i] for i in order]
            out = emulate_group(los, vals, Qs, W, 512)
            for (F, writes), lo, v, Q in zip(out, los, vals, Qs):
                assert np.all(writes == 1), (kind, n, order)
                np.testing.assert_allclose(F, brute(lo, v, Q, W), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_two_bands_disordered_data_end_in_bounds(seed):
    """Disordered first taps in one band of a pair (the other valid): the common walk ends
    and every index stays in its buffer."""
    rng = np.random.default_rng(100 + seed)
    W = 10
    lo_a, Q_a = ordered_case(rng, 700, SPACINGS["mixed"], W)
    lo_b = rng.integers(1, 3000, 700)
    lo_b[rng.random(700) < 0.3] = 1
    vals = [rng.normal(size=(700, W)), rng.normal(size=(700, W))]
    emulate_group([lo_a, lo_b], vals, [Q_a, 3000 + W + 1], W, 512, strict=False)
