"""CPU emulation of the spreading kernel's index logic (no GPU).

The matrix-core path spreads each (particle, direction, band) column's samples onto a uniform
grid: sample s adds its W tap values to grid points lo_s .. lo_s + W - 1.  The kernel walks the
samples in chunks of up to 256 and keeps running sums in a ring of kRing grid points (slot
q mod kRing).  A chunk takes the samples whose taps stay within kRing of the oldest unwritten
point (and leaves its last sample to the next chunk, so that the next first tap is known); a
table gives the first sample reaching each point of the chunk; each pair of adjacent points
(x0 = 2 y, x0 + 1) is summed over the samples reaching either, reading taps x0 - lo and
x0 + 1 - lo from rows padded with a zero tap on each side; a point below the next chunk's first
tap is final, is written and its slot cleared; points no sample reaches are written as zeros.  This module re-states that logic step by step, with the kernel's clamps and sizes, and
checks on random first-tap sequences -- dense, sparse (3 to 7 points per sample), gapped,
co-located -- at rings of 512 (the kernel's), 768 and 1024 that

* every index stays inside its buffer (first-sample table, padded tap rows, ring, column),
* no ring slot ever holds the running sums of two grid points at once,
* every grid point below Q is written exactly once and equals the brute-force sum of the taps
  that land on it,

and that on disordered data (which the kernel reports as a data error) the walk still ends in
bounds.
"""
import numpy as np
import pytest

CHUNK = 256


def emulate(lo_all, vals, Q, W, k_ring, strict=True):
    """Index logic of one column: returns (F, write counts).  vals[s, i] is sample s's value
    on tap i (one component stands for the four of the kernel)."""
    n = len(lo_all)
    F = np.zeros(Q)
    writes = np.zeros(Q, dtype=int)
    ring = np.zeros(k_ring)
    owner = np.full(k_ring, -1)  # grid point whose running sum a slot holds (-1: none)

    def clamp(v, a, b):
        return min(max(v, a), b)

    # tap rows as the kernel keeps them: a zero before tap 0 and after tap W - 1
    wpad = np.zeros((n, W + 2))
    wpad[:, 1:W + 1] = vals
    qdone, kc, guard = 0, 0, 0
    while kc < n:
        guard += 1
        assert guard < 10 * n + 10, "chunk walk does not end"
        cnt = min(CHUNK, n - kc)
        lo = lo_all[kc:kc + cnt]
        base = lo[0]
        more = kc + cnt < n
        fits = sum(1 for t in range(cnt) if lo[t] - qdone <= k_ring - W)
        take = max(min(fits, cnt - 1 if more else cnt), 1)
        top = lo[take - 1] + W - 1
        G = min(top - base + 1, k_ring)
        qfin = Q
        if kc + take < n:
            qfin = min(Q, lo[take] if take < cnt else top + 1)
        first = np.full(k_ring + W + 1, -12345)
        for t in range(take):
            prev = base - 1 if t == 0 else lo[t - 1] + W - 1
            mine = lo[t] + W - 1
            for x in range(max(prev + 1, base) - base, min(mine - base, G - 1) + 1):
                assert 0 <= x < len(first)
                first[x] = t
        for t in range(W + 1):
            assert 0 <= max(G, 0) + t < len(first)
            first[max(G, 0) + t] = take
        ring0 = base % k_ring
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
                acc[0] += wpad[kc + s, r]
                acc[1] += wpad[kc + s, r + 1]
            for j in range(2):
                x = x0 + j
                if x >= G:
                    continue
                q = base + x
                slot = ring0 + x if ring0 + x < k_ring else ring0 + x - k_ring
                assert 0 <= slot < k_ring
                if strict:
                    assert owner[slot] in (-1, q), f"slot {slot} holds point {owner[slot]} and {q}"
                v = ring[slot] + acc[j]
                if q < qfin:
                    assert 0 <= q < Q
                    F[q] = v
                    writes[q] += 1
                    ring[slot], owner[slot] = 0.0, -1
                else:
                    ring[slot], owner[slot] = v, q
        for q in range(qdone, min(base, qfin)):
            F[q] = 0.0
            writes[q] += 1
        for q in range(max(base + G, qdone), qfin):
            F[q] = 0.0
            writes[q] += 1
        qdone = max(qdone, qfin)
        kc += take
    return F, writes


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
@pytest.mark.parametrize("k_ring", [512, 768, 1024])
@pytest.mark.parametrize("kind", sorted(SPACINGS))
def test_every_point_written_once_and_equal_to_brute_force(kind, k_ring, W):
    rng = np.random.default_rng(sum(map(ord, kind)) * 7919 + k_ring * 31 + W)
    for n in (1, 2, 255, 256, 257, 700):
        lo, Q = ordered_case(rng, n, SPACINGS[kind], W)
        vals = rng.normal(size=(n, W))
        F, writes = emulate(lo, vals, Q, W, k_ring)
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


def test_sparse_first_chunk_spanning_the_ring():
    """The case the ring's origin rule exists for: spacings of 3 to 7 points, so that a first
    chunk's taps reach past point kRing while point 0 is still unwritten (rings of 512 and 768)."""
    rng = np.random.default_rng(12)
    for k_ring in (512, 768):
        hit = 0
        for _ in range(40):
            lo, Q = ordered_case(rng, 600, SPACINGS["sparse_3_7"], 10)
            hit += int(lo[min(254, len(lo) - 1)] + 9 >= k_ring)
            vals = rng.normal(size=(600, 10))
            F, writes = emulate(lo, vals, Q, 10, k_ring)
            assert np.all(writes == 1)
            np.testing.assert_allclose(F, brute(lo, vals, Q, 10), rtol=1e-12, atol=1e-12)
        assert hit > 0
