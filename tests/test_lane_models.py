"""CPU models of the lane-level steps of three kernels, checked against brute
force (no device).

* Segmented run sums over a 64-lane wavefront (the scatters and the
  pair-side weight gradient): a Hillis-Steele scan over row shifts of 1, 2, 4
  and 8 lanes within rows of 16 lanes, then carries from lanes 15, 31 and 47;
  each step adds the shifted partial sum only while no run start lies
  between.  Every lane must end with the sum of its run up to itself, so
  the last lane of each run holds the run's total, for keys in any order.
* The sorted-key variant used by the dual form's scatter (a step is taken
  when the shifted lane's key equals the lane's own, which is exact for
  sorted keys).
* The pair search's lane mapping: a wavefront takes one galaxy's candidates
  from 27 neighbour cells as one list (an exclusive prefix of the cell counts
  over lanes 0..26, a search of that prefix per lane), tests 64 entries at a
  time and places each kept pair by a ballot rank; the result must be the
  pairs of a serial loop over the cells, in the same order.
"""
import numpy as np


def _shr(vals, d, old):
    out = np.full(64, old, dtype=vals.dtype)
    for lane in range(64):
        if lane % 16 >= d:
            out[lane] = vals[lane - d]
    return out


def seg_runs(keys, v):
    lane = np.arange(64)
    lr, row = lane & 15, lane >> 4
    prev, nxt = np.roll(keys, 1), np.roll(keys, -1)
    h = ((lane == 0) | (prev != keys)).astype(int)
    tail = (lane == 63) | (nxt != keys)
    m = np.zeros(64, int)
    for bit, d in enumerate((1, 2, 4, 8)):
        hs = _shr(h, d, 1)
        c = (lr >= d) & (h == 0)
        m |= np.where(c, 1 << bit, 0)
        h = np.where(c, h | hs, h)
    for bit, (r, src) in enumerate(((1, 15), (2, 31), (3, 47))):
        cs = h[src]
        c = (row == r) & (h == 0)
        m |= np.where(c, 1 << (4 + bit), 0)
        h = np.where(c, h | cs, h)
    v = v.copy()
    for bit, d in enumerate((1, 2, 4, 8)):
        v = v + np.where(m & (1 << bit), _shr(v, d, 0.0), 0.0)
    for bit, src in enumerate((15, 31, 47)):
        v = v + np.where(m & (1 << (4 + bit)), v[src], 0.0)
    return v, tail


def sorted_runs(keys, v):
    lane = np.arange(64)
    row = lane >> 4
    k = [_shr(keys, d, np.iinfo(np.int64).min) for d in (1, 2, 4, 8)]
    m = [(k[i] == keys) for i in range(4)]
    m += [(row == 1) & (keys == keys[15]), (row == 2) & (keys == keys[31]),
          (row == 3) & (keys == keys[47])]
    tail = (lane == 63) | (np.roll(keys, -1) != keys)
    v = v.copy()
    for i, d in enumerate((1, 2, 4, 8)):
        v = v + np.where(m[i], _shr(v, d, 0.0), 0.0)
    for i, src in enumerate((15, 31, 47)):
        v = v + np.where(m[4 + i], v[src], 0.0)
    return v, tail


def _brute(keys, v):
    out = np.zeros(64)
    for lane in range(64):
        st = lane
        while st > 0 and keys[st - 1] == keys[lane]:
            st -= 1
        out[lane] = v[st:lane + 1].sum()
    return out, np.array([lane == 63 or keys[lane + 1] != keys[lane] for lane in range(64)])


def test_segmented_run_sums_any_key_order():
    rng = np.random.default_rng(0)
    for trial in range(3000):
        n = int(rng.integers(0, 65))
        keys = rng.integers(0, int(rng.integers(1, 10)), n)
        if trial % 2:
            keys = np.repeat(keys, rng.integers(1, 20, n))[:n]
        keys = np.concatenate([keys, -1 - np.arange(n, 64)])  # idle lanes: unique keys
        v = rng.normal(size=64)
        got, tail = seg_runs(keys, v)
        exp, etail = _brute(keys, v)
        assert np.allclose(got, exp, rtol=0, atol=1e-12)
        assert np.array_equal(tail, etail)
        for key in np.unique(keys):  # the run tails carry every contribution once
            assert abs(got[tail & (keys == key)].sum() - v[keys == key].sum()) < 1e-12


def test_sorted_key_run_sums():
    rng = np.random.default_rng(1)
    for trial in range(3000):
        n = int(rng.integers(0, 65))
        keys = np.sort(rng.integers(0, int(rng.integers(1, 40)), n))
        keys = np.concatenate([keys, 1000 + np.arange(64 - n)])
        v = rng.normal(size=64)
        got, tail = sorted_runs(keys, v)
        exp, etail = _brute(keys, v)
        assert np.allclose(got, exp, rtol=0, atol=1e-12)
        assert np.array_equal(tail, etail)


def _wave_pairs(qs, cn, keep):
    """Lane-level model: returns the kept (q) in output order."""
    lane = np.arange(64)
    cn64 = np.zeros(64, np.int64); cn64[:27] = cn
    qs64 = np.zeros(64, np.int64); qs64[:27] = qs
    inc = cn64.copy()
    d = 1
    while d < 32:  # Hillis-Steele inclusive scan, shifts up to 16
        up = np.concatenate([np.zeros(d, np.int64), inc[:-d]])
        inc = np.where(lane >= d, inc + up, inc)
        d <<= 1
    pre = inc - cn64
    total = int(inc[26])
    out = []
    for base in range(0, total, 64):
        idx = base + lane
        o = np.zeros(64, np.int64)
        for k in range(1, 27):
            o = np.where(pre[k] <= idx, k, o)
        q = qs64[o] + (idx - pre[o])
        ok = (idx < total) & np.array([keep(int(v)) for v in q]) & (idx < total)
        ballot = np.flatnonzero(ok)
        for r, ln in enumerate(ballot):  # rank = kept lanes below
            assert r == int(np.sum(ok[:ln]))
            out.append(int(q[ln]))
    return out


def test_pair_search_lane_mapping_keeps_the_serial_order():
    rng = np.random.default_rng(3)
    for trial in range(400):
        # 27 neighbour cells: empty, sparse or crowded, possibly cut by the
        # galaxy's own position
        cn = rng.choice([0, 0, 1, 2, 5, 40, 130], 27)
        qs = np.cumsum(np.concatenate([[int(rng.integers(0, 5))], cn[:-1] + rng.integers(0, 4, 26)]))
        keep_set = set(int(v) for v in rng.integers(0, int(qs[-1] + cn[-1] + 1), 200))
        keep = lambda v: (v % 3 != 0) or v in keep_set
        serial = [int(q) for o in range(27) for q in range(qs[o], qs[o] + cn[o]) if keep(int(q))]
        assert _wave_pairs(qs, cn, keep) == serial
