"""Pins of the oracle's TSC mass assignment (the paper's scheme, offered on
the plain FP64 path): the 1-D weights against their moments and the on-node
values, and the 3-D assignment against the CIC assignment averaged over a
unit box of shifts (TSC is CIC convolved with one more cell-wide box)."""
import numpy as np

from oracle.cic import cic_assign, tsc_assign, tsc_weights_1d


def test_tsc_weights_moments_and_on_node_values():
    u = np.concatenate([np.random.default_rng(0).random(500) * 64, [3.0, 3.5, 7.25, 0.0, 63.999]])
    lo, w = tsc_weights_1d(u)
    nodes = lo[:, None] + np.arange(3)[None, :]
    assert np.allclose(w.sum(1), 1.0, atol=1e-15)
    assert np.allclose((w * nodes).sum(1), u, atol=1e-12)                       # centroid
    assert np.allclose((w * (nodes - u[:, None]) ** 2).sum(1), 0.25, atol=1e-12)  # variance 3/12
    assert np.all(w >= 0)
    lo, w = tsc_weights_1d(np.array([5.0]))
    assert lo[0] == 4 and np.allclose(w[0], [0.125, 0.75, 0.125], atol=0)


def test_tsc_is_cic_averaged_over_a_unit_box_of_shifts():
    L, N = 16.0, 16
    pos = np.array([[3.3, 7.9, 12.02], [0.4, 15.7, 8.5], [5.0, 6.0, 7.0]])
    w = np.array([1.0, 0.6, 1.7])
    tsc = tsc_assign(pos, w, N, L)
    n = 40  # midpoint rule per axis on (-1/2, 1/2) cells
    t = (np.arange(n) + 0.5) / n - 0.5
    acc = np.zeros((N, N, N))
    d = L / N
    for a in t:
        for b in t:
            for c in t:
                acc += cic_assign(np.mod(pos + d * np.array([a, b, c]), L), w, N, L)
    acc /= n ** 3
    assert np.isclose(tsc.sum(), w.sum(), rtol=1e-14)
    assert np.max(np.abs(tsc - acc)) <= 1e-3 * np.max(tsc)
