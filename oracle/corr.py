"""Grid cross-correlation C(r) = N_c^-1 sum_x a(x) b(x + r) (oracle, FP64).

This is the real-space form of the paper's estimator numerator: equation
bpg_initial averages Re(conj(dg(k)) dp(k)) with a weight W(k); by Parseval
that equals sum_r W(r) C_pg(r) with the symmetric part of C (Methodology,
"Computing pair-galaxy bias").  Two independent evaluations:
  * ``fft_corr``: C = irfftn(conj(rfftn a) * rfftn b) / N_c (numpy's
    irfftn already divides by N_c once);
  * ``direct_corr``: the plain double sum over grid nodes, O(N_c^2), for
    grids of at most 32^3.
"""
from __future__ import annotations

import os

import numpy as np

try:
    import scipy.fft as _sfft
except Exception:  # pragma: no cover
    _sfft = None


def _workers():
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def rfftn(a):
    if _sfft is not None:
        return _sfft.rfftn(a, workers=_workers())
    return np.fft.rfftn(a)


def irfftn(A, shape):
    if _sfft is not None:
        return _sfft.irfftn(A, s=shape, workers=_workers())
    return np.fft.irfftn(A, s=shape)


def fft_corr(a: np.ndarray, b: np.ndarray, Fb=None) -> np.ndarray:
    """C[r] for r indexed like the grid (r_a = index, or index - N)."""
    Fa = rfftn(a)
    if Fb is None:
        Fb = rfftn(b)
    return irfftn(np.conj(Fa) * Fb, a.shape) / a.size


def direct_corr(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """O(N_c^2) definition: C[r] = mean over x of a[x] * b[(x + r) mod N]."""
    N = a.shape[0]
    out = np.zeros_like(a)
    for rx in range(N):
        bx = np.roll(b, -rx, axis=0)
        for ry in range(N):
            bxy = np.roll(bx, -ry, axis=1)
            for rz in range(N):
                out[rx, ry, rz] = np.sum(a * np.roll(bxy, -rz, axis=2))
    return out / a.size
