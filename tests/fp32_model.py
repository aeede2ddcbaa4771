"""CPU model of the device's FP32 transform chain (test infrastructure).

The device transforms each grid line with a Stockham schedule: radix-8
stages (64 = 8 x 8, 512 = 8 x 8 x 8), each a twiddle multiplication by the
FP64-computed, rounded stage twiddles and an in-register DFT built from
radix-4 butterflies and constant rotations; stages exchange the line through
LDS; passes along x, y and z store their results in FP32 between them.  This
module reproduces that arithmetic with NumPy, in a chosen precision:
  arith: precision of the butterflies and twiddle products,
  tw:    precision the stage twiddles are rounded to,
  xchg:  precision of the LDS exchange between stages,
  store: precision of the grids between passes (FP32 on the device).
It models the rounding of the device's schedule; it is not the oracle (the
oracle uses scipy's FFT in FP64 and shares nothing with this file).
"""
from __future__ import annotations

import math

import numpy as np

RADICES = {64: (8, 8), 128: (8, 8, 2), 256: (8, 8, 4), 512: (8, 8, 8)}


class Precision:
    def __init__(self, arith="f32", tw="f32", xchg="f32"):
        pick = {"f32": np.float32, "f64": np.float64}
        self.A, self.TW, self.X = pick[arith], pick[tw], pick[xchg]


def _rot(R, E, DIR, vx, vy, T):
    """v * exp(DIR 2 pi i E / R) with exact quarter turns."""
    e = E % R
    if e == 0:
        return vx, vy
    if 2 * e == R:
        return -vx, -vy
    if 4 * e == R:
        return (vy, -vx) if DIR < 0 else (-vy, vx)
    if 4 * e == 3 * R:
        return (-vy, vx) if DIR < 0 else (vy, -vx)
    c = T(math.cos(2.0 * math.pi * e / R))
    s = T(DIR * math.sin(2.0 * math.pi * e / R))
    return vx * c - vy * s, vx * s + vy * c


def _bfly4(DIR, a):
    (a0x, a0y), (a1x, a1y), (a2x, a2y), (a3x, a3y) = a
    t0 = (a0x + a2x, a0y + a2y)
    t1 = (a0x - a2x, a0y - a2y)
    t2 = (a1x + a3x, a1y + a3y)
    t3 = (a1x - a3x, a1y - a3y)
    r3 = (t3[1], -t3[0]) if DIR < 0 else (-t3[1], t3[0])
    return [(t0[0] + t2[0], t0[1] + t2[1]), (t1[0] + r3[0], t1[1] + r3[1]),
            (t0[0] - t2[0], t0[1] - t2[1]), (t1[0] - r3[0], t1[1] - r3[1])]


def _dft(R, DIR, x, T):
    """In-register DFT of size R: radix-4 split of the inputs by residue,
    sub-DFTs, rotations, radix-4 butterflies (natural order in and out)."""
    if R == 1:
        return x
    if R == 2:
        (ax, ay), (bx, by) = x
        return [(ax + bx, ay + by), (ax - bx, ay - by)]
    if R == 4:
        return _bfly4(DIR, x)
    M = R // 4
    y = [_dft(M, DIR, [x[4 * m + q] for m in range(M)], T) for q in range(4)]
    out = [None] * R
    for K in range(M):
        b = _bfly4(DIR, [y[0][K], _rot(R, K, DIR, *y[1][K], T), _rot(R, 2 * K, DIR, *y[2][K], T),
                         _rot(R, 3 * K, DIR, *y[3][K], T)])
        for q in range(4):
            out[K + q * M] = b[q]
    return out


def line_transform(re, im, DIR, p: Precision):
    """Unnormalised DFT along the last axis (DIR = -1 forward, +1 inverse)."""
    N = re.shape[-1]
    T = p.A
    xr, xi = re.astype(T), im.astype(T)
    Ns = 1
    rad = RADICES[N]
    for s, R in enumerate(rad):
        J = N // R
        br = [xr[..., r * J:(r + 1) * J] for r in range(R)]
        bi = [xi[..., r * J:(r + 1) * J] for r in range(R)]
        if Ns > 1:
            k = np.arange(J) % Ns
            for r in range(1, R):
                ang = -2.0 * math.pi * r * k / (Ns * R)
                wr = np.cos(ang).astype(p.TW).astype(T)
                wi = np.sin(ang).astype(p.TW).astype(T)
                if DIR > 0:
                    wi = -wi
                a, b = br[r], bi[r]
                br[r], bi[r] = a * wr - b * wi, a * wi + b * wr
        y = _dft(R, DIR, list(zip(br, bi)), T)
        outr, outi = np.empty_like(xr), np.empty_like(xi)
        j = np.arange(J)
        base = (j // Ns) * Ns * R + (j % Ns)
        for r in range(R):
            outr[..., base + r * Ns] = y[r][0]
            outi[..., base + r * Ns] = y[r][1]
        xr, xi = outr, outi
        Ns *= R
        if s < len(rad) - 1:  # exchange through LDS
            xr, xi = xr.astype(p.X).astype(T), xi.astype(p.X).astype(T)
    return xr.astype(np.float64), xi.astype(np.float64)


def passes(re, im, DIR, p: Precision, axes, store=np.float32, store_last=True):
    """Line transforms along `axes` in order, the grid stored in `store`
    precision between passes (and after the last when store_last)."""
    for n, ax in enumerate(axes):
        r, i = line_transform(np.moveaxis(re, ax, -1), np.moveaxis(im, ax, -1), DIR, p)
        re, im = np.moveaxis(r, -1, ax), np.moveaxis(i, -1, ax)
        if n < len(axes) - 1 or store_last:
            re, im = re.astype(store).astype(np.float64), im.astype(store).astype(np.float64)
    return re, im


def per_field_chain(rho_g, rho_pairs, gal: Precision, pair_xy: Precision, zpass: Precision,
                    inv: Precision, store=np.float32):
    """The per-field evaluation as the device schedules it: the galaxy grid
    transformed (x, y, z), its k = 0 mode cleared, stored FP32; each pair of
    normalised pair fields as one complex grid: x and y passes stored FP32,
    then the z pass (forward z, times conj(G), inverse z) in registers,
    stored FP32; inverse y stored FP32; inverse x.  Returns the correlation
    grid C (unnormalised inverse DFT of Z conj(G)) of every pair field.
    `store` is the precision of the inputs and of the grids between passes
    (FP32 on the device)."""
    st = lambda a: a.astype(store).astype(np.float64)
    gr, gi = passes(st(rho_g), np.zeros_like(rho_g), -1, gal, (0, 1, 2), store=store)
    gr[0, 0, 0] = gi[0, 0, 0] = 0.0
    out = []
    for j in range(0, len(rho_pairs), 2):
        a = st(rho_pairs[j])
        b = st(rho_pairs[j + 1]) if j + 1 < len(rho_pairs) else np.zeros_like(a)
        ar, ai = passes(a, b, -1, pair_xy, (0, 1), store=store)
        ar, ai = passes(ar, ai, -1, zpass, (2,), store_last=False)
        T = zpass.A
        zr, zi = ar.astype(T), ai.astype(T)
        Gr, Gi = gr.astype(store).astype(T), gi.astype(store).astype(T)
        xr, xi = (zr * Gr + zi * Gi).astype(np.float64), (zi * Gr - zr * Gi).astype(np.float64)
        cr, ci = passes(xr, xi, +1, zpass, (2,), store=store)
        cr, ci = passes(cr, ci, +1, inv, (1, 0), store_last=False, store=store)
        out.append(cr)
        if j + 1 < len(rho_pairs):
            out.append(ci)
    return out
