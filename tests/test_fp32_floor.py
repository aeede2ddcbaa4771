"""How far a single-precision transform chain can get on the most clustered
workload (CPU, no device).

The FP32 path runs the forward transforms, the cross-power product and the
inverse transform in single precision.  On the tiny HOD subset (40 halos of
49 candidates, 64^3) xi_pg reaches ~4.5, and the rounding of FP32 transforms
then shows on every bin at about one FP32 unit of that largest value.  This
test evaluates the same estimator with scipy's single-precision FFT in place
of the oracle's double-precision one, to show that the 1e-5 relative bar is
out of reach for any FP32 chain on this catalogue while 2^-23 max|xi_pg| is
the right order for the bound the device test states.
"""
import numpy as np
import scipy.fft as sfft

from oracle import bins as B
from oracle.cic import cic_assign
from oracle.pipeline import forward
from synth import get_config


def test_single_precision_chain_floor_on_tiny_hod_subset():
    wl = get_config("cfg4tiny")
    cat = wl.catalog()
    ref = forward(cat, wl)
    N, L = wl.N, wl.L
    table = B.lattice_table(wl.out_mode, wl.o1_edges, wl.o2_edges, L, N)
    R = B.n_out(wl.out_mode, wl.o1_edges, wl.o2_edges)
    pairs = ref["pairs"]
    rho_g = cic_assign(cat.positions(), np.ones(cat.n), N, L) / ref["wg"]
    G = sfft.rfftn(rho_g.astype(np.float32))
    G[0, 0, 0] = 0
    xi_ref = ref["xi_pg"]
    peak = float(np.max(np.abs(xi_ref[np.isfinite(xi_ref)])))
    worst_rel, worst_abs = 0.0, 0.0
    for f in range(wl.n_fields):
        if not np.all(np.isfinite(xi_ref[f])):
            continue
        sel = pairs["key"] == f
        rho_f = cic_assign(pairs["mid"][sel], pairs["w"][sel], N, L) / pairs["wsum"][f]
        A = sfft.rfftn(rho_f.astype(np.float32))
        A[0, 0, 0] = 0
        assert A.dtype == np.complex64 and G.dtype == np.complex64
        C = sfft.irfftn(np.conj(A) * G, s=rho_f.shape).astype(np.float64) * rho_f.size
        xi = B.bin_average(C, table, R)
        d = np.abs(xi - xi_ref[f])
        worst_rel = max(worst_rel, float(np.max(d / (1e-5 * np.maximum(np.abs(xi_ref[f]), 1e-2)))))
        worst_abs = max(worst_abs, float(np.max(d)))
    # the 1e-5 bar is missed several times over by a plain FP32 chain ...
    print(f"FP32 chain: worst ratio to the 1e-5 bar {worst_rel:.2f}, max abs {worst_abs:.2e}, "
          f"2^-23 max|xi| {2.0 ** -23 * peak:.2e}")
    assert worst_rel > 2.0, worst_rel
    # ... and the miss is of the order of one FP32 unit of the largest |xi|
    assert 0.5 * 2.0 ** -23 * peak < worst_abs < 16 * 2.0 ** -23 * peak, (worst_abs, peak)
