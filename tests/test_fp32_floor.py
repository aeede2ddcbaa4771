"""Where the single-precision error of the transform chain comes from, on the
most clustered workload (CPU, no device).

The tiny HOD subset (40 halos of 50 candidates, 64^3, no field galaxies)
reaches xi_pg ~ 4.4 while most bins hold |xi| ~ 1e-3 - 1e-2, so the bar
1e-5 max(|xi|, 1e-2) asks for an absolute error of 1e-7, about 0.2 of one
FP32 unit of the largest value.  A model of the device's transform schedule
(tests/fp32_model.py: the same radix-8 stages, rotations, stage twiddles,
LDS exchanges and FP32 storage between passes) shows:
  * in FP32 arithmetic it misses that bar by a factor of 1.5 - 3 on this
    catalogue, as the device kernels do (by up to 2.6);
  * with FP64 arithmetic in every pass but the grids still stored in FP32
    between passes, the rounding of the stored values alone takes 0.3 - 0.9
    of the bar: no single-precision storage of the spectra holds it with a
    margin here, whatever the arithmetic;
  * with the grids stored in FP64 (the plain FP64 path) the error is far
    below it;
  * no single part of the chain carries the error: any one of them in FP64
    arithmetic leaves at least 0.9 of the bar, and FP64 arithmetic inside the
    transforms needs FP64 twiddles and an FP64 exchange between stages too.
On the production workloads (512^3, 9e5 - 2e6 galaxies) the FP32 kernels
stay within 0.03 of the bar (tests/test_gpu_autotune.py).
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from fp32_model import Precision, line_transform, per_field_chain  # noqa: E402
from oracle import bins as B  # noqa: E402
from oracle.cic import cic_assign  # noqa: E402
from oracle.pipeline import forward  # noqa: E402
from synth import get_config  # noqa: E402

F32, F64 = Precision("f32", "f32", "f32"), Precision("f64", "f64", "f64")


@pytest.mark.parametrize("N", [64, 512])
def test_model_is_a_dft(N):
    """In FP64 the model's line transform is the DFT (forward and inverse, to
    rounding); in FP32 its error is that of an FP32 FFT (~1e-7)."""
    rng = np.random.default_rng(N)
    a = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    for DIR, ref in ((-1, np.fft.fft(a, axis=-1)), (+1, np.fft.ifft(a, axis=-1) * N)):
        r, i = line_transform(a.real, a.imag, DIR, F64)
        assert np.abs(r + 1j * i - ref).max() <= 1e-14 * np.abs(ref).max()
        r, i = line_transform(a.real, a.imag, DIR, F32)
        e = np.abs(r + 1j * i - ref).max() / np.abs(ref).max()
        assert 1e-8 < e < 5e-7


def _tiny_case(weights):
    wl = get_config("cfg4tiny")
    cat = wl.catalog()
    w = None
    if weights == "random":
        w = np.random.default_rng(5).uniform(0.5, 1.5, cat.n).astype(np.float32).astype(np.float64)
    ref = forward(cat, wl, w=w)
    N, L = wl.N, wl.L
    table = B.lattice_table(wl.out_mode, wl.o1_edges, wl.o2_edges, L, N)
    R = B.n_out(wl.out_mode, wl.o1_edges, wl.o2_edges)
    pairs = ref["pairs"]
    rho_g = cic_assign(cat.positions(), np.ones(cat.n) if w is None else w, N, L) / ref["wg"]
    rho = []
    for f in range(wl.n_fields):
        sel = pairs["key"] == f
        ws = pairs["wsum"][f]
        rho.append(cic_assign(pairs["mid"][sel], pairs["w"][sel], N, L) / ws if ws > 0
                   else np.zeros((N, N, N)))
    return ref, table, R, rho_g, rho


def _worst(C, ref, table, R):
    worst = 0.0
    for f, c in enumerate(C):
        e = ref["xi_pg"][f]
        if not np.all(np.isfinite(e)):
            continue
        d = np.abs(B.bin_average(c, table, R) - e)
        worst = max(worst, float(np.max(d / (1e-5 * np.maximum(np.abs(e), 1e-2)))))
    return worst


@pytest.mark.parametrize("weights", ["unit", "random"])
def test_single_precision_storage_sets_the_floor(weights):
    ref, table, R, rho_g, rho = _tiny_case(weights)
    cur = _worst(per_field_chain(rho_g, rho, F32, F32, F32, F32), ref, table, R)
    arith64 = _worst(per_field_chain(rho_g, rho, F64, F64, F64, F64), ref, table, R)
    store64 = _worst(per_field_chain(rho_g, rho, F64, F64, F64, F64, store=np.float64), ref, table, R)
    print(f"{weights}: FP32 arithmetic {cur:.2f}, FP64 arithmetic with FP32 storage {arith64:.2f}, "
          f"FP64 storage {store64:.4f} of the 1e-5 bar")
    assert cur > 1.3
    assert 0.25 < arith64 < 1.0
    assert store64 < 1e-3


@pytest.mark.parametrize("weights", ["unit", "random"])
def test_no_single_pass_in_double_precision_reaches_the_bar(weights):
    """The error is spread over the chain: taking any one of its four parts
    (galaxy transform, pair x/y passes, z pass with the cross-power, inverse
    y/x) to FP64 arithmetic, the rest in FP32, still leaves at least 0.9 of
    the bar; FP64 arithmetic inside the transforms also needs FP64 stage
    twiddles and an FP64 exchange between stages (either one in FP32 leaves
    at least 0.8)."""
    ref, table, R, rho_g, rho = _tiny_case(weights)
    for k in range(4):
        ps = [F64 if i == k else F32 for i in range(4)]
        e = _worst(per_field_chain(rho_g, rho, *ps), ref, table, R)
        print(f"{weights}: part {k} in FP64: {e:.2f} of the bar")
        assert e > 0.9
    for p in (Precision("f64", "f32", "f64"), Precision("f64", "f64", "f32")):
        e = _worst(per_field_chain(rho_g, rho, p, p, p, p), ref, table, R)
        print(f"{weights}: FP64 arithmetic, twiddles {p.TW.__name__}, exchange {p.X.__name__}: {e:.2f}")
        assert e > 0.8
