"""C-ABI checks that need no GPU: exported symbols, parameter validation and
the host-side tables (lattice counts n_b, pair-bin volumes) against the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import bins as OB
from oracle import finalize as OF
from paper_1705_03464_amd import Plan, PgxError, load_library
from paper_1705_03464_amd._lib import LIB_PATH
from synth import CONFIGS
from synth.configs import linbins, logbins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pgx.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB_PATH), reason="libpgx.so not built")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pgx_[a-z_]+)\s*\(", src)))


def test_option_flags_need_no_device():
    plan = Plan(100.0, 64, linbins(0.5, 10, 3), [0.0, 1.0], logbins(5.0, 45.0, 9))
    plan.keep_spectra(True)
    plan.keep_spectra(False)
    plan.use_graphs(False)
    plan.use_graphs(True)
    assert plan.dual_check() == -1.0  # no autotune has run


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB_PATH)
    syms = declared_symbols()
    assert "pgx_forward" in syms and "pgx_pairs_build" in syms
    for s in syms:
        assert hasattr(lib, s), s


@pytest.mark.parametrize("name", ["cfg0", "cfg1", "cfg2", "cfg3", "cfg4", "cfg4tiny", "cfg1w"])
def test_out_counts_and_volumes_match_oracle(name):
    wl = CONFIGS[name]
    plan = Plan.from_workload(wl)
    table = OB.lattice_table(wl.out_mode, wl.o1_edges, wl.o2_edges, wl.L, wl.N)
    assert np.array_equal(plan.out_counts(), table[2])
    norms = OB.lattice_weights(wl.out_mode, wl.o1_edges, wl.o2_edges, wl.L, wl.N, table)[1]
    assert np.allclose(plan.out_norms(), norms, rtol=1e-12, atol=0)
    dmax = wl.pair_dmax if wl.pair_mode == "rp_pi" else None
    vol = OF.field_volumes(wl.pair_mode, wl.p1_edges, wl.p2_edges, dmax)
    assert np.allclose(plan.field_volumes(), vol, rtol=1e-12, atol=0)
    assert plan.n_fields == wl.n_fields and plan.n_out == wl.n_out
    assert plan.window == OB.window(wl.out_mode, wl.o1_edges, wl.o2_edges, wl.L, wl.N)


@pytest.mark.parametrize("mode", ["shell", "r_mu", "rp_pi"])
def test_out_counts_other_modes(mode):
    L, N = 100.0, 64
    o1 = logbins(5.0, 45.0, 9) if mode != "rp_pi" else linbins(0.0, 45.0, 7)
    o2 = None if mode == "shell" else (linbins(0.0, 1.0, 5) if mode == "r_mu" else linbins(0.0, 30.0, 4))
    plan = Plan(L, N, linbins(0.5, 10, 3), [0.0, 1.0], o1, o2, out_mode=mode)
    assert np.array_equal(plan.out_counts(), OB.lattice_table(mode, o1, o2, L, N)[2])


def test_weighted_bin_parameters_are_validated():
    base = dict(L=200.0, N=64, p1_edges=linbins(0.5, 8, 3), p2_edges=[0.0, 1.0], out_mode="gsw")
    Plan(o1_edges=[15.0, 10.0, 0.8, 5.0, 60.0], **base)
    for par in ([0.0, 10.0, 0.8, 5.0, 60.0], [15.0, 10.0, -0.8, 5.0, 60.0],
                [15.0, 10.0, 0.8, 70.0, 60.0], [15.0, 10.0, 0.8, 5.0, 150.0],
                [15.0, 10.0, np.nan, 5.0, 60.0]):
        with pytest.raises(PgxError):
            Plan(o1_edges=par, **base)


def test_tsc_assignment_on_both_paths():
    base = dict(L=100.0, N=64, p1_edges=linbins(0.5, 10, 3), p2_edges=[0.0, 1.0],
                o1_edges=logbins(10, 40, 5), assignment="tsc")
    Plan(precision="fp64", **base).close()
    Plan(precision="fp32", **base).close()
    # an unknown scheme is rejected by the library
    import ctypes as C
    from paper_1705_03464_amd._lib import _Params, _edges
    e = _edges([0.5, 5.0]); o = _edges([10.0, 40.0])
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    prm = _Params(100.0, 64, 1, 0, 1, dp(e), 1, dp(_edges([0.0, 1.0])), 0.0, 0, 1, dp(o), 1, dp(o),
                  0, 0.0, 0, 0.0, 0.0, 0.0, 0.0, 0.0, 7)
    h = C.c_void_p()
    assert load_library().pgx_plan_create(C.byref(prm), C.byref(h)) == 1


def bad(**kw):
    base = dict(L=100.0, N=64, p1_edges=linbins(0.5, 10, 3), p2_edges=[0.0, 1.0],
                o1_edges=logbins(10, 40, 5))
    base.update(kw)
    with pytest.raises(PgxError) as e:
        Plan(**base)
    return e.value


def test_parameter_validation():
    assert bad(N=96).code == 4                        # not a power of two
    assert bad(N=2048).code == 4
    assert bad(L=-1.0).code == 1
    assert bad(p1_edges=[1.0, 0.5]).code == 1        # not ascending
    assert bad(p1_edges=[0.5, 40.0]).code == 1       # s_max >= L/3
    assert bad(o1_edges=[10.0, 50.0]).code == 1      # output reaches L/2
    assert bad(p2_edges=[0.0, 1.5]).code == 1        # |mu| > 1
    assert bad(pair_mode="rp_pi", pair_dmax=0.0).code == 1
    assert bad(o1_edges=[float("nan"), 3.0]).code == 1
    e = bad(p1_edges=[1.0, 1.0])
    assert "ascending" in str(e)


def test_valid_plans_touch_no_device():
    for wl in CONFIGS.values():
        p = Plan.from_workload(wl)
        p.close()


def test_workspace_bound_needs_no_device():
    """pgx_workspace_bytes is host arithmetic: it grows with the catalogue,
    covers at least the batch slots and galaxy spectrum of the FP32 path and
    the two grids of the FP64 path, and rejects negative sizes (the message
    is kept on the plan)."""
    wl = CONFIGS["cfg1"]
    p32 = Plan.from_workload(wl)
    a = p32.workspace_bytes(10 ** 6, 3 * 10 ** 6)
    b = p32.workspace_bytes(2 * 10 ** 6, 3 * 10 ** 8)
    assert b > a > (8 + 2) * 512 ** 3 * 8
    p32.keep_spectra(True)
    assert p32.workspace_bytes(10 ** 6, 3 * 10 ** 6) > a + 100 * 512 ** 3 * 8
    p64 = Plan.from_workload(wl, precision="fp64")
    assert p64.workspace_bytes(10 ** 6, 3 * 10 ** 6) > 2 * 512 ** 3 * 16
    with pytest.raises(PgxError) as e:
        p32.workspace_bytes(-1, 0)
    assert e.value.code == 1
    assert "negative" in load_library().pgx_last_error(p32._h).decode()
    p32.close(); p64.close()


def test_workspace_and_fixed_forward_argument_errors_need_no_device():
    import ctypes as C
    lib = load_library()
    p32 = Plan.from_workload(CONFIGS["cfg4tiny"])
    # a workspace must be 256-byte aligned
    assert lib.pgx_set_workspace(p32._h, C.c_void_p(0x1001), 1 << 20) == 1
    assert "aligned" in lib.pgx_last_error(p32._h).decode()
    # the allocation-free forward serves FP64 plain plans only
    code = lib.pgx_forward_fixed(p32._h, None, None, None, None, None, None, None, None)
    assert code == 4 and "FP64_PLAIN" in lib.pgx_last_error(p32._h).decode()
    # per-plan messages: a failure on one plan leaves another plan's message alone
    p2 = Plan.from_workload(CONFIGS["cfg4tiny"])
    assert lib.pgx_last_error(p2._h).decode() == ""
    p32.close(); p2.close()


def test_dual_recheck_argument_errors_need_no_device():
    import ctypes as C
    lib = load_library()
    d = C.c_double(0.0)
    assert lib.pgx_dual_recheck(None, None, 1, C.byref(d)) == 1   # EINVAL: no plan
    p = Plan.from_workload(CONFIGS["cfg4tiny"])
    assert lib.pgx_dual_recheck(p._h, None, 1, None) == 1         # EINVAL: no output
    assert "disagreement" in lib.pgx_last_error(p._h).decode()
    p.close()
