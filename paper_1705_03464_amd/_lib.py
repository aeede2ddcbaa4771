"""ctypes binding of libpgx.so (the C-ABI declared in include/pgx.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device arrays are torch CUDA tensors (torch is used for device memory
and streams).  There is no CPU fallback: if the library is missing or fails to
load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpgx.so")

STATUS = {0: "PGX_OK", 1: "PGX_EINVAL", 2: "PGX_ENOSPACE", 3: "PGX_EHIP", 4: "PGX_ENOTSUP",
          5: "PGX_ESTATE"}
PAIR_MODES = {"s_mu": 0, "rp_pi": 1}
OUT_MODES = {"shell": 0, "r_mu": 1, "rp_pi": 2, "gsw": 3}
PRECISIONS = {"fp64": 0, "fp32": 1}
QEFF_MODES = {"notsq": 0, "squeezed": 1, "const": 2}
ASSIGNMENTS = {"cic": 0, "tsc": 1}


class PgxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [
        ("L", C.c_double), ("N", C.c_int32), ("precision", C.c_int32), ("pair_mode", C.c_int32),
        ("n_p1", C.c_int32), ("p1_edges", C.POINTER(C.c_double)),
        ("n_p2", C.c_int32), ("p2_edges", C.POINTER(C.c_double)),
        ("pair_dmax", C.c_double), ("out_mode", C.c_int32),
        ("n_o1", C.c_int32), ("o1_edges", C.POINTER(C.c_double)),
        ("n_o2", C.c_int32), ("o2_edges", C.POINTER(C.c_double)),
        ("qeff_mode", C.c_int32), ("xi_w_const", C.c_double), ("batch", C.c_int32),
        ("w_sigma", C.c_double), ("w_rs", C.c_double), ("w_s0", C.c_double),
        ("w_rcut", C.c_double), ("w_rmax", C.c_double),
        ("assignment", C.c_int32),
    ]


_lib = None

_SIGS = {
    "pgx_plan_create": (C.c_int, [C.POINTER(_Params), C.POINTER(C.c_void_p)]),
    "pgx_plan_destroy": (C.c_int, [C.c_void_p]),
    "pgx_plan_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32)]),
    "pgx_out_counts": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "pgx_out_norms": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pgx_field_volumes": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pgx_pairs_build": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_int64, C.c_void_p, C.POINTER(C.c_int64), C.c_void_p,
                                  C.c_void_p]),
    "pgx_pairs_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pgx_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pgx_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p]),
    "pgx_keep_spectra": (C.c_int, [C.c_void_p, C.c_int32]),
    "pgx_use_graphs": (C.c_int, [C.c_void_p, C.c_int32]),
    "pgx_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "pgx_schedule": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "pgx_dual_check": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pgx_projected": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pgx_projected_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pgx_multipoles": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "pgx_multipoles_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pgx_set_schedule": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "pgx_dual_recheck": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "pgx_graph_replays": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "pgx_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "pgx_profile_read": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_char_p),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]),
    "pgx_last_error": (C.c_char_p, [C.c_void_p]),
    "pgx_build_digest": (C.c_char_p, []),
    "pgx_workspace_bytes": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "pgx_set_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "pgx_workspace_used": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "pgx_forward_fixed": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}


def load_library(path: Optional[str] = None):
    """Load libpgx.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libpgx.so not found at {p}: build it with "
                           "`python -m paper_1705_03464_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def build_digest() -> str:
    """SHA-256 of the sources the loaded library was built from."""
    return load_library().pgx_build_digest().decode()


def _check(code: int, plan=None):
    """Raise PgxError for a non-OK status, with the plan's (or, without a
    plan, the thread's) last error message."""
    if code != 0:
        msg = load_library().pgx_last_error(plan)
        raise PgxError(code, msg.decode() if msg else "")


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensors are required")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return t.data_ptr()


def _stream(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _edges(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Plan:
    """One plan of the pair-galaxy correlation (wraps pgx_plan).  With
    out_mode "gsw" (the paper's Gaussian-sigmoid weighting function, one
    weighted output bin) `o1_edges` carries its parameters
    (sigma, r_s, s_0, r_cut, r_max) and `o2_edges` is ignored."""

    def __init__(self, L: float, N: int, p1_edges: Sequence[float], p2_edges: Sequence[float],
                 o1_edges: Sequence[float], o2_edges: Optional[Sequence[float]] = None, *,
                 precision: str = "fp32", pair_mode: str = "s_mu", out_mode: str = "shell",
                 pair_dmax: float = 0.0, qeff_mode: str = "notsq", xi_w_const: float = 0.0,
                 batch: int = 0, assignment: str = "cic"):
        lib = load_library()
        gsw = out_mode == "gsw"
        wpar = [float(v) for v in o1_edges] if gsw else [0.0] * 5
        if gsw and len(wpar) != 5:
            raise ValueError("out_mode gsw takes (sigma, r_s, s_0, r_cut, r_max)")
        self._keep = [_edges(p1_edges), _edges(p2_edges), _edges([0.0, 1.0] if gsw else o1_edges),
                      _edges(o2_edges if o2_edges is not None else [0.0, 1.0])]
        e1, e2, e3, e4 = self._keep
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        prm = _Params(float(L), int(N), PRECISIONS[precision], PAIR_MODES[pair_mode],
                      e1.size - 1, dp(e1), e2.size - 1, dp(e2), float(pair_dmax),
                      OUT_MODES[out_mode], e3.size - 1, dp(e3), e4.size - 1, dp(e4),
                      QEFF_MODES[qeff_mode], float(xi_w_const), int(batch), *wpar,
                      ASSIGNMENTS[assignment])
        h = C.c_void_p()
        _check(lib.pgx_plan_create(C.byref(prm), C.byref(h)))
        self._h = h
        self.L, self.N, self.precision = float(L), int(N), precision
        nf, no = C.c_int32(), C.c_int32()
        win = (C.c_int32 * 3)()
        _check(lib.pgx_plan_info(h, C.byref(nf), C.byref(no), win))
        self.n_fields, self.n_out, self.window = nf.value, no.value, tuple(win)
        self.n_gal = 0
        self.n_pairs = 0

    @classmethod
    def from_workload(cls, wl, precision: Optional[str] = None, batch: int = 0) -> "Plan":
        return cls(wl.L, wl.N, wl.p1_edges, wl.p2_edges, wl.o1_edges, wl.o2_edges,
                   precision=precision or wl.precision, pair_mode=wl.pair_mode,
                   out_mode=wl.out_mode, pair_dmax=wl.pair_dmax, qeff_mode=wl.qeff_mode,
                   xi_w_const=wl.xi_w_const, batch=batch,
                   assignment=getattr(wl, "assignment", "cic"))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().pgx_plan_destroy(self._h)
            self._h = None
        self._ws = None  # the workspace outlives the plan that uses it

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # host-side queries
    def out_counts(self) -> np.ndarray:
        a = np.zeros(self.n_out, np.int64)
        _check(load_library().pgx_out_counts(self._h, a.ctypes.data_as(C.POINTER(C.c_int64))), self._h)
        return a

    def out_norms(self) -> np.ndarray:
        """Denominator of xi per output bin: n_b, or sum of W for "gsw"."""
        a = np.zeros(self.n_out, np.float64)
        _check(load_library().pgx_out_norms(self._h, a.ctypes.data_as(C.POINTER(C.c_double))), self._h)
        return a

    def field_volumes(self) -> np.ndarray:
        a = np.zeros(self.n_fields, np.float64)
        _check(load_library().pgx_field_volumes(self._h, a.ctypes.data_as(C.POINTER(C.c_double))), self._h)
        return a

    # device calls
    def pairs_build(self, x, y, z, stream=None, w=None, with_wsum: bool = False):
        """Pair catalogue of the galaxies at (x, y, z) (float64 device
        tensors); returns (n_pairs, counts[F]), and the per-field pair-weight
        sums for the weights w (float32, None = unit) when with_wsum."""
        import torch
        n = int(x.shape[0])
        for t in (x, y, z):
            if t.dtype != torch.float64 or t.shape[0] != n:
                raise ValueError("positions must be float64 tensors of equal length")
        if w is not None and (w.dtype != torch.float32 or w.shape[0] != n):
            raise ValueError("weights must be a float32 tensor of length n_gal")
        counts = torch.zeros(self.n_fields, dtype=torch.int64, device=x.device)
        wsum = torch.empty(self.n_fields, dtype=torch.float64, device=x.device) if with_wsum else None
        np_ = C.c_int64()
        _check(load_library().pgx_pairs_build(self._h, _ptr(x), _ptr(y), _ptr(z), _ptr(w), n,
                                              _stream(stream), C.byref(np_), _ptr(counts),
                                              _ptr(wsum)), self._h)
        self.n_gal = n
        self.n_pairs = np_.value
        if with_wsum:
            return np_.value, counts, wsum
        return np_.value, counts

    # caller-owned workspace (device memory allocated with torch)
    def workspace_bytes(self, n_gal: int, n_pairs: int) -> int:
        """Upper bound of the plan's device memory for such a catalogue
        (pgx_workspace_bytes)."""
        b = C.c_size_t()
        _check(load_library().pgx_workspace_bytes(self._h, int(n_gal), int(n_pairs), C.byref(b)),
               self._h)
        return b.value

    def set_workspace(self, nbytes: Optional[int], device=None):
        """Place every device buffer of the plan in a torch-allocated region
        of `nbytes` bytes (None: back to the plan's own allocations).  This
        discards the plan's device state; call pairs_build next."""
        import torch
        lib = load_library()
        if nbytes is None:
            _check(lib.pgx_set_workspace(self._h, None, 0), self._h)
            self._ws = None
            return None
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        ws = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        _check(lib.pgx_set_workspace(self._h, ws.data_ptr(), ws.numel()), self._h)
        self._ws = ws  # kept alive as long as the plan uses it
        return ws

    def workspace_used(self) -> tuple:
        """(bytes in use, peak bytes) of the attached workspace."""
        a, b = C.c_size_t(), C.c_size_t()
        _check(load_library().pgx_workspace_used(self._h, C.byref(a), C.byref(b)), self._h)
        return a.value, b.value

    def pairs_export(self, stream=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        f = torch.empty(self.n_pairs, dtype=torch.int32, device=dev)
        i = torch.empty_like(f)
        j = torch.empty_like(f)
        _check(load_library().pgx_pairs_export(self._h, _ptr(f), _ptr(i), _ptr(j), _stream(stream)), self._h)
        return f, i, j

    def _outputs(self, w):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if w is not None:
            if w.dtype != torch.float32 or w.shape[0] != self.n_gal:
                raise ValueError("weights must be a float32 tensor of length n_gal")
        F, R = self.n_fields, self.n_out
        kw = dict(dtype=torch.float64, device=dev)
        return dict(wsum=torch.empty(F, **kw), xi_gg=torch.empty(R, **kw),
                    xi_pg=torch.empty(F, R, **kw), xi_dp=torch.empty(F, **kw),
                    b_pg=torch.empty(F, R, **kw), q_eff=torch.empty(F, R, **kw))

    def forward(self, w=None, stream=None) -> dict:
        out = self._outputs(w)
        _check(load_library().pgx_forward(self._h, _ptr(w), _stream(stream), _ptr(out["wsum"]),
                                          _ptr(out["xi_gg"]), _ptr(out["xi_pg"]), _ptr(out["xi_dp"]),
                                          _ptr(out["b_pg"]), _ptr(out["q_eff"])), self._h)
        self.forward_count = getattr(self, "forward_count", 0) + 1
        return out

    def forward_fixed(self, w=None, stream=None) -> dict:
        """The allocation-free forward of an FP64 plain plan (pgx_forward_fixed):
        the same outputs as forward(), its work memory in the library's fixed
        per-device scratch array."""
        out = self._outputs(w)
        _check(load_library().pgx_forward_fixed(self._h, _ptr(w), _stream(stream), _ptr(out["wsum"]),
                                                _ptr(out["xi_gg"]), _ptr(out["xi_pg"]),
                                                _ptr(out["xi_dp"]), _ptr(out["b_pg"]),
                                                _ptr(out["q_eff"])), self._h)
        return out

    def backward(self, g_b_pg=None, g_q_eff=None, g_xi_pg=None, g_xi_gg=None, g_xi_dp=None,
                 stream=None):
        """dL/dw for the last forward, given upstream gradients of the outputs."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        F, R = self.n_fields, self.n_out

        def prep(g, shape):
            if g is None:
                return None
            g = g.to(device=dev, dtype=torch.float64).contiguous()
            if tuple(g.shape) != shape:
                raise ValueError(f"upstream gradient of shape {tuple(g.shape)}, expected {shape}")
            return g
        gs = [prep(g_b_pg, (F, R)), prep(g_q_eff, (F, R)), prep(g_xi_pg, (F, R)),
              prep(g_xi_gg, (R,)), prep(g_xi_dp, (F,))]
        grad = torch.empty(self.n_gal, dtype=torch.float32, device=dev)
        _check(load_library().pgx_backward(self._h, _stream(stream), *[_ptr(g) for g in gs],
                                           _ptr(grad)), self._h)
        return grad

    def projected(self, xi_dp, stream=None):
        """Projected 2PCF w_p [n_p1] of an (r_p, |pi|) plan from xi(d_p) [F]
        (pgx_projected)."""
        import torch
        x = xi_dp.to(dtype=torch.float64).contiguous()
        out = torch.empty(len(self._keep[0]) - 1, dtype=torch.float64, device=x.device)
        _check(load_library().pgx_projected(self._h, _stream(stream), _ptr(x), _ptr(out)), self._h)
        return out

    def projected_backward(self, g_w_p, stream=None):
        """dL/dxi(d_p) [F] from dL/dw_p [n_p1] (pgx_projected_backward)."""
        import torch
        g = g_w_p.to(dtype=torch.float64).contiguous()
        out = torch.empty(self.n_fields, dtype=torch.float64, device=g.device)
        _check(load_library().pgx_projected_backward(self._h, _stream(stream), _ptr(g), _ptr(out)),
               self._h)
        return out

    def multipoles(self, lmax: int = 2, stream=None):
        """Legendre multipoles l = 0, 2, .., lmax of xi_pg in the angle between
        the pair axis and the pair-to-galaxy direction, for the weights and
        galaxy spectrum of the last forward (pgx_multipoles): FP64 tensor
        [n_fields, n_out, lmax // 2 + 1]."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        out = torch.empty(self.n_fields, self.n_out, lmax // 2 + 1, dtype=torch.float64, device=dev)
        _check(load_library().pgx_multipoles(self._h, _stream(stream), int(lmax), _ptr(out)), self._h)
        return out

    def multipoles_backward(self, g_xi_l, stream=None):
        """dL/dw for the last multipoles call given dL/dxi_l (pgx_multipoles_backward)."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        g = g_xi_l.to(device=dev, dtype=torch.float64).contiguous()
        grad = torch.empty(self.n_gal, dtype=torch.float32, device=dev)
        _check(load_library().pgx_multipoles_backward(self._h, _stream(stream), _ptr(g), _ptr(grad)), self._h)
        return grad

    def keep_spectra(self, enable: bool = True):
        """Keep the pair-field spectra of each forward for the adjoint (memory
        permitting); see pgx_keep_spectra."""
        _check(load_library().pgx_keep_spectra(self._h, 1 if enable else 0), self._h)

    def autotune(self, stream=None) -> dict:
        """Time candidate batch sizes and kernel variants on the current pair
        catalogue and keep the fastest; returns the schedule (pgx_autotune)."""
        out = (C.c_int32 * 5)()
        _check(load_library().pgx_autotune(self._h, _stream(stream), out), self._h)
        return self._sched(out)

    def schedule(self) -> dict:
        """The batch size and kernel variants in use."""
        out = (C.c_int32 * 5)()
        _check(load_library().pgx_schedule(self._h, out), self._h)
        return self._sched(out)

    def dual_check(self) -> float:
        """The dual form's xi disagreement with the per-field transforms in
        the last autotune, in units of 1e-5 max(|xi|, 1e-2); -1 if not
        measured (pgx_dual_check)."""
        d = C.c_double()
        _check(load_library().pgx_dual_check(self._h, C.byref(d)), self._h)
        return d.value

    def dual_recheck(self, fallback: bool = True, stream=None) -> float:
        """The dual form's check again on the last forward's weights; with
        `fallback`, a disagreement above 0.5 switches the plan to the
        per-field transforms.  -1 when the dual form is not in use
        (pgx_dual_recheck).  A backward needs a new forward afterwards."""
        d = C.c_double()
        _check(load_library().pgx_dual_recheck(self._h, _stream(stream), int(bool(fallback)), C.byref(d)),
               self._h)
        return d.value

    def set_schedule(self, batch: int, ypass_variant: int = 0, yinv_variant: int = 0,
                     zpass_variant: int = 0, algorithm: int = 0, stream=None):
        """Apply a schedule (pgx_set_schedule); algorithm 1 = dual form."""
        arr = (C.c_int32 * 5)(batch, ypass_variant, yinv_variant, zpass_variant, algorithm)
        _check(load_library().pgx_set_schedule(self._h, _stream(stream), arr), self._h)

    @staticmethod
    def _sched(out) -> dict:
        return dict(batch=int(out[0]), ypass_variant=int(out[1]), yinv_variant=int(out[2]),
                    zpass_variant=int(out[3]), algorithm=int(out[4]))

    def use_graphs(self, enable: bool = True):
        """Record the forward / adjoint launch sequences into HIP graphs and
        replay them (default on); see pgx_use_graphs."""
        _check(load_library().pgx_use_graphs(self._h, 1 if enable else 0), self._h)

    def graph_replays(self) -> tuple:
        """(forward, backward) graph replay counts."""
        f, b = C.c_int64(0), C.c_int64(0)
        _check(load_library().pgx_graph_replays(self._h, C.byref(f), C.byref(b)), self._h)
        return f.value, b.value

    def profile(self, enable: bool = True):
        """Start (clearing counters) or stop per-kernel event timing."""
        _check(load_library().pgx_profile(self._h, 1 if enable else 0), self._h)

    def profile_read(self) -> list:
        """[(name, launches, ms, algorithmic bytes)] for every timed kernel kind."""
        lib = load_library()
        res = []
        k = 0
        while True:
            nm = C.c_char_p(); n = C.c_int64(); ms = C.c_double(); by = C.c_double()
            code = lib.pgx_profile_read(self._h, k, C.byref(nm), C.byref(n), C.byref(ms), C.byref(by))
            if code == 1:
                break
            _check(code, self._h)
            res.append((nm.value.decode(), n.value, ms.value, by.value))
            k += 1
        return res
