"""Throughput of the pair-galaxy cross-correlation hot path on one MI355X.

One step = the whole path over one synthetic catalogue: pair catalogue
(validation, cell list, pair search with integer keys, bucketing), galaxy
field and spectrum, every pair field's correlation with the galaxy field,
bin sums, the finalisation (xi_gg, xi_pg, xi_dp, b_pg, Q_eff), and (default
--mode fwdbwd) the adjoint of a loss sum (b_pg - b_ref)^2 back to the galaxy
weights through the torch.autograd wrapper (for the HOD workload, on to the
HOD parameters).
Default workload: the 512^3 production case (L = 1000 Mpc/h, ~9.2e5 clustered
galaxies, 200 (s, |mu|) pair fields, 20 log r-bins over 10-80 Mpc/h).

Before the warm-up the plan's autotuner picks the batch schedule (unless
--no-autotune).  The timed region replays the recorded launch graphs (unless
--no-graphs); the same steps are then run again eagerly with HIP events
around every pass kernel for the per-kernel table.

Prints ONE JSON line.  `value` = pair fields per second over the timed steps
(forward + adjoint by default; `forward_only` gives the forward rate).
`step_hbm_frac` = algorithmic bytes of every instrumented pass kernel of a
step (the schedule in use: per-field transforms or the dual form) / step
time / 8 TB/s.  `roofline` is for the kernel with the largest share of the
profiled pass: algorithmic bytes per launch / mean launch time, both
measured in this run with HIP events on the launch stream.
Every device buffer of the plan lives in a workspace allocated with torch
(pgx_workspace_bytes, pgx_set_workspace), sized from a first pair build.
`hod` repeats the forward + adjoint measurement on the HOD workload (512^3,
2e6 weighted candidates, 20 x 20 bins, the loss carried on to the HOD
parameters), with fewer steps and no CPU baseline.
`multipoles` times pgx_multipoles (l = 0, 2 of every field in the angle
between the pair axis and the pair-to-galaxy direction) after a forward;
`fp64_plain` times the one-field-at-a-time FP64 GPU path's forward;
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(wl, cat, n_fields_sample=2):
    """Oracle timed on a bounded sample: the pair search and galaxy side in
    full, plus `n_fields_sample` pair fields; extrapolated to all fields."""
    import numpy as np
    from oracle.pairs import pairs_for
    from oracle.pipeline import galaxy_side, pair_field_xi
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    pairs = pairs_for(cat, wl)
    t1 = time.perf_counter()
    gal = galaxy_side(cat, wl)
    t2 = time.perf_counter()
    counts = pairs["counts"]
    # the most populated fields (the cost of a field grows with its pairs only
    # through the mass assignment; the transforms dominate)
    fields = list(np.argsort(counts)[::-1][:n_fields_sample])
    for f in fields:
        pair_field_xi(pairs, int(f), gal, wl)
    t3 = time.perf_counter()
    per_field = (t3 - t2) / n_fields_sample
    total = (t1 - t0) + (t2 - t1) + wl.n_fields * per_field
    return {
        "value": wl.n_fields / total,
        "unit": "pair fields/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"pair search + galaxy field in full ({t1 - t0:.1f} s + {t2 - t1:.1f} s) and "
                   f"{n_fields_sample} of {wl.n_fields} pair fields ({per_field:.1f} s each), "
                   f"extrapolated to all fields; FP64 numpy/scipy.fft with {cores} workers"),
    }


def measured_traffic(kernel, batch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE, WRITE_SIZE scaled by a plain copy), or None when the
    kernel sources or the batch size differ from the profiled run."""
    p = os.path.join(ROOT, "profiles", "hbm_traffic_cfg1_512.txt")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_1705_03464_amd import build_digest
    if d.get("sources_sha256") != build_digest() or d.get("batch") != batch:
        return None
    return d.get("bytes_per_launch", {}).get(kernel)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cfg1")
    ap.add_argument("--assignment", choices=["cic", "tsc"], default=None,
                    help="override the workload's mass assignment (the paper's TSC or CIC)")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--mode", choices=["fwd", "fwdbwd"], default="fwdbwd")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default batch schedule")
    ap.add_argument("--no-graphs", action="store_true", help="eager launches in the timed region")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true",
                    help="skip timing the one-field-at-a-time FP64 GPU path")
    ap.add_argument("--kernels", action="store_true", help="print the per-kernel table to stderr")
    ap.add_argument("--no-multipoles", action="store_true", help="skip timing pgx_multipoles")
    ap.add_argument("--no-hod", action="store_true", help="skip the HOD workload's record")
    ap.add_argument("--no-workspace", action="store_true",
                    help="let the plan allocate its own device memory")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (torch) three times; used to "
                         "scale the FETCH_SIZE / WRITE_SIZE counters of a profiler run")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1705_03464_amd import Plan, load_library
    from synth import get_config

    if a.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 4, "copies": 3}), flush=True)
        return 0
    load_library()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    from paper_1705_03464_amd import build_digest
    from paper_1705_03464_amd.build import sources_digest
    digest = build_digest()
    wl = get_config(a.config)
    if a.assignment is not None:
        wl = wl.scaled(assignment=a.assignment)
    res = measure(wl, a, a.steps, a.warmup, with_extras=True)
    rec = {
        "metric": "pair-field xi_pg cross-correlations/s at 512^3 (fwd, fwd+bwd), % HBM peak",
        "value": res["value"],
        "unit": "pair fields/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": res["config"],
        "step_hbm_frac": res["step_hbm_frac"],
        "step_gb": res["step_gb"],
        "ms_per_step_eager_profiled": res["ms_per_step_eager_profiled"],
        "roofline": res["roofline"],
        "library": {"sources_sha256": digest, "matches_tree": digest == sources_digest()},
    }
    for k in ("forward_only", "multipoles", "fp64_plain", "workspace"):
        if res.get(k) is not None:
            rec[k] = res[k]
    if not a.no_hod and a.config != "cfg4" and a.mode == "fwdbwd":
        # the HOD workload: forward + adjoint on to the HOD parameters
        hs = max(2, min(a.steps, 5))
        h = measure(get_config("cfg4"), a, hs, 1, with_extras=False)
        rec["hod"] = {k: h[k] for k in ("value", "unit", "ms_per_step", "step_hbm_frac", "step_gb",
                                         "ms_per_step_eager_profiled", "roofline", "config",
                                         "forward_only", "workspace") if h.get(k) is not None}
        rec["hod"]["steps"] = hs
    if not a.no_cpu_baseline:
        _log("[bench] timing the CPU oracle on a bounded sample ...")
        rec["cpu_baseline"] = cpu_baseline(wl, wl.catalog())
    print(json.dumps(rec), flush=True)
    return 0


def measure(wl, a, steps, warmup, with_extras):
    """Forward + adjoint (or forward) steps of one workload: autotuned
    schedule, timed graph replays, an eager profiled pass with HIP events per
    kernel, the forward-only rate; with_extras adds the multipoles and the
    FP64 plain path's forward."""
    import numpy as np
    import torch
    from paper_1705_03464_amd import Plan, hod_weights, pair_galaxy_xi
    cat = wl.catalog()
    _log(f"[bench] {wl.name}: n_gal={cat.n} N={wl.N} fields={wl.n_fields} bins={wl.n_out}")
    dev = torch.device("cuda", 0)
    x = torch.as_tensor(cat.x, dtype=torch.float64, device=dev)
    y = torch.as_tensor(cat.y, dtype=torch.float64, device=dev)
    z = torch.as_tensor(cat.z, dtype=torch.float64, device=dev)
    plan = Plan.from_workload(wl, precision="fp32", batch=a.batch)
    plan.use_graphs(not a.no_graphs)
    hod = wl.weighted
    if hod:
        from synth.configs import HOD_FIDUCIAL
        th0 = [HOD_FIDUCIAL[k] for k in ("logMcut", "logM1", "sigma", "alpha")]
        hm = torch.as_tensor(cat.halo_mass, dtype=torch.float64, device=dev)
        kind = torch.as_tensor(cat.kind.astype(np.int64), device=dev)
    ones = torch.ones(cat.n, dtype=torch.float32, device=dev)

    def weights(grad):
        if hod:
            theta = torch.tensor(th0, dtype=torch.float64, device=dev, requires_grad=grad)
            return hod_weights(theta, hm, kind)
        return ones.clone().requires_grad_(grad)

    w_step = weights(False).detach()

    def step_fwd():
        plan.keep_spectra(False)  # no adjoint follows
        plan.pairs_build(x, y, z)
        return plan.forward(w_step)

    def step_fwdbwd():
        plan.pairs_build(x, y, z)
        out = pair_galaxy_xi(plan, weights(True))
        b = out["b_pg"]
        # sum over the finite entries, without a data-dependent shape (no
        # host synchronisation inside the step)
        r = torch.where(torch.isfinite(b), b - 1.0, torch.zeros_like(b))
        loss = (r * r).sum()
        loss.backward()
        return out

    def timed(fn, n, profile=False):
        if profile:
            plan.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            out = fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = None
        if profile:
            prof = plan.profile_read()
            plan.profile(False)
        return out, (t1 - t0) * 1e3 / n, prof

    # every device buffer of the plan in a torch-allocated workspace, sized
    # for this catalogue from a first pair build
    workspace = None
    if not a.no_workspace:
        P0, _ = plan.pairs_build(x, y, z)
        plan.keep_spectra(a.mode == "fwdbwd")
        nb = plan.workspace_bytes(cat.n, P0)
        # the bound counts the optional stores (kept spectra, kernel stores),
        # which the plan makes only when they fit: cap it at what the device has
        free = torch.cuda.mem_get_info()[0]
        cap = int(free * 0.92)
        workspace = {"bytes": min(nb, cap), "bound": nb}
        plan.set_workspace(min(nb, cap))
    schedule = plan.schedule() if a.no_autotune else None
    if not a.no_autotune:
        plan.pairs_build(x, y, z)
        # the autotuner checks the dual form on the weights of the last forward:
        # run one with the step's weights first
        plan.keep_spectra(a.mode == "fwdbwd")
        plan.forward(w_step)
        t0 = time.perf_counter()
        schedule = plan.autotune()
        _log(f"[bench] autotune {time.perf_counter() - t0:.1f} s: {schedule}")
    step = step_fwdbwd if a.mode == "fwdbwd" else step_fwd
    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        _log(f"[bench] warmup {i + 1}/{warmup} done")
    # timed region: the production configuration (launch graphs replayed)
    out, ms_step, _ = timed(step, steps)
    replays = plan.graph_replays()
    _log(f"[bench] timed {steps} steps ({a.mode}): {ms_step:.2f} ms/step, n_pairs={plan.n_pairs}, "
         f"graph replays (fwd, bwd) so far {replays}")
    value = wl.n_fields / (ms_step * 1e-3)
    # the same steps again, eagerly, with HIP events around every pass kernel
    _, ms_prof, prof = timed(step, steps, profile=True)
    _log(f"[bench] profiled (eager) {steps} steps: {ms_prof:.2f} ms/step")
    fwd_only = None
    if a.mode == "fwdbwd":
        step_fwd()
        step_fwd()
        torch.cuda.synchronize()
        _, ms_f, _ = timed(step_fwd, max(2, steps))
        v_f = wl.n_fields / (ms_f * 1e-3)
        fwd_only = {"value": round(v_f, 2), "unit": "pair fields/s", "ms_per_step": round(ms_f, 3)}
        _log(f"[bench] forward only: {ms_f:.2f} ms/step")
    multipoles = None
    if with_extras and not a.no_multipoles and wl.out_mode == "shell" and float(wl.o1_edges[0]) > 0:
        step_fwd()  # the forward whose weights and galaxy spectrum it reads
        plan.multipoles(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            plan.multipoles(2)
        torch.cuda.synchronize()
        ms_m = (time.perf_counter() - t0) * 1e3 / 3
        multipoles = {"lmax": 2, "bin_kernels": wl.n_out * 6, "ms_per_call": round(ms_m, 2),
                      "value": round(wl.n_fields / (ms_m * 1e-3), 2),
                      "unit": "pair fields/s (l = 0 and 2 of every field)"}
        _log(f"[bench] multipoles (l <= 2): {ms_m:.2f} ms/call")
    if a.kernels:
        for name, n, ms, by in prof:
            _log(f"  {name:16s} launches {n:5d}  {ms / max(n, 1):8.3f} ms/launch  "
                 f"{by / max(n, 1) / 1e9:8.3f} GB/launch  {by / (ms * 1e-3) / 1e9 if ms > 0 else 0:8.1f} GB/s"
                 f"  share {ms / (ms_prof * steps):.3f}")
    step_bytes = sum(p[3] for p in prof) / steps
    # against the timed step (the launch-graph replays the value is quoted on)
    step_hbm_frac = step_bytes / (ms_step * 1e-3) / (HBM_PEAK_GBS * 1e9)
    dom = max(prof, key=lambda p: p[2])
    name, n, ms, by = dom
    achieved = (by / n) / (ms / n * 1e-3) / 1e9
    traffic = (measured_traffic(name, plan.schedule()["batch"])
               if wl.name == "cfg1" and wl.assignment == "cic" else None)
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": name,
        "bytes_per_launch": by / n, "ms_per_launch": ms / n,
        "kernel_share_of_step": round(ms / (ms_prof * steps), 3),
    }
    if workspace is not None:
        workspace["peak"] = plan.workspace_used()[1]
    finite = np.isfinite(out["xi_pg"].detach().cpu().numpy())
    res = {
        "value": round(value, 2), "unit": "pair fields/s", "ms_per_step": round(ms_step, 3),
        "config": {
            "workload": wl.description,
            "name": wl.name, "N": wl.N, "L": wl.L, "n_gal": cat.n, "n_pairs": plan.n_pairs,
            "pair_fields": wl.n_fields, "out_bins": wl.n_out, "finite_rows": int(finite.any(1).sum()),
            "step": ("pairs_build + forward + adjoint (autograd)" if a.mode == "fwdbwd"
                     else "pairs_build + forward"),
            "hod_weights": bool(hod), "assignment": wl.assignment, "parallelism": "single GPU",
            "schedule": plan.schedule(), "autotuned": not a.no_autotune,
            "dual_form_check": round(plan.dual_check(), 4),
            "launch_graphs": not a.no_graphs,
        },
        "step_hbm_frac": round(step_hbm_frac, 4),
        "step_gb": round(step_bytes / 1e9, 2),
        "ms_per_step_eager_profiled": round(ms_prof, 3),
        "roofline": roofline,
        "forward_only": fwd_only,
        "multipoles": multipoles,
        "workspace": workspace,
    }
    plan.close()
    if with_extras and not a.no_fp64_plain:
        _log("[bench] timing the one-field-at-a-time FP64 GPU path (forward) ...")
        p64 = Plan.from_workload(wl, precision="fp64")
        p64.pairs_build(x, y, z)
        p64.forward(w_step)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p64.forward(w_step)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) * 1e3
        p64.close()
        ms_fwd = fwd_only["ms_per_step"] if fwd_only else ms_step
        res["fp64_plain"] = {"ms_per_forward": round(ms64, 1),
                             "value": round(wl.n_fields / (ms64 * 1e-3), 2), "unit": "pair fields/s",
                             "speedup_fp32_batched_fwd": round(ms64 / ms_fwd, 2)}
        _log(f"[bench] FP64 plain forward: {ms64:.1f} ms")
    del x, y, z
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    sys.exit(main())
