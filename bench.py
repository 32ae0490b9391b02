#!/usr/bin/env python3
"""Throughput of the gas-kinetic flux + update step on one MI355X.

Default workload: 2D shock/boundary-layer interaction, 1024 x 512 wall-stretched grid,
Mach-2 inflow, 8-degree oblique shock from the top boundary, adiabatic no-slip wall,
frozen seeded k/omega.  A step is one explicit time step of the whole path (CFL time
step, strain rate, every face flux, conservative update, residual).  The FP64 form is
the headline `value`; the FP32-flux form (flux arithmetic in FP32, everything else FP64)
is reported beside it with its error against the FP64 run, and so is the same workload
with k and omega transported by the k-omega equations instead of frozen, with
third-order MUSCL face values, with fifth-order WENO face values, and with the
multi-dimensional expansion.  The degree of
rarefaction eps_hat = tau/tau_hat (the turbulent Knudsen number) of the SBLI run is
reported as a diagnostic; the mode that puts eps_hat into the time weights is measured on a
1024^2 mixing layer (it does not stay physical on the SBLI mesh with an explicit global
step, where it leaves the shock generator's jump with almost no kinetic dissipation).

Prints one JSON line.  --gpus above 1 is refused: the benchmark measures one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 78.6    # scalar FP32 VALU at the same rate (packed FP32 is not used)
FP32_PACKED_PEAK_TFLOPS = 157.3   # the published FP32 vector peak (packed)
HBM_PEAK_GBS = 8000.0


# The GPU's clocks rise from their idle state over the first ~25 ms of sustained load
# (measured on the SBLI step: 115 us for the first step, 77 us/step after 5 ms, a steady
# 70 us/step from ~25 ms on), and fall back while the host prepares the next leg.  Each
# timed section is therefore preceded by _spin(): 40 ms of steps of a separate SBLI solve
# (kept for the run), which leaves the measured solves' own step counts untouched.
SPIN_MS = 40.0
_SPINNER = []


def _spin(ms=SPIN_MS):
    import torch

    from inputs import cases as C
    from paper_1302_2132_amd import Solver
    if not _SPINNER or _SPINNER[1] > 1500:       # a fresh solve within the stated 2000 steps
        if _SPINNER:
            _SPINNER[0].close()
        _SPINNER[:] = [Solver(C.sbli(1024, 512)), 0]
    s = _SPINNER[0]
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        s.step(40)
        _SPINNER[1] += 40
        torch.cuda.synchronize()


def _leg(case, steps, warmup, eps_field=False):
    """Clock spin-up and warm-up, then `steps` plain steps on the clock (the throughput),
    then the same number again with every launch carrying its own start/stop event pair
    (the per-kernel durations).  The state read back has advanced warmup + 2 * steps steps."""
    import torch

    from paper_1302_2132_amd import Solver, gks_kernel_times, gks_set_timing
    s = Solver(case)
    _spin()
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gks_set_timing(s.h, True)
    s.step(steps)
    kt = gks_kernel_times(s.h)
    gks_set_timing(s.h, False)
    r = s.residual()
    W = s.fields("cons")
    eps = s.fields("eps") if eps_field else None
    s.close()
    return {"seconds": t1 - t0, "kernels": kt, "res": r, "W": W, "steps_done": warmup + 2 * steps, "eps": eps}


def _stated_steps_error(c64, c32, steps):
    """The full-size workload stepped `steps` times in both forms (the configuration's stated
    run, outside any timed region): per-field error of the FP32-flux state against the FP64
    one (max |x32 - x64| / max |x64|), and the time both reached."""
    import numpy as np

    from paper_1302_2132_amd import Solver
    W, t = {}, {}
    for name, c in (("fp64", c64), ("fp32_flux", c32)):
        s = Solver(c)
        s.step(steps)
        t[name] = s.residual()["t"]
        W[name] = s.fields("cons")
        s.close()
    err = [float(np.max(np.abs(W["fp32_flux"][m] - W["fp64"][m])) / np.max(np.abs(W["fp64"][m])))
           for m in range(c64.nvar)]
    return {"steps": steps, "max_rel_err_vs_fp64_gpu_per_field": err, "time_fp64": t["fp64"],
            "time_fp32_flux": t["fp32_flux"]}


# the files that define the kernels' code (the host unit gks_lib.hip only instantiates them)
KERNEL_SOURCES = ("gks_flux.hpp", "gks_kernels.hpp", "gks_device.hpp", "gks_inst.hip", "erfc_poly.hpp")
TRAFFIC_SUMMARIES = (os.path.join(ROOT, "profiles", "k_tile2_sbli_1024x512_hbm_traffic.md"),
                     os.path.join(ROOT, "profiles", "k_tile3_isotropic_256_trace_and_traffic.md"),
                     os.path.join(ROOT, "profiles", "k_tile2_mixing_layer_1024_tauhat_trace_and_traffic.md"),
                     os.path.join(ROOT, "profiles", "k_face_isotropic_256_options_trace_and_traffic.md"))


def _profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summaries, or
    None when it was not profiled or the kernel sources have changed since its counters
    were taken."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1302_2132_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    for path in TRAFFIC_SUMMARIES:
        try:
            text = open(path).read().splitlines()
        except OSError:
            continue
        vals = dict(line.split(": ", 1) for line in text if ": " in line and not line.startswith(("|", "#")))
        v = vals.get(f"traffic_bytes_per_launch {kernel}")
        if v and vals.get("kernel_sources_sha", "").strip() == h.hexdigest()[:16]:
            return float(v)
    return None


def _roofline(case, leg, steps, flops_face, peak):
    """ALU roofline of the flux kernel: algorithmic flops of every face of the mesh, once
    (the fused 2D and 3D kernels also recompute their tiles' side faces and do the update,
    which are not counted), over that kernel's average launch duration."""
    n = case.n
    faces = (n[0] + 1) * n[1] + n[0] * (n[1] + 1) if case.dim == 2 else \
        (n[0] + 1) * n[1] * n[2] + n[0] * (n[1] + 1) * n[2] + n[0] * n[1] * (n[2] + 1)
    face_s = leg["kernels"]["face_ms"] / 1e3 / steps
    achieved = flops_face * faces / face_s / 1e12
    r = "float" if case.precision == "fp32_flux" else "double"
    # variant bits of the face kernels: 1 k-omega transport, 2 tau_hat, 4 third-order MUSCL,
    # 8 multi-dimensional expansion, 16 WENO5 face values
    recon = getattr(case, "recon", "muscl2")
    v = ((1 if getattr(case, "kw_transport", False) else 0) | (2 if getattr(case, "eps_mode", "dt") == "tauhat" else 0)
         | (4 if recon == "muscl3" else 0) | (8 if getattr(case, "multi_d", False) else 0)
         | (16 if recon == "weno5" else 0))
    # 2D: the fused tile kernel; 3D: the fused z-marching tile kernel, or the face kernel for
    # the multi-dimensional expansion and WENO5
    if case.dim == 2:
        kernel = f"k_tile2<{r},{v}>"
    else:
        kernel = f"k_tile3<{r},{v}>" if (v & (8 | 16)) == 0 else f"k_face<{r},3,64,{v}>"
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved / peak, 4), "traffic": _profiled_traffic(kernel),
           "kernel": kernel, "flops_per_face": flops_face, "faces_per_launch": faces,
           "avg_launch_us": round(face_s * 1e6, 2)}
    if r == "float":
        # the FP32-flux kernels keep their p dt parts in FP64 and issue scalar FP32 (packed FP32
        # is off), so their roof is the FP64/scalar-FP32 VALU rate; against the published packed
        # FP32 peak the fraction is frac_of_packed_fp32_peak
        out["peak_basis"] = "scalar FP32 / FP64 VALU rate (packed FP32 not used)"
        out["frac_of_packed_fp32_peak"] = round(achieved / FP32_PACKED_PEAK_TFLOPS, 4)
    return out


def _iso_leg(steps=20, warmup=3, options=True):
    """3D periodic isotropic box 256^3 (Ma_t 0.5), FP32-flux (the configuration's form) and
    FP64, with the FP32-flux error against FP64 after the same steps; with `options`, also
    the box with k-omega transport and with WENO5 face values (FP32 flux)."""
    import numpy as np

    from inputs import cases as C
    from paper_1302_2132_amd import gks_face_flops
    out = {"workload": "isotropic_256^3: 3D periodic decaying box, k0=4 spectrum, Ma_t 0.5, CFL 0.5",
           "cells": 256 ** 3}
    legs = {}
    for prec in ("fp32_flux", "fp64"):
        c = C.isotropic_box(256, precision=prec)
        leg = _leg(c, steps, warmup)
        legs[prec] = leg
        out[prec] = {"value": c.ncells * steps / leg["seconds"], "unit": "cell-updates/s",
                     "ms_per_step": leg["seconds"] * 1e3 / steps,
                     "roofline": _roofline(c, leg, steps, gks_face_flops(3, prec), FP64_PEAK_TFLOPS),
                     "kernel_ms_per_step": {k: round(v / steps, 4) for k, v in leg["kernels"].items()
                                            if k != "steps"}}
    W32, W64 = legs["fp32_flux"]["W"], legs["fp64"]["W"]
    err = [float(np.max(np.abs(W32[m] - W64[m])) / np.max(np.abs(W64[m]))) for m in range(5)]
    out["fp32_flux"]["max_rel_err_vs_fp64_gpu_per_field"] = err
    out["fp32_flux"]["after_steps"] = leg["steps_done"]
    if options:
        # the 3D options: k-omega transport (the fused kernel, the k-omega fluxes formed in
        # its update) and WENO5 face values (the face-kernel path: fluxes through HBM, a
        # separate update), FP32 flux as the box's form
        from paper_1302_2132_amd import gks_face_flops_recon, gks_kw_face_flops
        for name, opt, flops in (("kw_transport_fp32_flux", {"kw_transport": True},
                                  gks_face_flops(3, "fp32_flux") + gks_kw_face_flops()),
                                 ("weno5_fp32_flux", {"recon": "weno5"}, gks_face_flops_recon(3, "weno5"))):
            c = C.isotropic_box(256, precision="fp32_flux")
            for k, v in opt.items():
                setattr(c, k, v)
            leg = _leg(c, steps, warmup)
            out[name] = {"value": c.ncells * steps / leg["seconds"], "unit": "cell-updates/s",
                         "ms_per_step": leg["seconds"] * 1e3 / steps,
                         "vs_fused_step": (c.ncells * steps / leg["seconds"]) / out["fp32_flux"]["value"],
                         "roofline": _roofline(c, leg, steps, flops, FP64_PEAK_TFLOPS),
                         "kernel_ms_per_step": {k: round(v / steps, 4) for k, v in leg["kernels"].items()
                                                if k != "steps"}}
    return out


def _batch_leg(steps=200, count=64, check=8):
    """64 independent 2D meshes of uneven size (64^2..512^2; mixing layers and
    Galilean-shifted shock tubes), FP32-flux, `steps` steps each: the plain per-case loop
    (each solve stepped on its own, one after the other) against one batch whose
    persistent kernels walk all meshes per launch (online-autotuned shapes, one captured
    graph per step).  Both timings include every step; the autotuner's steps are real
    steps of the batch."""
    import numpy as np
    import torch

    from inputs import cases as C
    from paper_1302_2132_amd import Batch, Solver
    from paper_1302_2132_amd.autotune import autotune
    cases = C.batch_cases(count, seed=3, steps=steps, precision="fp32_flux")
    cell_updates = sum(c.ncells for c in cases) * steps
    solvers = [Solver(c) for c in cases]
    _spin()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    ref = [solvers[i].fields("cons") for i in range(check)]
    for s in solvers:
        s.close()
    del solvers
    torch.cuda.empty_cache()

    solvers = [Solver(c) for c in cases]
    b = Batch(solvers, capacity=count)
    _spin()
    t0 = time.perf_counter()
    shape, tune_steps, tune_s = autotune(b, use_cache=False)
    b.capture()
    b.step(steps - tune_steps)
    st = b.status()
    t_batch = time.perf_counter() - t0
    same = all(np.array_equal(solvers[i].fields("cons"), ref[i]) for i in range(check))
    ok_steps = bool(np.all(st["steps"] == steps))
    b.close()
    for s in solvers:
        s.close()
    return {
        "workload": f"{count} 2D meshes 64^2..512^2 (mixing layers, shifted shock tubes), FP32-flux, "
                    f"{steps} steps each (seed 3)",
        "cells": int(sum(c.ncells for c in cases)),
        "batched_value": cell_updates / t_batch, "loop_value": cell_updates / t_loop,
        "unit": "cell-updates/s", "speedup_vs_loop": t_loop / t_batch,
        "batched_s": t_batch, "loop_s": t_loop,
        "autotune": {"shape": shape, "steps": tune_steps, "seconds": tune_s},
        "all_members_stepped": ok_steps, "bitwise_equal_to_loop_first_%d" % check: same,
    }


def _serve_leg(reduced=False):
    """Poisson-arrival stream of solves (seeded, mean 20 req/s) mixing 2D mixing layers
    (FP64), shock/boundary-layer interactions (N x N/2, FP32-flux) and 3D isotropic boxes
    (FP32-flux); each runs to a residual fall of 1e-6 or its step cap.  Continuous
    batching (smallest expected work first) against the FIFO one-solve-at-a-time loop on
    the same trace.  The default is the stated trace (256 requests, 2D 128^2..1024^2, 3D
    64^3..128^3, 5000-step cap); --serve-reduced runs a smaller one (48 requests, 2D
    128^2..512^2, 3D 32^3..64^3, 2000 steps) that also offers more than one GPU serves."""
    from inputs import cases as C
    from paper_1302_2132_amd.serve import run_batched, run_fifo
    if not reduced:
        reqs = C.serve_trace(256, seed=4, rate=20.0)
        desc = "256 requests, 20 req/s, 2D 128^2..1024^2 (SBLI N x N/2), 3D 64^3..128^3, tol 1e-6 or 5000 steps"
    else:
        reqs = C.serve_trace(48, seed=4, rate=20.0, n2d=(128, 512), n3d=(32, 64), max_steps=2000)
        desc = "48 requests, 20 req/s, 2D 128^2..512^2 (SBLI N x N/2), 3D 32^3..64^3, tol 1e-6 or 2000 steps"
    # a request arrives with its initial state: build every payload before the clock starts
    payload = {r["id"]: C.request_case(r) for r in reqs}
    make = lambda r: payload[r["id"]]   # noqa: E731

    def log(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    shortest, _ = run_batched(reqs, make, quantum=20, log=log, order="shortest")
    fifo, _ = run_fifo(reqs, make, quantum=20, log=log)
    return {"trace": desc + " (seed 4; payloads built before the clock starts)",
            "batched_shortest_first": shortest, "fifo_loop": fifo,
            "p50_ratio_fifo_over_batched": fifo["p50_latency_s"] / shortest["p50_latency_s"],
            "p99_ratio_fifo_over_batched": fifo["p99_latency_s"] / shortest["p99_latency_s"],
            "throughput_ratio_batched_over_fifo": shortest["cell_updates_per_s"] / fifo["cell_updates_per_s"]}


def _cpu_baseline(case, target_s=15.0):
    """The oracle timed on the host's cores over a bounded sample of the workload; the state
    it reaches also checks the GPU's FP64 and FP32-flux solves run for the same steps from
    the same initial state (per field, max |gpu - oracle| / max |oracle|)."""
    import numpy as np

    import oracle
    from paper_1302_2132_amd import Solver
    threads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16), 16)
    t0 = time.perf_counter()
    r = oracle.run(case, 1, nthreads=threads)
    t1 = time.perf_counter()
    one = t1 - t0
    more = max(0, min(20, int(target_s / max(one, 1e-3)) - 1))
    if more:
        t2 = time.perf_counter()
        r = oracle.run(case, more, nthreads=threads, W=r["W"], t0=r["t"])
        t3 = time.perf_counter()
        total, steps = one + (t3 - t2), 1 + more
    else:
        total, steps = one, 1
    check = {"after_steps": steps}
    for prec in ("fp64", "fp32_flux"):
        c = case.copy()
        c.precision = prec
        s = Solver(c)
        s.step(steps)
        W = s.fields("cons")
        s.close()
        check[f"{prec}_max_rel_err_vs_oracle_per_field"] = [
            float(np.max(np.abs(W[m] - r["W"][m])) / np.max(np.abs(r["W"][m]))) for m in range(case.nvar)]
    # the oracle's own operation count of one face flux (its counting build), beside the
    # kernel's count of its closed form that the rooflines use
    from paper_1302_2132_amd import gks_face_flops
    ops = {}
    for dim in (2, 3):
        nv = dim + 2
        st = np.array([1.0, 0.3, -0.1, 0.05, 2.3][:nv - 1] + [2.3])
        sl = np.linspace(0.5, -0.5, nv)
        cnt, _ = oracle.face_op_counts(dim, st, st * 1.01, sl, -sl, st, st * 1.02, 0.005, 0.005, 1e-3, 10.0, 5.0,
                                       3e-3, mu=1e-3, c_a=0.1)
        ops[f"{dim}d"] = {"oracle_ops_per_face": cnt, "oracle_total": sum(cnt.values()),
                          "kernel_flops_per_face": gks_face_flops(dim)}
    return {"value": case.ncells * steps / total, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} FP64 steps of the full {case.n[0]}x{case.n[1]} workload "
                      f"({total:.1f} s, OpenMP over faces/cells)",
            "gpu_vs_oracle": check, "face_operation_counts": ops}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-flux leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D isotropic-box leg")
    ap.add_argument("--no-kw", action="store_true", help="skip the k-omega transport leg")
    ap.add_argument("--no-tauhat", action="store_true", help="skip the tau_hat rarefaction leg")
    ap.add_argument("--no-muscl3", action="store_true", help="skip the third-order MUSCL leg")
    ap.add_argument("--no-multid", action="store_true", help="skip the multi-dimensional expansion leg")
    ap.add_argument("--no-weno5", action="store_true", help="skip the WENO5 leg")
    ap.add_argument("--serve-reduced", action="store_true", help="served leg on a reduced 48-request trace")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (3 times), to calibrate "
                         "the HBM byte counters of a profiler against a known traffic")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "repeats": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(sharding a solve over several GPUs is designed, not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from inputs import cases as C
    from paper_1302_2132_amd import gks_face_flops, gks_face_flops_multid, gks_face_flops_recon, gks_kw_face_flops
    assert torch.cuda.is_available(), "bench.py needs a HIP device"

    case = C.sbli(1024, 512)
    K, Wm = args.steps, args.warmup
    leg64 = _leg(case, K, Wm, eps_field=True)
    value = case.ncells * K / leg64["seconds"]
    flops2d = gks_face_flops(2, "fp64")
    out = {
        "metric": "cell-updates/s FP64 vs FP32-flux at stated err; p50/p99 served solve latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1, "steps": K, "warmup": Wm, "clock_spinup_ms_before_warmup": SPIN_MS,
        "ms_per_step": leg64["seconds"] * 1e3 / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "sbli_1024x512: 2D Mach-2 shock/boundary-layer interaction, "
                               "8-deg oblique shock, adiabatic no-slip wall, tanh wall-stretched y, "
                               "frozen seeded k/omega, CFL 0.5",
                   "cells": case.ncells, "precision": "fp64"},
        "roofline": _roofline(case, leg64, K, flops2d, FP64_PEAK_TFLOPS),
        "kernel_ms_per_step": {k: round(v / K, 4) for k, v in leg64["kernels"].items() if k != "steps"},
        "eps_hat_diagnostic": {"after_steps": leg64["steps_done"], "max": float(leg64["eps"].max()),
                               "p99": float(np.percentile(leg64["eps"], 99)),
                               "p50": float(np.percentile(leg64["eps"], 50))},
    }
    if not args.no_fp32:
        c32 = C.sbli(1024, 512, precision="fp32_flux")
        leg32 = _leg(c32, K, Wm)
        err = []
        for m in range(case.nvar):
            ref = leg64["W"][m]
            err.append(float(np.max(np.abs(leg32["W"][m] - ref)) / np.max(np.abs(ref))))
        out["fp32_flux"] = {
            "value": c32.ncells * K / leg32["seconds"], "unit": "cell-updates/s",
            "ms_per_step": leg32["seconds"] * 1e3 / K,
            "max_rel_err_vs_fp64_gpu_per_field": err, "after_steps": leg32["steps_done"],
            "roofline": _roofline(c32, leg32, K, flops2d, FP32_PEAK_TFLOPS),
            "kernel_ms_per_step": {k: round(v / K, 4) for k, v in leg32["kernels"].items() if k != "steps"},
            "at_stated_steps": _stated_steps_error(case, c32, 2000),
        }
    if not args.no_kw:
        ckw = C.sbli(1024, 512)
        ckw.kw_transport = True
        legkw = _leg(ckw, K, Wm)
        vkw = ckw.ncells * K / legkw["seconds"]
        out["kw_transport"] = {
            "workload": "sbli_1024x512 as above, k and omega transported (2006 k-omega model), FP64",
            "value": vkw, "unit": "cell-updates/s", "ms_per_step": legkw["seconds"] * 1e3 / K,
            "vs_frozen": vkw / value,
            "roofline": _roofline(ckw, legkw, K, flops2d + gks_kw_face_flops(), FP64_PEAK_TFLOPS),
            "kernel_ms_per_step": {k: round(v / K, 4) for k, v in legkw["kernels"].items() if k != "steps"},
        }
    if not args.no_muscl3:
        c3 = C.sbli(1024, 512)
        c3.recon = "muscl3"
        leg3 = _leg(c3, K, Wm)
        v3 = c3.ncells * K / leg3["seconds"]
        out["muscl3"] = {
            "workload": "sbli_1024x512 as above with third-order MUSCL face values (limited kappa = 1/3), FP64",
            "value": v3, "unit": "cell-updates/s", "ms_per_step": leg3["seconds"] * 1e3 / K,
            "vs_muscl2": v3 / value,
            "roofline": _roofline(c3, leg3, K, gks_face_flops_recon(2, "muscl3"), FP64_PEAK_TFLOPS),
            "kernel_ms_per_step": {k: round(v / K, 4) for k, v in leg3["kernels"].items() if k != "steps"},
        }
    if not args.no_weno5:
        c5 = C.sbli(1024, 512)
        c5.recon = "weno5"
        leg5 = _leg(c5, K, Wm)
        v5 = c5.ncells * K / leg5["seconds"]
        out["weno5"] = {
            "workload": "sbli_1024x512 as above with fifth-order WENO face values (index space), FP64",
            "value": v5, "unit": "cell-updates/s", "ms_per_step": leg5["seconds"] * 1e3 / K,
            "vs_muscl2": v5 / value,
            "roofline": _roofline(c5, leg5, K, gks_face_flops_recon(2, "weno5"), FP64_PEAK_TFLOPS),
            "kernel_ms_per_step": {k: round(v / K, 4) for k, v in leg5["kernels"].items() if k != "steps"},
        }
    if not args.no_multid:
        cmd = C.sbli(1024, 512)
        cmd.multi_d = True
        legmd = _leg(cmd, K, Wm)
        vmd = cmd.ncells * K / legmd["seconds"]
        out["multi_d"] = {
            "workload": "sbli_1024x512 as above with the multi-dimensional expansion (tangential slopes), FP64",
            "value": vmd, "unit": "cell-updates/s", "ms_per_step": legmd["seconds"] * 1e3 / K,
            "vs_1d_expansion": vmd / value,
            "roofline": _roofline(cmd, legmd, K, gks_face_flops_multid(2), FP64_PEAK_TFLOPS),
            "kernel_ms_per_step": {k: round(v / K, 4) for k, v in legmd["kernels"].items() if k != "steps"},
        }
    if not args.no_tauhat:
        legs = {}
        for mode in ("dt", "tauhat"):
            cm = C.mixing_layer(1024, seed=3)
            cm.eps_mode = mode
            legs[mode] = (cm, _leg(cm, K, Wm, eps_field=True))
        cth, legth = legs["tauhat"]
        vth = cth.ncells * K / legth["seconds"]
        vdt = cth.ncells * K / legs["dt"][1]["seconds"]
        e = legth["eps"]
        out["tauhat"] = {
            "workload": "mixing_layer_1024x1024 (periodic double shear layer, Ma 0.3), FP64, rarefaction "
                        "eps = tau/tau_hat (tau_hat = rho/|D rho|) against eps = tau/dt on the same workload",
            "value": vth, "unit": "cell-updates/s", "ms_per_step": legth["seconds"] * 1e3 / K,
            "dt_mode_value": vdt, "vs_dt_mode": vth / vdt,
            "roofline": _roofline(cth, legth, K, flops2d, FP64_PEAK_TFLOPS),
            "kernel_ms_per_step": {k: round(v / K, 4) for k, v in legth["kernels"].items() if k != "steps"},
            "eps_hat_after_steps": legth["steps_done"], "eps_hat_max": float(e.max()),
            "eps_hat_p99": float(np.percentile(e, 99)),
        }
    if not args.no_3d:
        out["isotropic_3d"] = _iso_leg()
    if not args.no_batch:
        out["batched"] = _batch_leg()
    if not args.no_serve:
        out["served"] = _serve_leg(args.serve_reduced)
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
