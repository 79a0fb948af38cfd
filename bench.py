#!/usr/bin/env python3
"""Throughput benchmark of the spectral Gaussian-random-field hot path on one MI355X.

A step is one pass of the hot path over the 3-D workload (256^3 cells, spacing 1 m,
exponential covariance ell=(16,16,4), sigma^2=4, N=4096 modes): FP64-reduced per-axis
phase tables, the matrix-core separable contraction, and the fused log-normal epilogue
writing K.  The metric is mode-cell evaluations per second; the plain FP32 direct
sum on the same workload is timed beside it, and every variant's error against the FP64
oracle is measured on sampled cells by the CPU-baseline leg.

Prints ONE JSON line.  Inputs are synthetic and already resident in HBM when the timed
region starts; mode tables come from the library's sampler (host), outside the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import tempfile
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "mode·cell evals/s: FP32 direct sum vs MFMA separable at rel-RMS≤1e-3"
HBM_PEAK = 8.0e12            # B/s
MFMA_F16_PEAK = 2.5e15       # dense fp16/bf16 flop/s
# ALU roofline of the direct sums: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 3.93e13 lane-ops/s;
# v_cos_f32 issues at half rate on gfx950 and every mode-point needs one cosine; on grids every
# mode-cell is two full-rate FMAs (the angle sum of the x and (y,z) phases): the same peak.
COS_PEAK = 256 * 4 * 16 * 2.4e9 / 2.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def field_errors(np, y, ref, sigma):
    """rel-RMS and max |dY| / sigma of a sample against the FP64 oracle."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return {"rel_rms": float(np.sqrt(np.mean((y - ref) ** 2) / np.mean(ref ** 2))),
            "max_abs_over_sigma": float(np.max(np.abs(y - ref)) / sigma), "samples": int(y.size)}


def indicator_errors(np, ind, ref, thresholds, band, sigma):
    """Facies indices against the oracle's: mismatches outside the stated error band of the
    thresholds (must be 0) and the number of samples inside the band (band in units of Y)."""
    thr = np.atleast_1d(np.asarray(thresholds, dtype=np.float64))
    want = (ref[:, None] > thr[None, :]).sum(axis=1)
    near = np.any(np.abs(ref[:, None] - thr[None, :]) <= band, axis=1)
    return {"mismatch_outside_band": int(np.count_nonzero((np.asarray(ind) != want) & ~near)),
            "in_band": int(np.count_nonzero(near)), "band_over_sigma": band / sigma, "samples": int(len(ref))}


def grad_errors(np, got, ref):
    """rel-L2 of each gradient block against the oracle's exact gradients."""
    out = {}
    for k in ("dphi", "dk", "dsigma", "dell"):
        a = np.asarray(got[k].detach().cpu().numpy() if hasattr(got[k], "detach") else got[k], np.float64).ravel()
        b = np.atleast_1d(np.asarray(ref[k], np.float64)).ravel()
        out[k] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    return out


# Error bands (x sigma) each path states before any run: the indicator tolerance.
BAND = {"direct_f32": 1e-4, "direct_f64": 1e-6, "sep_f16": 1e-2, "sep_bf16": 5e-2, "sep_f16_x3": 2e-4,
        "sep_bf16_x3": 4e-4}


def sha(path: Path) -> str:
    return hashlib.sha256(path.read_bytes()).hexdigest()[:16]


def read_traffic(name: str, kernel_src: Path):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if still current."""
    p = ROOT / "profiles" / f"traffic_{name}.txt"
    if not p.exists():
        return None
    kv = {}
    for line in p.read_text().splitlines():
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != sha(kernel_src):  # counters taken on another version of the kernel
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline (oracle) leg")
    ap.add_argument("--no-extras", action="store_true", help="only the headline workload")
    ap.add_argument("--only", default=None, help="time a single grid method (profiling runs)")
    ap.add_argument("--extras", default="grid2d,points,epilogue,adjoint,pluri,krige,batch,probe",
                    help="comma-separated extra workloads to time (grid2d, points, epilogue, adjoint, pluri, "
                         "krige, batch, probe)")
    ap.add_argument("--extras-only", action="store_true", help="skip the headline workload (profiling runs)")
    ap.add_argument("--spinup-ms", type=float, default=500.0,
                    help="untimed GPU work before the first timed loop (steady clocks)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy (for scaling PMC byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build targets one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by cells or instances, with no exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2212_10961_amd.grf as grf
    from paper_2212_10961_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4}))
        return

    if args.extras_only:
        print(json.dumps({"extras": extras(args, grf, wl, torch, np, dev)}))
        return

    cfg = wl.WORKLOADS["grid3d_256_exp"]
    sigma = math.sqrt(cfg["sigma2"])
    shape = cfg["shape"]
    C = int(np.prod(shape))
    N = cfg["n_modes"]
    z, phi = grf.make_modes(cfg["dim"], cfg["cov"], N, cfg["seed"])
    modes = grf.modes_from_tables(z, phi, sigma, cfg["ell"], device=dev)

    methods = ["sep_f16", "sep_f16_x3", "sep_bf16_x3", "sep_bf16", "direct_f32"]
    if args.only:
        methods = [args.only]
    bufs = {}
    for m in methods:
        ws = torch.empty(grf.grid_workspace_bytes(modes, shape, m), dtype=torch.uint8, device=dev)
        out = {"k": torch.empty(C, dtype=torch.float32, device=dev)}
        bufs[m] = (ws, out)

    def step(m):
        # one pass of the path: tables, sum and the log-normal epilogue writing K (FP32)
        ws, out = bufs[m]
        grf.field_grid(modes, shape, method=m, mu=cfg["mu"], want_y=False, want_k=True, out=out, workspace=ws)

    # Bring the GPU to a steady clock before anything is timed (untimed).
    t_end = time.perf_counter() + args.spinup_ms * 1e-3
    while time.perf_counter() < t_end:
        for _ in range(10):
            step(methods[0])
        torch.cuda.synchronize()

    results = {}
    for m in methods:
        steps = args.steps if m.startswith("sep") else max(3, min(args.steps, 10))
        warm = args.warmup if m.startswith("sep") else min(args.warmup, 2)
        log(f"[bench] {m}: warmup {warm}, steps {steps}")
        for _ in range(warm):
            step(m)
        torch.cuda.synchronize()
        with grf.KernelTimer() as kt:
            t0 = time.perf_counter()
            for _ in range(steps):
                step(m)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        kms, nl = kt.read()
        ms = (t1 - t0) * 1e3 / steps
        results[m] = {"ms_per_step": ms, "kernel_ms": kms / max(nl, 1), "launches": nl, "steps": steps,
                      "mode_cells_per_s": N * C / (ms * 1e-3), "warmup": warm}
        log(f"[bench] {m}: {ms:.3f} ms/step, main kernel {kms / max(nl, 1):.3f} ms")

    # ------------------------------------------------------------ CPU baseline (oracle) + errors
    cpu = None
    errs = {}
    if not args.no_cpu:
        import oracle
        threads = oracle.threads()
        probe = wl.sample_cells(C, 4096, 4242)
        t0 = time.perf_counter()
        oracle.field_cells(z, phi, sigma, cfg["ell"], shape, probe)
        dt = time.perf_counter() - t0
        rate = probe.size * N / max(dt, 1e-9)
        m_cells = int(min(max(12.0 * rate / N, 1024), 4_000_000))  # ~12 s of oracle work
        cells = wl.sample_cells(C, m_cells, 4243)
        log(f"[bench] cpu_baseline: oracle on {cells.size} sampled cells x {N} modes, {threads} threads")
        t0 = time.perf_counter()
        ref = oracle.field_cells(z, phi, sigma, cfg["ell"], shape, cells)
        dt = time.perf_counter() - t0
        cpu = {"value": cells.size * N / dt, "unit": "mode·cell/s", "cores": threads, "kind": "oracle",
               "sample": f"{cells.size} seeded random cells of the 256^3 grid x {N} modes (FP64 direct sum), "
                         f"{dt:.1f} s", "cpu_model": cpu_model()}
        # the same oracle on one thread (a smaller sample of ~3 s)
        oracle.set_threads(1)
        one = wl.sample_cells(C, int(min(max(3.0 * rate / threads / N, 256), 200_000)), 4244)
        t0 = time.perf_counter()
        oracle.field_cells(z, phi, sigma, cfg["ell"], shape, one)
        dt1 = time.perf_counter() - t0
        oracle.set_threads(threads)
        cpu["one_thread"] = {"value": one.size * N / dt1, "unit": "mode·cell/s",
                             "sample": f"{one.size} seeded random cells x {N} modes, {dt1:.1f} s"}
        idx = torch.from_numpy(cells).to(dev)
        kref = oracle.lognormal(ref, cfg["mu"])
        for m in methods:
            ws, out = bufs[m]
            # Y for the error check from one more (untimed) evaluation of the same method
            yfull = grf.field_grid(modes, shape, method=m, mu=cfg["mu"], workspace=ws)["y"]
            y = yfull[idx].double().cpu().numpy()
            k = out["k"][idx].double().cpu().numpy()
            del yfull
            rel = float(np.sqrt(np.mean((y - ref) ** 2) / np.mean(ref ** 2)))
            errs[m] = {"rel_rms": rel, "max_abs_over_sigma": float(np.max(np.abs(y - ref)) / sigma),
                       "k_max_rel": float(np.max(np.abs(k - kref) / kref)), "cells": int(cells.size)}
            results[m].update(errs[m])
            log(f"[bench] {m}: rel_rms {rel:.2e}")

    # ------------------------------------------------------------ headline: best variant at rel-RMS <= 1e-3
    # Without a measured error, only forms whose error bound is below the bar qualify
    # (the one-pass bf16 form has rel-RMS ~2e-3 and never does).
    ok = [m for m in methods if m.startswith("sep") and
          (errs[m]["rel_rms"] <= 1e-3 if m in errs else m != "sep_bf16")]
    head = min(ok, key=lambda m: results[m]["ms_per_step"]) if ok else methods[0]
    r = results[head]
    passes = 3 if head.endswith("x3") else 1
    flops = 4.0 * N * C * passes if head.startswith("sep") else None
    src = ROOT / "paper_2212_10961_amd" / "csrc" / ("sep.hip" if head.startswith("sep") else "direct.hip")
    if flops:
        achieved = flops / (r["kernel_ms"] * 1e-3)
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": MFMA_F16_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": achieved / MFMA_F16_PEAK, "traffic": read_traffic(f"{head}_grid3d_256_exp", src),
                "kernel": f"k_sep ({head})", "kernel_ms": r["kernel_ms"],
                "algorithmic": f"4 flop per mode-cell per pass x {N} modes x {C} cells x {passes} pass"}
    else:
        achieved = N * C / (r["kernel_ms"] * 1e-3)
        roof = {"bound": "alu", "achieved": achieved, "peak": COS_PEAK, "unit": "mode·cell/s",
                "frac": achieved / COS_PEAK, "traffic": None, "kernel": "k_direct_grid", "kernel_ms": r["kernel_ms"]}

    line = {
        "metric": METRIC, "value": r["mode_cells_per_s"], "unit": "mode·cell/s", "n_gpus": 1,
        "steps": r["steps"], "warmup": r["warmup"], "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"sep_f16": "f16", "sep_bf16": "bf16", "sep_f16_x3": "f16x3", "sep_bf16_x3": "bf16x3",
                  "direct_f32": "f32"}.get(head, head),
        "data": "synthetic",
        "config": {"workload": "grid3d_256_exp", "grid": list(shape), "spacing_m": 1.0, "cov": "exponential",
                   "ell": list(cfg["ell"]), "sigma2": cfg["sigma2"], "n_modes": N, "seed": cfg["seed"],
                   "method": head, "outputs": "K=exp(mu+Y), fp32 (Y for the error check from an untimed call)",
                   "step": "per-axis FP64 phase tables + separable contraction + fused epilogue"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": {m: {k: v for k, v in results[m].items()} for m in methods},
    }
    if "direct_f32" in results:
        d = results["direct_f32"]
        line["direct_f32"] = {"mode_cells_per_s": d["mode_cells_per_s"], "ms_per_step": d["ms_per_step"],
                              "roofline": {"bound": "alu", "achieved": N * C / (d["kernel_ms"] * 1e-3),
                                           "peak": COS_PEAK, "unit": "mode·cell/s",
                                           "frac": N * C / (d["kernel_ms"] * 1e-3) / COS_PEAK},
                              "speedup_of_headline": d["ms_per_step"] / r["ms_per_step"]}

    if not args.no_extras and not args.only:
        line["extras"] = extras(args, grf, wl, torch, np, dev)
    print(json.dumps(line))


def _timed(torch, grf, fn, steps, warm):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    with grf.KernelTimer() as kt:
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    kms, nl = kt.read()
    return (t1 - t0) * 1e3 / steps, kms / max(nl, 1)


def extras(args, grf, wl, torch, np, dev):
    sel = set(s.strip() for s in args.extras.split(",") if s.strip())
    err = not args.no_cpu  # errors against the FP64 oracle (CPU) beside each leg's timing
    out = {}
    if "grid2d" in sel:
        out.update(grid2d_extra(grf, wl, torch, np, dev, err))
    if "points" in sel:
        out.update(points_extra(grf, wl, torch, np, dev, err))
    if "epilogue" in sel:
        out.update(epilogue_extra(grf, wl, torch, np, dev))
    if "adjoint" in sel:
        out.update(adjoint_extra(grf, wl, torch, np, dev, err))
    if "pluri" in sel:
        out.update(pluri_extra(grf, wl, torch, np, dev))
    if "krige" in sel:
        out.update(krige_extra(grf, wl, torch, np, dev))
    if "batch" in sel:
        try:
            out["batch512_2d"] = batch_extra(grf, wl, torch, np, dev, err)
        except grf.GrfError as e:
            out["batch512_2d"] = {"error": str(e)}
    if "probe" in sel:
        out["cos_rate_probe"] = cos_probe(torch, dev)
    return out


def cos_probe(torch, dev):
    """Measured issue rate of the hardware cosine in a register loop (alone, and in the point
    sum's per-term mix), beside the nominal half-rate peak used for the direct-sum rooflines."""
    import ctypes
    lib = ctypes.CDLL(str(ROOT / "paper_2212_10961_amd" / "libgrf_probe.so"))
    lib.grf_probe_cos_rates.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    blocks = 256 * 8
    buf = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    a, b = ctypes.c_double(), ctypes.c_double()
    torch.cuda.synchronize()
    rc = lib.grf_probe_cos_rates(ctypes.c_void_p(buf.data_ptr()), blocks, 4096, 5, ctypes.byref(a), ctypes.byref(b))
    if rc != 0:
        return {"error": rc}
    return {"cos_per_s": a.value, "cos_mix_terms_per_s": b.value, "nominal_peak": COS_PEAK,
            "cos_frac_of_nominal": a.value / COS_PEAK, "mix_frac_of_nominal": b.value / COS_PEAK,
            "probe": f"{blocks} blocks x 256 lanes x 4096 iterations x 8 chains, best of 5",
            "mix": "acc = fma(w, cos(x + acc q), acc): one cosine, one FMA and one multiply-add per term"}


def grid2d_extra(grf, wl, torch, np, dev, err):
    """The plain FP64 method on the 64x64 Gaussian workload (N = 1000), beside the FP32 direct
    sum: launch-latency-bound, reported in microseconds with the errors of both."""
    c = wl.WORKLOADS["grid2d_64_gauss"]
    log("[bench] extras: grid2d_64_gauss")
    sg = math.sqrt(c["sigma2"])
    z, phi = grf.make_modes(2, c["cov"], c["n_modes"], c["seed"])
    m = grf.modes_from_tables(z, phi, sg, c["ell"], device=dev)
    shape = c["shape"]
    C = int(np.prod(shape))
    f64 = grf.field_grid_f64(m, shape, mu=c["mu"])
    ms64, k64 = _timed(torch, grf, lambda: grf.field_grid_f64(m, shape, mu=c["mu"]), 50, 5)
    ws = torch.empty(grf.grid_workspace_bytes(m, shape, "direct_f32"), dtype=torch.uint8, device=dev)
    o32 = {"y": torch.empty(C, device=dev), "k": torch.empty(C, device=dev)}
    ms32, k32 = _timed(torch, grf, lambda: grf.field_grid(m, shape, method="direct_f32", mu=c["mu"], want_k=True,
                                                          out=o32, workspace=ws), 50, 5)
    res = {"cells": C, "n_modes": c["n_modes"], "mode_cells": C * c["n_modes"],
           "direct_f64": {"us_per_call": ms64 * 1e3, "kernel_us": k64 * 1e3},
           "direct_f32": {"us_per_call": ms32 * 1e3, "kernel_us": k32 * 1e3}}
    if err:
        import oracle
        ref = oracle.field_grid(z, phi, sg, c["ell"], shape)
        kref = oracle.lognormal(ref, c["mu"])
        y64 = f64["y"].cpu().numpy()
        res["direct_f64"].update(field_errors(np, y64, ref, sg))
        res["direct_f64"]["k_max_rel"] = float(np.max(np.abs(f64["k"].cpu().numpy() - kref) / kref))
        res["direct_f32"].update(field_errors(np, o32["y"].double().cpu().numpy(), ref, sg))
        res["direct_f32"]["k_max_rel"] = float(np.max(np.abs(o32["k"].double().cpu().numpy() - kref) / kref))
    return {"grid2d_64_gauss": res}


def points_extra(grf, wl, torch, np, dev, err=False):
    out = {}
    # unstructured points, FP64 phase reduction per mode and point, indicator epilogue
    c = wl.WORKLOADS["points_2m_gauss"]
    log("[bench] extras: points_2m_gauss")
    z, phi = grf.make_modes(3, c["cov"], c["n_modes"], c["seed"])
    m = grf.modes_from_tables(z, phi, math.sqrt(c["sigma2"]), c["ell"], device=dev)
    x = torch.from_numpy(wl.points_uniform(c["n_points"], c["box"], c["point_seed"])).to(dev)
    o = {"y": torch.empty(c["n_points"], device=dev), "ind": torch.empty(c["n_points"], dtype=torch.uint8, device=dev)}
    work = c["n_points"] * c["n_modes"]
    res = {}
    # the default form for this many points (binned), then the per-point FP64 phase form
    for form in ("direct_f32_binned", "direct_f32_pointwise"):
        ws = torch.empty(grf.points_workspace_bytes(m, c["n_points"], form), dtype=torch.uint8, device=dev)
        ms, kms = _timed(torch, grf, lambda: grf.field_points(m, x, method=form, thresholds=[c["threshold"]],
                                                              want_ind=True, out=o, workspace=ws), 20, 3)
        res[form] = {"ms_per_call": ms, "kernel_ms": kms, "mode_points_per_s": work / (ms * 1e-3),
                     "roofline": {"bound": "alu", "achieved": work / (kms * 1e-3), "peak": COS_PEAK,
                                  "unit": "mode·point/s", "frac": work / (kms * 1e-3) / COS_PEAK,
                                  "kernel": "k_points_binned" if form.endswith("binned") else "k_direct_points"}}
        del ws
    head = res["direct_f32_binned"]
    out["points_2m_gauss"] = {"ms_per_call": head["ms_per_call"], "mode_points_per_s": head["mode_points_per_s"],
                              "roofline": head["roofline"], "forms": res,
                              "indicator_fraction": float(o["ind"].float().mean().item())}
    if err:
        import oracle
        sg = math.sqrt(c["sigma2"])
        idx = wl.sample_cells(c["n_points"], 32768, 4245)
        it = torch.from_numpy(idx).to(dev)
        ref = oracle.field_points(z, phi, sg, c["ell"], x[it].cpu().numpy())
        r = out["points_2m_gauss"]
        for form in ("direct_f32_pointwise", "direct_f32_binned"):
            grf.field_points(m, x, method=form, thresholds=[c["threshold"]], want_ind=True, out=o)
            e = field_errors(np, o["y"][it].double().cpu().numpy(), ref, sg)
            e["indicator"] = indicator_errors(np, o["ind"][it].cpu().numpy(), ref, [c["threshold"]],
                                              BAND["direct_f32"] * sg, sg)
            res[form]["errors"] = e
        r["errors"] = res["direct_f32_binned"]["errors"]
    return out


def epilogue_extra(grf, wl, torch, np, dev):
    out = {}
    # stand-alone epilogue over the 256^3 field: read Y, write K and the indicator
    n = 256 ** 3
    y = torch.randn(n, device=dev)
    eo = {"k": torch.empty(n, device=dev), "ind": torch.empty(n, dtype=torch.uint8, device=dev)}
    log("[bench] extras: epilogue")
    ms, kms = _timed(torch, grf, lambda: grf.epilogue(y, mu=0.0, thresholds=[0.5], want_ind=True, out=eo), 20, 3)
    nbytes = n * (4 + 4 + 1)
    out["epilogue_256^3"] = {"ms_per_call": ms, "roofline": {"bound": "hbm", "achieved": nbytes / (kms * 1e-3) / 1e9,
                                                             "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                                             "frac": nbytes / (kms * 1e-3) / HBM_PEAK,
                                                             "algorithmic": "4 B read + 4 B + 1 B written per cell"}}
    return out


def adjoint_extra(grf, wl, torch, np, dev, err=False):
    out = {}
    # adjoint workload: loss = mean squared misfit of ln K against a target field (seed 50) at
    # 10,000 observation cells (forward + backward), and the dense variant over every cell
    c = wl.WORKLOADS["adjoint_grid3d_128"]
    log("[bench] extras: adjoint_grid3d_128")
    sg = math.sqrt(c["sigma2"])
    z, phi = grf.make_modes(3, c["cov"], c["n_modes"], c["seed"])
    m = grf.modes_from_tables(z, phi, sg, c["ell"], device=dev)
    zt, pt = grf.make_modes(3, c["cov"], c["n_modes"], c["target_seed"])
    mt = grf.modes_from_tables(zt, pt, sg, c["ell"], device=dev)
    Cg = int(np.prod(c["shape"]))
    cells = wl.distinct_cells(Cg, c["n_obs"], c["obs_seed"])
    ii = np.stack([cells % 128, (cells // 128) % 128, cells // (128 * 128)], axis=1)
    xo_np = np.ascontiguousarray(ii + 0.5)
    xo = torch.from_numpy(xo_np).to(dev)
    # dL/dY of L = (1/M) sum (mu + Y - mu - Y_target)^2 at the observations (mu cancels)
    gy = (2.0 / c["n_obs"]) * (grf.field_points(m, xo)["y"] - grf.field_points(mt, xo)["y"])
    f_ms, f_k = _timed(torch, grf, lambda: grf.field_points(m, xo), 10, 2)
    b_ms, b_k = _timed(torch, grf, lambda: grf.field_backward(m, xo, gy), 10, 2)
    yg = grf.field_grid(m, c["shape"], method="direct_f32")["y"]
    gd = (2.0 / Cg) * (yg - grf.field_grid(mt, c["shape"], method="direct_f32")["y"])
    del yg
    df_ms, df_k = _timed(torch, grf, lambda: grf.field_grid(m, c["shape"], method="direct_f32"), 3, 1)
    # dense adjoint, separable form (the default on this grid) and the direct per-cell form;
    # the direct form also with the forward's Y handed back (dL/dsigma = sum g Y / sigma)
    db_ms, db_k = _timed(torch, grf, lambda: grf.field_backward_grid(m, c["shape"], gd, method="sep_bf16_x3"), 10, 2)
    dd_ms, dd_k = _timed(torch, grf, lambda: grf.field_backward_grid(m, c["shape"], gd, method="direct_f32"), 3, 1)
    yd = grf.field_grid(m, c["shape"], method="direct_f32")["y"]
    ds_ms, ds_k = _timed(torch, grf, lambda: grf.field_backward_grid(m, c["shape"], gd, y_saved=yd,
                                                                    method="direct_f32"), 3, 1)
    # separable adjoint work: rows ny nz (y padded to 32) x K = 128 (x padded) x 4 ldp
    # columns, three bf16 passes
    ldp = (c["n_modes"] + 63) // 64 * 64
    rows = ((c["shape"][1] + 31) // 32 * 32) * c["shape"][2]
    sep_flop = 2.0 * rows * 128 * 4 * ldp * 3
    sf_ms, sf_k = _timed(torch, grf, lambda: grf.field_grid(m, c["shape"], method="sep_f16"), 10, 2)
    out["adjoint_grid3d_128"] = {
        "obs": {"fwd_ms": f_ms, "bwd_ms": b_ms, "bwd_over_fwd": b_ms / f_ms,
                "bwd_mode_points_per_s": c["n_obs"] * c["n_modes"] / (b_k * 1e-3)},
        "dense": {"fwd_direct_ms": df_ms, "fwd_sep_f16_ms": sf_ms,
                  "bwd_sep_bf16_x3_ms": db_ms, "bwd_sep_over_fwd_sep": db_ms / sf_ms,
                  "bwd_sep_mode_cells_per_s": Cg * c["n_modes"] / (db_k * 1e-3),
                  "bwd_sep_roofline": {"bound": "mfma", "achieved": sep_flop / (db_k * 1e-3) / 1e12,
                                       "peak": MFMA_F16_PEAK / 1e12, "unit": "TFLOP/s",
                                       "frac": sep_flop / (db_k * 1e-3) / MFMA_F16_PEAK},
                  "bwd_direct_ms": dd_ms, "bwd_direct_over_fwd_direct": dd_ms / df_ms,
                  "bwd_direct_roofline": {"bound": "alu", "achieved": Cg * c["n_modes"] / (dd_k * 1e-3),
                                          "peak": COS_PEAK, "unit": "mode·cell/s",
                                          "frac": Cg * c["n_modes"] / (dd_k * 1e-3) / COS_PEAK},
                  "bwd_direct_saved_y_ms": ds_ms,
                  "bwd_direct_saved_y_roofline": {"bound": "alu", "achieved": Cg * c["n_modes"] / (ds_k * 1e-3),
                                                  "peak": COS_PEAK, "unit": "mode·cell/s",
                                                  "frac": Cg * c["n_modes"] / (ds_k * 1e-3) / COS_PEAK}}}
    if err:
        # gradients against the oracle's exact FP64 gradients (same dL/dY values, widened)
        import oracle
        r = out["adjoint_grid3d_128"]
        ref = oracle.grad_points(z, phi, sg, c["ell"], xo_np, gy.double().cpu().numpy())
        r["obs"]["grad_rel_l2"] = grad_errors(np, grf.field_backward(m, xo, gy), ref)
        log("[bench] adjoint: oracle dense gradient over 2,097,152 cells")
        t0 = time.perf_counter()
        refd = oracle.grad_points(z, phi, sg, c["ell"], oracle.grid_centres(c["shape"]), gd.double().cpu().numpy())
        r["dense"]["oracle_s"] = time.perf_counter() - t0
        r["dense"]["grad_rel_l2_sep_bf16_x3"] = grad_errors(
            np, grf.field_backward_grid(m, c["shape"], gd, method="sep_bf16_x3"), refd)
        r["dense"]["grad_rel_l2_direct_f32"] = grad_errors(
            np, grf.field_backward_grid(m, c["shape"], gd, method="direct_f32"), refd)
    return out


def pluri_extra(grf, wl, torch, np, dev):
    # bitruncated (pluri-Gaussian) facies on the 1024x512 grid: two fields + the rule pass
    c = wl.WORKLOADS["pluri_2d_1024x512"]
    log("[bench] extras: pluri_2d_1024x512")
    f1, f2 = c["fields"]
    ms_ = []
    for f in (f1, f2):
        z, phi = grf.make_modes(2, f["cov"], c["n_modes"], f["seed"])
        ms_.append(grf.modes_from_tables(z, phi, math.sqrt(f["sigma2"]), f["ell"], device=dev))
    rule = grf.trunc2(c["t"], c["s"], c["rule"], c["values"])
    C = int(np.prod(c["shape"]))
    res = {"cells": C, "mode_cells": 2 * C * c["n_modes"]}
    for meth in ("sep_f16", "direct_f32"):
        o = {"facies": torch.empty(C, dtype=torch.uint8, device=dev), "value": torch.empty(C, device=dev)}
        ws = torch.empty(1 << 28, dtype=torch.uint8, device=dev)
        steps = 20 if meth.startswith("sep") else 5
        ms, _ = _timed(torch, grf, lambda: grf.pluri_grid(ms_[0], ms_[1], c["shape"], rule, h=c["h"], method=meth,
                                                          want_value=True, out=o, workspace=ws), steps, 3)
        res[meth] = {"ms_per_call": ms, "mode_cells_per_s": 2 * C * c["n_modes"] / (ms * 1e-3),
                     "facies_fractions": [float(v) for v in
                                          (torch.bincount(o["facies"].long(), minlength=4).double() / C).cpu()]}
    # the stand-alone rule pass over a 256^3 pair of fields: read 2 x 4 B, write 1 B facies + 4 B value
    n = 256 ** 3
    y1, y2 = torch.randn(n, device=dev), torch.randn(n, device=dev)
    po = {"facies": torch.empty(n, dtype=torch.uint8, device=dev), "value": torch.empty(n, device=dev)}
    ms, kms = _timed(torch, grf, lambda: grf.pluri_apply(y1, y2, rule, want_value=True, out=po), 20, 3)
    nbytes = n * (4 + 4 + 1 + 4)
    res["rule_pass_256^3"] = {"ms_per_call": ms, "roofline": {
        "bound": "hbm", "achieved": nbytes / (kms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
        "frac": nbytes / (kms * 1e-3) / HBM_PEAK, "algorithmic": "2 x 4 B read + 1 B facies + 4 B value per cell"}}
    return {"pluri_2d_1024x512": res}


def krige_extra(grf, wl, torch, np, dev):
    # conditioning the 128^3 model field (seed 5) on 2,000 of the adjoint workload's observation
    # cells, valued from the target field (seed 50): FP64 Cholesky of the 2000 x 2000 system and
    # the FP32 correction sum over every cell (one sqrt and one exp2 per cell-observation pair)
    c = wl.WORKLOADS["adjoint_grid3d_128"]
    log("[bench] extras: krige_grid3d_128")
    sg = math.sqrt(c["sigma2"])
    z, phi = grf.make_modes(3, c["cov"], c["n_modes"], c["seed"])
    m = grf.modes_from_tables(z, phi, sg, c["ell"], device=dev)
    zt, pt = grf.make_modes(3, c["cov"], c["n_modes"], c["target_seed"])
    mt = grf.modes_from_tables(zt, pt, sg, c["ell"], device=dev)
    Cg = int(np.prod(c["shape"]))
    M = 2000
    cells = wl.distinct_cells(Cg, c["n_obs"], c["obs_seed"])[:M]
    ii = np.stack([cells % 128, (cells // 128) % 128, cells // (128 * 128)], axis=1)
    xo = torch.from_numpy(np.ascontiguousarray(ii + 0.5)).to(dev)
    dobs = grf.field_points(mt, xo)["y"]
    y = grf.field_grid(m, c["shape"], method="direct_f32")["y"]
    w_ms, w_k = _timed(torch, grf, lambda: grf.krige_weights(m, xo, dobs, c["cov"]), 5, 1)
    alpha, info = grf.krige_weights(m, xo, dobs, c["cov"])
    yc = y.clone()
    a_ms, a_k = _timed(torch, grf, lambda: grf.krige_apply_grid(m, xo, alpha, c["shape"], yc, c["cov"]), 5, 1)
    pairs = Cg * M
    trans_peak = COS_PEAK / 2.0  # two transcendentals (sqrt, exp2) per pair at half rate
    return {"krige_grid3d_128": {
        "n_obs": M, "cholesky_info": int(info.item()), "weights_ms": w_ms, "cholesky_and_solve_ms": w_k,
        "apply_ms": a_ms, "apply_pairs_per_s": pairs / (a_k * 1e-3),
        "apply_roofline": {"bound": "alu", "achieved": pairs / (a_k * 1e-3), "peak": trans_peak,
                           "unit": "cell·obs pair/s", "frac": pairs / (a_k * 1e-3) / trans_peak}}}


def batch_extra(grf, wl, torch, np, dev, err=False):
    inst = wl.batch_instances()
    log("[bench] extras: batch512_2d")
    items, total, tables = [], 0, []
    for p in inst:
        z, phi = grf.make_modes(2, p["cov"], p["n_modes"], p["seed"])
        tables.append((z, phi))
        m = grf.modes_from_tables(z, phi, math.sqrt(p["sigma2"]), p["ell"], device=dev)
        cells = p["shape"][0] * p["shape"][1]
        total += cells
        items.append((m, p["shape"], torch.empty(cells, device=dev)))
    # error sample: 4096 seeded cells of every instance plus 16 whole instances from the lower
    # size quartile, against the FP64 oracle (computed once for both methods)
    sample = None
    if err:
        import oracle
        sizes = np.array([p["shape"][0] * p["shape"][1] for p in inst])
        whole = set(int(i) for i in np.argsort(sizes)[:128:8])
        sample = []
        t0 = time.perf_counter()
        for i, p in enumerate(inst):
            C = int(sizes[i])
            cells = np.arange(C, dtype=np.int64) if i in whole else wl.sample_cells(C, 4096, 7000 + i)
            ref = oracle.field_cells(tables[i][0], tables[i][1], math.sqrt(p["sigma2"]), p["ell"], p["shape"], cells)
            sample.append((cells, ref))
        oracle_s = time.perf_counter() - t0

    def batch_err(meth):
        ys = np.concatenate([items[i][2][torch.from_numpy(cl).to(dev)].double().cpu().numpy()
                             for i, (cl, _) in enumerate(sample)])
        refs = np.concatenate([r for _, r in sample])
        e = field_errors(np, ys, refs, 1.0)
        e["whole_instances"] = 16
        e["oracle_s"] = oracle_s
        return e
    res = {"instances": len(inst), "cells": total, "mode_cells": total * 2048}
    # the same 512 evaluations as separate eval_field_grid calls (one workspace, sized for the largest)
    wsb = max(grf.grid_workspace_bytes(m, shape, "sep_f16") for m, shape, _ in items)
    wsp = torch.empty(wsb, dtype=torch.uint8, device=dev)
    sep_ms, _ = _timed(torch, grf, lambda: [grf.field_grid(m, shape, method="sep_f16", out={"y": y}, workspace=wsp)
                                            for m, shape, y in items], 3, 1)
    res["sep_f16_separate_calls"] = {"ms_per_batch": sep_ms, "mode_cells_per_s": total * 2048 / (sep_ms * 1e-3)}
    for meth in ("sep_f16", "direct_f32"):
        # tuned tile choices persist in a per-user cache file between runs
        plan = grf.Plan(meth, graph=True, autotune=True,
                        tune_cache=os.path.join(tempfile.gettempdir(), "grf_tune_cache.txt"))
        steps = 10 if meth.startswith("sep") else 2
        ms, kms = _timed(torch, grf, lambda: plan.run(items), steps, 2)
        res[meth] = {"ms_per_batch": ms, "persistent_kernel_ms": kms, "mode_cells_per_s": total * 2048 / (ms * 1e-3),
                     "plan": plan.info()}
        if sample is not None:
            res[meth]["errors"] = batch_err(meth)
        plan.close()
    return res


if __name__ == "__main__":
    main()
