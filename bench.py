#!/usr/bin/env python3
"""Benchmark: forward + backward ASM propagations per second through a
diffractive network on one MI355X.

Workload (one "step"): 64 complex64 fields of 1024 x 1024 (amplitude =
seeded blurred noise, zero phase) pass through 5 trainable phase masks, each
followed by angular-spectrum propagation over 10 cm (spacing 8 um, 700 nm,
2x zero padding to 2048 x 2048); an MSE loss on the output intensity against
a seeded target is fused into the last propagation; the backward pass runs
the adjoint propagations and accumulates the 5 mask gradients.  That is
64 x 5 forward + 64 x 5 adjoint = 640 propagations per step, every one of
them in the library's HIP kernels (the Python side only enqueues calls).

Prints one JSON line (see the keys below).  --gpus must be 1: the library
runs on a single GPU.

``--workload poly4f`` measures the polychromatic 4f imaging workload instead
(251 wavelengths x 3 propagations of a 1000^2 complex64 field padded to
2048^2, weighted incoherent sum fused): forward propagations per second.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
VALU_FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published (packed FP32 FMA)
# The library is built without packed FP32 instructions: each lane retires
# one FP32 FMA per cycle, 256 CU x 64 lanes x 2 flop x 2.4 GHz.
VALU_FP32_NONPACKED_TFLOPS = 78.6
VALU_FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector, published


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--batch", type=int, default=64)
    p.add_argument("--n", type=int, default=1024)
    p.add_argument("--layers", type=int, default=5)
    p.add_argument("--method", choices=["asm", "di", "auto"], default="asm",
                   help="propagation method of the network's layers (the headline figure is asm)")
    p.add_argument("--workload", choices=["diffnet", "poly4f", "resample", "anylength", "suite", "uneven"],
                   default="diffnet")
    p.add_argument("--fwhm-nm", type=float, default=10.0, help="poly4f: spectral FWHM")
    p.add_argument("--cache-tables", action="store_true",
                   help="poly4f: build the DI tables once, before the timed region (reported separately)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--uneven-sizes", default="",
                   help="uneven: keep only the jobs of these field sizes (comma-separated)")
    p.add_argument("--uneven-count", type=int, default=0,
                   help="uneven: keep at most this many of the selected jobs (0: all)")
    p.add_argument("--cpu-sample-fields", type=int, default=0,
                   help="fields in the CPU oracle sample (0 = one per host thread)")
    p.add_argument("--cpu-child", default="", help=argparse.SUPPRESS)
    p.add_argument("--cpu-sample-layers", type=int, default=3,
                   help="layers (of the workload's masks) in the CPU oracle sample")
    p.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    p.add_argument("--no-autotune", action="store_true",
                   help="run with the built-in schedule instead of tuning one before the timed region")
    p.add_argument("--plain-steps", type=int, default=1,
                   help="timed steps of the unfused plain form (0 = skip the comparison)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a 256 MiB device copy (for scaling FETCH_SIZE / WRITE_SIZE)")
    return p.parse_args()


def copy_calibration():
    """A plain device-to-device copy of known size: 3 x 256 MiB."""
    import torch
    x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 256 * 1024 * 1024, "copies": 3}))
    return 0


# Files that hold the propagation kernels' device code and launch shapes.
KERNEL_SOURCES = ("fft.hpp", "kernels.hpp", "launch.hpp", "launch_impl.hpp", "inst_f32.hip", "inst_f64.hip",
                  "queue.hpp", "queue_impl.hpp", "queue_f32.hip", "queue_f64.hip")


def _code_only(text: str) -> str:
    """C++ source without comments and blank lines, each line stripped (the
    kernel files hold no string literal with a comment marker)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*", "", ln).strip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def kernel_source_digest() -> str:
    """SHA-256 over the propagation kernels' code (file names + the sources
    without comments), so that records taken on the kernels stay valid
    across comment-only edits and lapse on any change to the code."""
    import hashlib
    d = os.path.join(ROOT, "paper_2411_18591_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()


def measured_traffic(kernel_label: str, launch_fields: int):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE
    counter runs, or None when none were taken for this kernel, the kernel
    sources changed since, or a launch now covers a different number of
    fields."""
    path = os.path.join(ROOT, "profiles", "diffnet_1024_c64_hbm_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_digest() or rec.get("launch_fields") != launch_fields:
        return None
    ent = rec.get("per_launch", {}).get(kernel_label.split(".", 1)[-1])
    return None if ent is None else int(ent["bytes"])


def counted_valu(kernel_label: str, launch_fields: int):
    """VALU issue of a kernel from the committed SQ counter runs
    (`profiles/diffnet_1024_c64_counters.json`), or None when they were not
    taken for it, the kernel sources changed since, or a launch covers a
    different number of fields."""
    path = os.path.join(ROOT, "profiles", "diffnet_1024_c64_counters.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_digest() or rec.get("launch_fields") != launch_fields:
        return None
    ent = rec.get("per_launch", {}).get(kernel_label.split(".", 1)[-1])
    if ent is None:
        return None
    return {"frac": ent["valu_busy_frac"], "frac_at_2p4GHz": ent["valu_busy_frac_at_2p4GHz"],
            "lane_instr_per_point_transform": ent["lane_instr_per_point_transform"],
            "source": "SQ_INSTS_VALU / (256 CUs x cycles), profiles/diffnet_1024_c64_counters.json"}


def fft_flops(L: int) -> float:
    """Conventional flop count of one complex FFT of length L."""
    return 5.0 * L * math.log2(L)


def kernel_model(name: str, wl, chunk_fields: int, c: int = 8):
    """Algorithmic bytes and flops of ONE launch of a propagation kernel for
    this workload (N x N field, P x P padded, `chunk_fields` fields per
    launch, `c` bytes per complex value: 8 for c64, 16 for c128).  Bytes are what the kernel must read and write in the 3-pass
    decomposition (field in/out, the N x P intermediate in/out, masks and
    gradients); flops count 5 L log2 L per length-L FFT plus 6 per complex
    multiply."""
    N, P = wl["n"], wl["padded"]
    f = chunk_fields
    if ".row_fwd_" in name:
        by = f * (N * N * c + N * P * c) + (N * N * 4 if name.startswith("fwd") else 0)
        fl = f * (N * fft_flops(P) + (6 * N * N if name.startswith("fwd") else 0))
    elif ".col_" in name:
        by = f * 2 * N * P * c
        fl = f * P * (2 * fft_flops(P) + 6 * P)
    elif ".row_mid_" in name:
        # fused layer boundary: intermediate in, layer output (forward) or
        # input gradient (backward) out, intermediate of the next layer out
        if name.startswith("fwd"):
            by = f * (2 * N * P * c + N * N * c) + N * N * 4
        else:  # reads the saved layer input (the link gradient, transient in
            # the training step, is not stored); mask in, gradient partials out
            by = f * (2 * N * P * c + N * N * c) + 2 * N * N * 4
        fl = f * N * 2 * fft_flops(P)
    elif ".row_inv_" in name:
        if name.startswith("fwd"):
            by = f * (N * P * c + N * N * c)
        else:  # reads g rows + saved input, writes grad_in, mask in / grad out
            by = f * (N * P * c + 2 * N * N * c) + 2 * N * N * 4
        fl = f * N * fft_flops(P)
    else:
        return None
    return by, fl


def load_inputs(wl_def):
    """The workload's seeded inputs (fields, masks, target), cached as an
    npz file under TMPDIR so child processes and repeated runs share them."""
    import numpy as np
    B, N, L = wl_def.batch, wl_def.n, wl_def.layers
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"toprop_bench_{B}_{N}_{L}.npz")
    if os.path.exists(cache):
        with np.load(cache) as z:
            return z["u0"], z["masks"], z["target"]
    print(f"[bench] generating inputs: {B} x {N}^2 fields, {L} masks", file=sys.stderr, flush=True)
    t0 = time.time()
    u0_np, masks_np, target_np = wl_def.fields(), wl_def.masks(), wl_def.target()
    try:
        tmp = cache + f".{os.getpid()}.npz"
        np.savez(tmp, u0=u0_np, masks=masks_np, target=target_np)
        os.replace(tmp, cache)
    except OSError:
        pass
    print(f"[bench] inputs ready in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    return u0_np, masks_np, target_np


def main():
    args = parse()
    if args.cpu_child:
        return cpu_child(args)
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(sharding across GPUs is not implemented)"}))
        return 2
    if args.workload == "poly4f":
        return run_poly4f(args)
    if args.workload == "resample":
        return run_resample(args)
    if args.workload == "anylength":
        return run_anylength(args)
    if args.workload == "suite":
        return run_suite(args)
    if args.workload == "uneven":
        import torch
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        res = run_uneven(args, dev)
        print(json.dumps({"metric": "uneven batch: time per forward + adjoint step", "unit": "ms", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "data": "synthetic (seeded, as in workloads/)", "configs": {"uneven_c64": res}}))
        return 0
    import workloads
    wl_def = workloads.DiffractiveNetWorkload(batch=args.batch, n=args.n, layers=args.layers)
    B, N, L = wl_def.batch, wl_def.n, wl_def.layers
    P = 2 * N
    u0_np, masks_np, target_np = load_inputs(wl_def)
    # The CPU baseline runs first, in child processes, while no GPU work is
    # in flight (and before this process touches the GPU).
    cpu, sample = (None, None)
    if not args.no_cpu_baseline:
        cpu, sample = cpu_baseline(args, wl_def)

    import numpy as np
    import torch

    import paper_2411_18591_amd as tp
    from paper_2411_18591_amd import _capi
    from paper_2411_18591_amd.diffnet import DiffractiveNet

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    opt = tp.Optics(dy=wl_def.d, dx=wl_def.d, wavelength=wl_def.wavelength, z=wl_def.z, pad=2,
                    method=args.method)
    method = tp.resolve_method(opt, N, N).upper()
    net = DiffractiveNet(torch.from_numpy(u0_np).to(dev), torch.from_numpy(masks_np).to(dev),
                         torch.from_numpy(target_np).to(dev), opt)
    loss = net.loss
    step = net.step
    # The launch schedule of the padded grid (column configuration, chunk,
    # fields per row-pass workgroup), tuned by the library's autotuner on one
    # layer's forward propagation of the whole batch before anything is timed.
    plan = None
    schedule = {"tuned": False, "plan": None}
    if not args.no_autotune:
        print("[bench] autotune", file=sys.stderr, flush=True)
        tuned, plan = tp.autotune(net.u[0], opt, phase=net.masks[0])
        del tuned
        torch.cuda.synchronize()
        print(f"[bench] plan {plan}", file=sys.stderr, flush=True)
        # The autotuner times one layer's forward propagation; the step is a
        # chained forward + backward.  The tuned plan is checked on the step
        # itself against the built-in schedule (a few untimed steps each) and
        # the faster one is kept.
        def step_ms(n=3):
            step()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                step()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / n
        t_tuned = step_ms()
        tp.plan_clear()
        t_builtin = step_ms()
        keep = "tuned" if t_tuned < t_builtin else "built-in"
        if keep == "tuned":
            tp.plan_set(P, P, plan["col_variant"], plan["chunk_mb"], us=plan["us"], row_fpb=plan["row_fpb"])
        schedule = {"tuned": True, "plan": plan if keep == "tuned" else None, "autotuner_plan": plan,
                    "kept": keep, "step_ms": {"tuned": round(t_tuned, 3), "built_in": round(t_builtin, 3)}}
        print(f"[bench] schedule {schedule}", file=sys.stderr, flush=True)

    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] timed region", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    t_wall = time.perf_counter()
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    props = 2 * B * L
    value = props / (ms_step / 1000.0)
    print(f"[bench] {ms_step:.3f} ms/step, loss {float(loss.item()):.6e}", file=sys.stderr, flush=True)

    # Per-kernel durations: the same K steps again, every launch bracketed by
    # HIP events on its own stream (the events cost a few microseconds per
    # launch, so this pass is kept out of the throughput above).
    prof = {}
    prof_ms_step = None
    if not args.no_profile:
        print("[bench] profiled pass", file=sys.stderr, flush=True)
        _capi.profile_begin()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        prof = _capi.profile_end()
        prof_ms_step = ev0.elapsed_time(ev1) / args.steps

    # Algorithmic HBM bytes of one step (fields in/out of every propagation,
    # the loss gradient, masks and mask gradients; no padded intermediates).
    c = 8
    fwd_bytes = L * B * N * N * 2 * c + B * N * N * c + N * N * 4 + L * N * N * 4
    bwd_bytes = (L - 1) * B * N * N * 3 * c + B * N * N * 2 * c + L * N * N * 4 * 3
    step_bytes = fwd_bytes + bwd_bytes
    hbm_frac_step = step_bytes / (ms_step / 1000.0) / (HBM_PEAK_GBS * 1e9)

    # Dominant kernel: largest total GPU time in the timed region.
    wl = {"n": N, "padded": P}
    chunk = max(1, min(B, (128 << 20) // (N * P * c)))
    kern = []
    for name, (cnt, ms) in prof.items():
        m = kernel_model(name, wl, chunk)
        kern.append((ms, name, cnt, m))
    kern.sort(reverse=True)
    roofline = None
    kernels_out = {}
    for ms, name, cnt, m in kern:
        avg_us = 1000.0 * ms / cnt
        entry = {"launches": cnt, "avg_us": round(avg_us, 2), "share": round(ms / sum(k[0] for k in kern), 4)}
        if m:
            by, fl = m
            entry["GB_s"] = round(by / (avg_us * 1e-6) / 1e9, 1)
            entry["TFLOP_s"] = round(fl / (avg_us * 1e-6) / 1e12, 2)
        kernels_out[name] = entry
    if kern and kern[0][3]:
        ms, name, cnt, (by, fl) = kern[0]
        avg_s = ms / cnt / 1000.0
        gbs = by / avg_s / 1e9
        tfs = fl / avg_s / 1e12
        f_h = gbs / HBM_PEAK_GBS
        f_a = tfs / VALU_FP32_PEAK_TFLOPS
        # the committed counter records were taken with the built-in schedule
        same_run = (N, B, L, method) == (1024, 64, 5, "ASM") and schedule["plan"] is None
        traffic = measured_traffic(name, chunk) if same_run else None
        valu = counted_valu(name, chunk) if same_run else None
        # bound: the resource closer to saturation, the ALU side taken at the
        # rate this build can reach (no packed FP32); reported against the
        # published peak, with the non-packed view beside it
        if tfs / VALU_FP32_NONPACKED_TFLOPS >= f_h:
            roofline = {"bound": "alu", "achieved": round(tfs, 3), "peak": VALU_FP32_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(f_a, 4), "traffic": traffic,
                        "kernel": name, "avg_us": round(avg_s * 1e6, 2),
                        "nonpacked_view": {"peak": VALU_FP32_NONPACKED_TFLOPS,
                                           "frac": round(tfs / VALU_FP32_NONPACKED_TFLOPS, 4)},
                        "hbm_view": {"achieved_GB_s": round(gbs, 1), "frac": round(f_h, 4)},
                        "valu_issue_counted": valu}
        else:
            roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(f_h, 4), "traffic": traffic,
                        "kernel": name, "avg_us": round(avg_s * 1e6, 2),
                        "alu_view": {"achieved_TFLOP_s": round(tfs, 3), "frac": round(f_a, 4)}}

    # The same step through the unfused plain form (one field per launch
    # sequence, every intermediate in HBM), timed the same way.
    plain = None
    if args.plain_steps > 0:
        loss_fused = float(loss.item())
        print("[bench] plain form", file=sys.stderr, flush=True)
        step(plain=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.plain_steps):
            step(plain=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        p_ms = ev0.elapsed_time(ev1) / args.plain_steps
        plain = {"value": round(props / (p_ms / 1000.0), 1), "unit": "propagations/s",
                 "ms_per_step": round(p_ms, 3), "steps": args.plain_steps,
                 "hbm_roofline_frac": round(step_bytes / (p_ms / 1000.0) / (HBM_PEAK_GBS * 1e9), 5),
                 "loss_rel_diff_vs_fused": abs(float(loss.item()) - loss_fused) / abs(loss_fused),
                 "fused_speedup": round(p_ms / ms_step, 2)}

    parity = None
    if sample is not None:
        parity = parity_on_sample(sample, u0_np, masks_np, target_np, opt)

    out = {
        "metric": f"fwd+bwd {method} propagations/s at 1024^2 c64; % of HBM roofline vs plain form",
        "value": round(value, 1),
        "unit": "propagations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic (seeded blurred-noise fields, uniform random phase masks, blurred target)",
        "config": {
            "workload": f"diffractive network: {B} x {N}^2 complex64 fields, {L} phase masks, "
                        f"{method} z=10 cm, 8 um, 700 nm, padded to {P}^2, MSE loss, fwd+bwd to masks",
            "global_batch": B, "grid": N, "padded": P, "layers": L,
            "propagations_per_step": props,
        },
        "hbm_roofline_step": {"algorithmic_bytes": step_bytes, "frac": round(hbm_frac_step, 4)},
        "schedule": schedule,
        "profiled_pass_ms_per_step": None if prof_ms_step is None else round(prof_ms_step, 4),
        "plain_form": plain,
        "roofline": roofline,
        "kernels": kernels_out,
        "wall_s": round(t_wall, 3),
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
    }
    print(json.dumps(out))
    return 0


def dominant_roofline(prof, wl, chunk):
    """Roofline entry of the kernel with the largest GPU time (no traffic)."""
    kern = []
    for name, (cnt, ms) in prof.items():
        m = kernel_model(name, wl, chunk)
        if m:
            kern.append((ms, name, cnt, m))
    if not kern:
        return None
    ms, name, cnt, (by, fl) = max(kern)
    avg_s = ms / cnt / 1000.0
    gbs, tfs = by / avg_s / 1e9, fl / avg_s / 1e12
    f_h, f_a = gbs / HBM_PEAK_GBS, tfs / VALU_FP32_PEAK_TFLOPS
    if tfs / VALU_FP32_NONPACKED_TFLOPS >= f_h:
        return {"bound": "alu", "achieved": round(tfs, 3), "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(f_a, 4), "traffic": None, "kernel": name, "avg_us": round(avg_s * 1e6, 2),
                "nonpacked_view": {"peak": VALU_FP32_NONPACKED_TFLOPS,
                                   "frac": round(tfs / VALU_FP32_NONPACKED_TFLOPS, 4)},
                "hbm_view": {"achieved_GB_s": round(gbs, 1), "frac": round(f_h, 4)}}
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(f_h, 4), "traffic": None, "kernel": name, "avg_us": round(avg_s * 1e6, 2),
            "alu_view": {"achieved_TFLOP_s": round(tfs, 3), "frac": round(f_a, 4)}}


def run_poly4f(args):
    """Polychromatic 4f imaging: one image = every wavelength through
    P_f, lens, P_2f, lens, P_f with the weighted intensity summed (one
    library call)."""
    import numpy as np
    import torch

    import paper_2411_18591_amd as tp
    from paper_2411_18591_amd import _capi
    from paper_2411_18591_amd.fourf import FourF
    import workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    wl = workloads.Polychromatic4fWorkload(fwhm=args.fwhm_nm * 1e-9)
    u_np = wl.field()
    u = torch.from_numpy(u_np).to(dev)
    lams, wts = wl.wavelengths(), wl.weights()
    sys4f = FourF(wl.f, wl.d, wl.d, method=args.method, cache_tables=args.cache_tables)
    methods = sorted({tp.resolve_method(sys4f._opt(lam, z), wl.n, wl.n) for lam in lams for z in (wl.f, 2 * wl.f)})
    I = torch.zeros((wl.n, wl.n), dtype=torch.float32, device=dev)

    def step():
        I.zero_()
        sys4f.image(u, lams, wts, out=I)

    table_ms = None
    if args.cache_tables:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()  # builds and keeps the DI tables
        torch.cuda.synchronize()
        table_ms = round(1000.0 * (time.perf_counter() - t0), 2)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    props = 3 * len(lams)
    prof = {}
    if not args.no_profile:
        _capi.profile_begin()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        prof = _capi.profile_end()
    P = 2048
    wlm = {"n": wl.n, "padded": P}
    roofline = dominant_roofline(prof, wlm, 1)
    c = 8
    step_bytes = props * 2 * wl.n * wl.n * c
    kernels_out = {k: {"launches": n, "avg_us": round(1000.0 * ms / n, 2)} for k, (n, ms) in
                   sorted(prof.items(), key=lambda kv: -kv[1][1])}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        pick = [len(lams) // 2 - 1, len(lams) // 2, len(lams) // 2 + 1]
        ua = u_np.astype(np.complex128)
        meth = {"ASM": oracle.ASM, "DI": oracle.DI}
        t0 = time.perf_counter()
        acc = np.zeros((wl.n, wl.n))
        for k in pick:
            lam = lams[k]
            L = oracle.lens(wl.n, wl.n, wl.d, wl.d, lam, wl.f)
            def prop(v, z):
                m = meth.get(args.method.upper())
                if m is None:
                    m = oracle.resolve_method(wl.n, wl.n, wl.d, wl.d, lam, z)
                return oracle.propagate(v, wl.d, wl.d, lam, z, m, padded=(P, P))
            v = prop(ua, wl.f)
            v = prop(oracle.modulate(v, L), 2 * wl.f)
            v = prop(oracle.modulate(v, L), wl.f)
            acc += wts[k] * oracle.intensity(v)
        dt = time.perf_counter() - t0
        cpu = {"value": round(3 * len(pick) / dt, 3), "unit": "propagations/s", "cores": 1, "kind": "oracle",
               "sample": f"3 of {len(lams)} wavelengths through the 4f system ({3 * len(pick)} FP64 "
                         f"propagations of 1000^2 -> 2048^2, {dt:.1f} s; one field, one thread)"}
    out = {
        "metric": "polychromatic 4f imaging: forward propagations/s at 1000^2 c64",
        "value": round(props / (ms_step / 1000.0), 1),
        "unit": "propagations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic (seeded blurred-noise amplitude, uniform phase; Gaussian spectrum)",
        "config": {
            "workload": f"polychromatic 4f imaging: {len(lams)} wavelengths 575-825 nm (FWHM "
                        f"{args.fwhm_nm:g} nm), 1000^2 complex64, 10 um, f = 200 mm, padded to 2048^2, "
                        f"methods {'/'.join(methods)}, weighted intensity sum fused",
            "wavelengths": len(lams), "grid": wl.n, "padded": P, "propagations_per_step": props,
            "di_tables": ("built once before the timed region (first image incl. building: "
                          f"{table_ms} ms)") if args.cache_tables else "built within every image's call",
        },
        "hbm_roofline_step": {"algorithmic_bytes": step_bytes,
                              "frac": round(step_bytes / (ms_step / 1000.0) / (HBM_PEAK_GBS * 1e9), 4)},
        "roofline": roofline,
        "kernels": kernels_out,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


def run_resample(args):
    """Resampling onto another grid: 64 complex64 fields of 1024^2 (8 um)
    interpolated bilinearly onto 1500^2 (5.5 um), forward and adjoint (the
    gradient map).  HBM-bound: algorithmic bytes = fields in + fields out."""
    import numpy as np
    import torch

    import paper_2411_18591_amd as tp
    from paper_2411_18591_amd import _capi

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    B, n, m = 64, 1024, 1500
    gen = torch.Generator(device=dev).manual_seed(7001)
    u = torch.randn((B, n, n), dtype=torch.complex64, device=dev, generator=gen)
    gi = tp.Grid(n, n, 8e-6, 8e-6)
    go = tp.Grid(m, m, 5.5e-6, 5.5e-6)
    out = torch.empty((B, m, m), dtype=torch.complex64, device=dev)
    back = torch.empty_like(u)

    def step():
        tp.resample(u, gi, go, "bilinear", out=out)
        tp.resample(out, gi, go, "bilinear", adjoint=True, out=back)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    _capi.profile_begin()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = _capi.profile_end()
    per_dir = B * (n * n + m * m) * 8
    kern = {}
    best = None
    for name, (cnt, ms) in prof.items():
        avg_s = ms / cnt / 1000.0
        gbs = per_dir / avg_s / 1e9
        kern[name] = {"launches": cnt, "avg_us": round(avg_s * 1e6, 2), "GB_s": round(gbs, 1)}
        if best is None or ms > best[0]:
            best = (ms, name, avg_s, gbs)
    roofline = None
    if best:
        roofline = {"bound": "hbm", "achieved": round(best[3], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(best[3] / HBM_PEAK_GBS, 4), "traffic": None, "kernel": best[1],
                    "avg_us": round(best[2] * 1e6, 2)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        k = 4
        un = u[:k].cpu().numpy()
        t0 = time.perf_counter()
        oracle.resample(un, (n, n, 8e-6, 8e-6, 0.0, 0.0), (m, m, 5.5e-6, 5.5e-6, 0.0, 0.0), oracle.BILINEAR)
        dt = time.perf_counter() - t0
        cpu = {"value": round(k / dt, 3), "unit": "fields/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} fields forward (numpy, {dt:.1f} s)"}
    print(json.dumps({
        "metric": "bilinear resampling fwd+adjoint: fields/s at 1024^2 -> 1500^2 c64",
        "value": round(2 * B / (ms_step / 1000.0), 1), "unit": "fields/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic (seeded complex Gaussian fields)",
        "config": {"workload": f"resampling: {B} x {n}^2 complex64 (8 um) -> {m}^2 (5.5 um), bilinear, "
                               "forward and adjoint"},
        "roofline": roofline, "kernels": kern, "cpu_baseline": cpu}))
    return 0


def _event_ms(fn, steps, warmup):
    """Mean milliseconds of fn() between two events on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def run_anylength(args):
    """Padding that is not a power of two: 16 complex64 fields of 1000^2
    (8 um, 700 nm, AS 10 cm, phase mask) padded 2x to 2000^2 (the unfused
    path with mixed-radix line transforms), forward and adjoint, beside the
    same fields padded to 2002^2 (2 * 7 * 11 * 13: Bluestein line transforms)
    and to 2048^2 (the fused path).  Beside it, the paper's own examples at
    their native 2x padding against the power-of-two rounding: a Gaussian
    Schell-model coherence propagation on a 50^2 grid (100^2 / 128^2), and
    the 4f image of a 1000^2 field per wavelength (2000^2 / 2048^2, 25
    wavelengths per call)."""
    import numpy as np
    import torch

    import paper_2411_18591_amd as tp

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    B, n = 16, 1000
    gen = torch.Generator(device=dev).manual_seed(7101)
    u = torch.randn((B, n, n), dtype=torch.complex64, device=dev, generator=gen)
    phi = torch.rand((n, n), dtype=torch.float32, device=dev, generator=gen) * 6.2832
    res = {}
    for name, P in (("2000", 2000), ("2002", 2002), ("2048", 2048)):
        opt = tp.Optics(dy=8e-6, dx=8e-6, wavelength=0.7e-6, z=0.1, padded=(P, P))
        out = torch.empty_like(u)
        gin = torch.empty_like(u)

        def step():
            tp.propagate(u, opt, out=out, phase=phi)
            tp.propagate_backward(out, opt, grad_in=gin, phase=phi)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(dev)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        res[name] = {"ms_per_step": round(ms, 3), "propagations_per_s": round(2 * B / (ms / 1000.0), 1),
                     "padded": opt.padded_shape(n, n)}
    # the paper's own small-grid and 4f examples at their native 2x padding
    native = {}
    g = 50
    G = torch.randn((g, g, g, g), dtype=torch.complex64, device=dev, generator=gen)
    for name, rp in (("gsm_coherence_50_pad100", False), ("gsm_coherence_50_pad128", True)):
        opt = tp.Optics(dy=10e-6, dx=10e-6, wavelength=0.7e-6, z=0.02, pad=2, round_pow2=rp)
        native[name] = {"ms": round(_event_ms(lambda: tp.coherence_propagate(G, opt), args.steps, args.warmup), 4),
                        "padded": opt.padded_shape(g, g)}
    from paper_2411_18591_amd.fourf import FourF
    lams = [650e-9 + 100e-9 * k / 24 for k in range(25)]
    wts = [1.0 / 25] * 25
    for name, P in (("fourf_1000_pad2000_per_wavelength", 2000), ("fourf_1000_pad2048_per_wavelength", 2048)):
        sys4f = FourF(0.2, 10e-6, 10e-6, method="asm", padded=(P, P))
        ms = _event_ms(lambda: sys4f.image(u[0], lams, wts), max(1, args.steps // 2), 1)
        native[name] = {"ms": round(ms / 25, 4), "padded": [P, P]}
    ms = res["2000"]["ms_per_step"]
    step_bytes = 2 * B * n * n * 16
    print(json.dumps({
        "metric": "fwd+adjoint propagations/s at 1000^2 padded 2000^2 c64 (non-power-of-two padding)",
        "value": res["2000"]["propagations_per_s"], "unit": "propagations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic (seeded complex Gaussian fields, uniform phase mask)",
        "config": {"workload": f"{B} x {n}^2 complex64, AS z = 10 cm, 8 um, 700 nm, phase mask, padded 2x to "
                               "2000^2 (unfused path, mixed-radix line transforms); the same fields padded to "
                               "2002^2 (Bluestein line transforms) and 2048^2 (fused path) for comparison"},
        "hbm_roofline_step": {"algorithmic_bytes": step_bytes,
                              "frac": round(step_bytes / (ms / 1000.0) / (HBM_PEAK_GBS * 1e9), 5)},
        "bluestein_2002": res["2002"], "pow2_2048": res["2048"], "paper_examples_native_padding": native,
        "roofline": None, "cpu_baseline": None,
        "not_measured": "roofline: the unfused mixed-radix passes have no per-launch model here; cpu_baseline: "
                        "the oracle transforms extents that are not powers of two with its O(n^2) DFT, meant "
                        "for small grids"}))
    return 0


def _timed(step, steps, warmup):
    """Mean milliseconds of `step` between two events (after `warmup` runs),
    and the per-kernel profile of one more pass."""
    import torch

    from paper_2411_18591_amd import _capi
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    _capi.profile_begin()
    step()
    torch.cuda.synchronize()
    prof = _capi.profile_end()
    top = sorted(prof.items(), key=lambda kv: -kv[1][1])[:3]
    _timed.last_profile = prof
    return ms, {k: {"launches": n, "avg_us": round(1000.0 * t / n, 2)} for k, (n, t) in top}


def model_roofline(prof, n, padded, fields_per_launch, c=8):
    """Roofline entry of the kernel with the largest GPU time in `prof` (one
    profiled step: name -> (launches, total ms)) among those `kernel_model`
    covers: N x N fields padded to P x P, `fields_per_launch(name, launches)`
    fields per launch, `c` bytes per complex value.  complex128 kernels are
    priced against the FP64 vector peak, complex64 ones against FP32."""
    best = None
    for name, (cnt, ms) in prof.items():
        if cnt <= 0:
            continue
        f = fields_per_launch(name, cnt)
        m = kernel_model(name, {"n": n, "padded": padded}, f, c) if f else None
        if m and (best is None or ms > best[0]):
            best = (ms, name, cnt, f, m)
    if best is None:
        return None
    ms, name, cnt, f, (by, fl) = best
    avg_s = ms / cnt / 1000.0
    gbs, tfs = by / avg_s / 1e9, fl / avg_s / 1e12
    peak = VALU_FP64_PEAK_TFLOPS if c == 16 else VALU_FP32_PEAK_TFLOPS
    return {"bound": "alu", "achieved": round(tfs, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(tfs / peak, 4), "traffic": None, "kernel": name, "avg_us": round(avg_s * 1e6, 2),
            "fields_per_launch": f, "algorithmic_bytes_per_launch": int(by), "flops_per_launch": int(fl),
            "hbm_view": {"achieved_GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}}


def _oracle_rate(fn, units, budget_s):
    """Runs fn() (one unit of `units` propagations) until `budget_s` of wall
    time have passed (at least once); returns (units / s, runs, seconds)."""
    runs, t0 = 0, time.perf_counter()
    while True:
        fn()
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            return units * runs / el, runs, el


def run_suite(args):
    """The other workloads, one step each, timed on one GPU:
    a Gaussian beam through z, lens, z (256^2 complex128: latency); polarized
    focusing (8 wavelengths x 3 components x 2048^2 complex64, Jones + lens,
    Fresnel, weighted-intensity loss, gradient to f); a Gaussian Schell
    source (64^4 complex64 coherence, mask + lens, MSE of the diagonal,
    gradient to the mask); 128 uneven jobs (256^2 .. 4096^2, forward and
    adjoint in one call each)."""
    import numpy as np
    import torch

    import paper_2411_18591_amd as tp
    import workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    res = {}

    g = workloads.GaussianLensWorkload()
    u = torch.from_numpy(g.field()).to(dev)
    o1 = tp.Optics(dy=g.d, dx=g.d, wavelength=g.wavelength, z=g.z1, pad=g.pad)
    o2 = tp.Optics(dy=g.d, dx=g.d, wavelength=g.wavelength, z=g.z2, pad=g.pad)
    mid, out = torch.empty_like(u), torch.empty_like(u)

    def gauss():
        tp.propagate_jobs([u, mid], [o1, o2], outs=[mid, out], elements=[{}, {"lens_f": g.f}])
    ms, top = _timed(gauss, max(args.steps, 20), args.warmup)
    res["gaussian_lens_256_c128"] = {
        "ms_per_step": round(ms, 4), "propagations_per_step": 2, "propagations_per_s": round(2 / (ms / 1000.0), 1),
        "kernels": top,
        "roofline": model_roofline(_timed.last_profile, g.n, 2 * g.n, lambda name, cnt: 1, c=16)}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        u_h = g.field()
        lens = oracle.lens(g.n, g.n, g.d, g.d, g.wavelength, g.f)

        def gauss_oracle():
            a = oracle.propagate(u_h, g.d, g.d, g.wavelength, g.z1, oracle.ASM, g.pad)
            return oracle.propagate(a * lens, g.d, g.d, g.wavelength, g.z2, oracle.ASM, g.pad)
        rate, runs, secs = _oracle_rate(gauss_oracle, 2, 2.0)
        got = out.cpu().numpy()
        exp = gauss_oracle()
        res["gaussian_lens_256_c128"]["error_vs_oracle"] = float(
            f"{np.linalg.norm(got - exp) / np.linalg.norm(exp):.3e}")
        res["gaussian_lens_256_c128"]["cpu_baseline"] = {
            "value": round(rate, 2), "unit": "propagations/s", "cores": host_threads(), "kind": "oracle",
            "sample": f"the whole step (z1, lens, z2) in FP64, {runs} runs in {secs:.1f} s"}

    w = workloads.PolarizedWorkload()
    E = torch.from_numpy(w.field()).to(dev)
    W = torch.from_numpy(w.weight()).to(dev)
    K = len(w.wavelengths)
    outs, grads = torch.empty_like(E), torch.empty_like(E)
    losses = torch.zeros(K, dtype=torch.float64, device=dev)
    gfs = torch.zeros(K, dtype=torch.float64, device=dev)
    J = tp.jones3(tp.waveplate(w.qwp_angle, np.pi / 2), tp.linear_polarizer(w.lp_angle))
    opts = [tp.Optics(dy=w.d, dx=w.d, wavelength=float(lam), z=w.z, method="fresnel", pad=w.pad)
            for lam in w.wavelengths]
    els = [dict(jones=J, lens_f=w.f, epi=tp._capi.TO_EPI_WEIGHTED, epi_ref=W, epi_scale=w.d * w.d,
                epi_grad=grads[k], epi_loss=losses[k]) for k in range(K)]

    def polarized():
        losses.zero_()
        gfs.zero_()
        tp.propagate_jobs(list(E), opts, outs=list(outs), elements=els, ncomp=3)
        tp.propagate_backward_jobs(list(grads), opts, saved_ins=list(E), grad_ins=[None] * K, grad_fs=list(gfs),
                                   elements=[dict(jones=J, lens_f=w.f)] * K, ncomp=3)
    ms, top = _timed(polarized, args.steps, args.warmup)
    res["polarized_8x3x2048_c64"] = {
        "ms_per_step": round(ms, 3), "propagations_per_step": 2 * 3 * K,
        "propagations_per_s": round(2 * 3 * K / (ms / 1000.0), 1), "kernels": top,
        # every launch of a job covers its three components
        "roofline": model_roofline(_timed.last_profile, w.n, 2 * w.n, lambda name, cnt: 3)}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        J_h = np.array(J, dtype=np.complex128)
        E0 = E[0].cpu().numpy().astype(np.complex128)
        lam0 = float(w.wavelengths[0])
        lens0 = oracle.lens(w.n, w.n, w.d, w.d, lam0, w.f)

        def pol_oracle():
            m = oracle.jones_apply(E0, J_h) * lens0
            return oracle.propagate(m, w.d, w.d, lam0, w.z, oracle.FRESNEL, w.pad)
        print("[bench] polarized: FP64 oracle on one wavelength", file=sys.stderr, flush=True)
        rate, runs, secs = _oracle_rate(pol_oracle, 3, 3.0)
        exp = pol_oracle()
        got = outs[0].cpu().numpy()
        res["polarized_8x3x2048_c64"]["error_vs_oracle"] = {
            "wavelength_0_field": float(f"{np.linalg.norm(got - exp) / np.linalg.norm(exp):.3e}")}
        res["polarized_8x3x2048_c64"]["cpu_baseline"] = {
            "value": round(rate, 3), "unit": "propagations/s", "cores": host_threads(), "kind": "oracle",
            "sample": f"one wavelength forward (Jones, lens, three Fresnel component propagations of "
                      f"{w.n}^2 on {2 * w.n}^2) in FP64, {runs} runs in {secs:.1f} s"}
    del E, outs, grads

    c = workloads.CoherenceWorkload()
    G0 = torch.from_numpy(c.gamma()).to(dev)
    pg = torch.from_numpy(c.mask()).to(dev)
    T = torch.from_numpy(c.target()).to(dev)
    oc = tp.Optics(dy=c.d, dx=c.d, wavelength=c.wavelength, z=c.z, pad=c.pad)
    n = c.n
    gphi = torch.zeros_like(pg)

    def coherence():
        out, gG, L = tp.coherence_propagate(G0, oc, loss_kind="mse", loss_ref=T, loss_scale=1.0 / (n * n),
                                            phase=pg, lens_f=c.f)
        gphi.zero_()
        tp.coherence_propagate(gG, oc, adjoint=True, saved_in=G0, grad_phase=gphi, phase=pg, lens_f=c.f)
    ms, top = _timed(coherence, args.steps, args.warmup)
    slices = 4 * n * n
    prof = _timed.last_profile
    # the step's slice propagations split evenly over the launches of a pass
    col_launches = sum(cnt for name, (cnt, _) in prof.items() if ".col_" in name)

    def coh_fields(name, cnt):
        return slices // col_launches if col_launches and slices % col_launches == 0 else None
    res["gaussian_schell_64^4_c64"] = {"ms_per_step": round(ms, 3), "slice_propagations_per_step": slices,
                                        "slice_propagations_per_s": round(slices / (ms / 1000.0), 1),
                                        "kernels": top,
                                        "roofline": model_roofline(prof, n, 2 * n, coh_fields)}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        G_h = c.gamma().astype(np.complex128)
        print("[bench] coherence: FP64 oracle on the 64^4 forward propagation", file=sys.stderr, flush=True)
        rate, runs, secs = _oracle_rate(
            lambda: oracle.coherence_propagate(G_h, c.d, c.d, c.wavelength, c.z, oracle.ASM, c.pad), 2 * n * n, 2.0)
        res["gaussian_schell_64^4_c64"]["cpu_baseline"] = {
            "value": round(rate, 1), "unit": "slice propagations/s", "cores": host_threads(), "kind": "oracle",
            "sample": f"the unmodulated forward 4-D propagation ({2 * n * n} slice propagations of {n}^2 on "
                      f"{2 * n}^2) in FP64, {runs} runs in {secs:.1f} s"}
    del G0

    res["uneven_128_jobs_c64"] = run_uneven(args, dev)
    print(json.dumps({"metric": "other workloads: time per step", "unit": "ms", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "data": "synthetic (seeded, as in workloads/)", "configs": res}))
    return 0


def run_uneven(args, dev):
    """The uneven batch: 128 independent jobs (256^2 .. 4096^2, random
    wavelength, distance and spacing, ASM, 2x padding, complex64), one
    forward call and one backward call over all of them per step
    (`--uneven-sizes` / `--uneven-count` select a subset)."""
    import torch

    import paper_2411_18591_amd as tp
    import workloads
    jobs = workloads.uneven_jobs()
    if args.uneven_sizes:
        keep = {int(x) for x in args.uneven_sizes.split(",") if x}
        jobs = [j for j in jobs if j.n in keep]
    if args.uneven_count > 0:
        jobs = jobs[:args.uneven_count]
    us, gs, ops = [], [], []
    gen = torch.Generator(device=dev).manual_seed(5301)
    for j in jobs:
        us.append(torch.randn((j.n, j.n), dtype=torch.complex64, device=dev, generator=gen))
        gs.append(torch.randn((j.n, j.n), dtype=torch.complex64, device=dev, generator=gen))
        ops.append(tp.Optics(dy=j.d, dx=j.d, wavelength=j.wavelength, z=j.z, pad=2))
    uo = [torch.empty_like(x) for x in us]
    gi = [torch.empty_like(x) for x in gs]

    def uneven():
        tp.propagate_jobs(us, ops, outs=uo)
        tp.propagate_backward_jobs(gs, ops, grad_ins=gi)
    ms, top = _timed(uneven, args.steps, args.warmup)
    elems = sum(j.n * j.n for j in jobs)
    res = {"jobs": len(jobs), "ms_per_step": round(ms, 3), "propagations_per_step": 2 * len(jobs),
           "propagations_per_s": round(2 * len(jobs) / (ms / 1000.0), 1),
           "field_elements_per_job_sum": elems, "kernels": top, "roofline": uneven_roofline(top)}
    # The same step captured by the library into two HIP graphs that it owns
    # (the forward call and the adjoint call, every lane and job-queue launch
    # included; `to_graph_create`) and replayed: no host launch work per
    # kernel.  The replays' outputs must equal the eager step's bit for bit.
    torch.cuda.synchronize()
    ref = [t.clone() for t in uo + gi]
    _, g_fwd = tp.propagate_jobs(us, ops, outs=uo, graph=True)
    _, g_bwd = tp.propagate_backward_jobs(gs, ops, grad_ins=gi, graph=True)

    def replay():
        g_fwd.launch()
        g_bwd.launch()
    torch.cuda.synchronize()
    for t in uo + gi:
        t.zero_()
    ms_g, _ = _timed(replay, args.steps, 1)
    same = all(torch.equal(a, b) for a, b in zip(uo + gi, ref))
    res["graph"] = {"ms_per_step": round(ms_g, 3), "propagations_per_s": round(2 * len(jobs) / (ms_g / 1000.0), 1),
                    "outputs_equal_eager": same, "captured_by": "library (to_graph_create)"}
    g_fwd.close()
    g_bwd.close()
    del ref
    if not args.no_cpu_baseline:
        uneven()
        torch.cuda.synchronize()
        res.update(uneven_cpu_leg(jobs, us, gs, uo, gi))
    return res


def uneven_roofline(top):
    """Roofline entry of the uneven batch's dominant kernel (largest total
    GPU time): one launch covers one field of a square job padded to L x L
    (N = L / 2), whose nominal flops and algorithmic bytes `kernel_model`
    gives; launches on the four lanes overlap, so the per-launch time (and
    the fraction) is a lower bound on what the kernel reaches alone."""
    if not top:
        return None
    name, rec = next(iter(top.items()))
    try:
        L = int(name.rsplit("_L", 1)[1])
    except (IndexError, ValueError):
        return None
    m = kernel_model(name, {"n": L // 2, "padded": L}, 1)
    if not m:
        return None
    by, fl = m
    avg_s = rec["avg_us"] * 1e-6
    tfs, gbs = fl / avg_s / 1e12, by / avg_s / 1e9
    return {"bound": "alu", "achieved": round(tfs, 3), "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tfs / VALU_FP32_PEAK_TFLOPS, 4), "traffic": None, "kernel": name,
            "avg_us": rec["avg_us"], "hbm_view": {"achieved_GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}}


def uneven_cpu_leg(jobs, us, gs, uo, gi):
    """CPU-baseline leg of the uneven workload: the FP64 oracle on every job
    (the same inputs, copied to the host), timed on the host cores, and each
    job's relative L2 error of the library's output field and input gradient
    against it."""
    import numpy as np

    import oracle
    oracle.build()
    threads = host_threads()
    per_job, secs = [], 0.0
    print(f"[bench] uneven: FP64 oracle on {len(jobs)} jobs, {threads} threads", file=sys.stderr, flush=True)
    for k, j in enumerate(jobs):
        u = us[k].cpu().numpy().astype(np.complex128)
        g = gs[k].cpu().numpy().astype(np.complex128)
        t0 = time.perf_counter()
        eu = oracle.propagate(u, j.d, j.d, j.wavelength, j.z, oracle.ASM, 2)
        eg = oracle.propagate(g, j.d, j.d, j.wavelength, j.z, oracle.ASM, 2, adjoint=True)
        secs += time.perf_counter() - t0
        ru = float(np.linalg.norm(uo[k].cpu().numpy() - eu) / np.linalg.norm(eu))
        rg = float(np.linalg.norm(gi[k].cpu().numpy() - eg) / np.linalg.norm(eg))
        per_job.append({"job": k, "n": j.n, "u_out_rel_l2": float(f"{ru:.3e}"), "g_in_rel_l2": float(f"{rg:.3e}")})
        if k % 16 == 15:
            print(f"[bench] uneven: oracle {k + 1}/{len(jobs)} jobs, {secs:.1f} s", file=sys.stderr, flush=True)
    worst = {}
    for r in per_job:
        w = worst.setdefault(r["n"], [0.0, 0.0])
        w[0], w[1] = max(w[0], r["u_out_rel_l2"]), max(w[1], r["g_in_rel_l2"])
    return {"error_vs_oracle": {"bar": "c64 field <= 2e-5", "all_within_bar": all(
                max(r["u_out_rel_l2"], r["g_in_rel_l2"]) <= 2e-5 for r in per_job),
                                "worst_by_n": {str(n): {"u_out": w[0], "g_in": w[1]} for n, w in sorted(worst.items())},
                                "per_job": per_job},
            "cpu_baseline": {"value": round(2 * len(jobs) / secs, 3), "unit": "propagations/s", "cores": threads,
                             "kind": "oracle", "host_cpu": host_cpu_model(),
                             "sample": f"all {len(jobs)} jobs, forward and adjoint ({2 * len(jobs)} FP64 "
                                       f"propagations, {secs:.1f} s; lines of each transform shared among "
                                       f"the threads)"}}


def host_threads() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (the GPU machine sets it to its CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        return ""


def cpu_child(args):
    """Child-process leg of the CPU baseline (``--cpu-child OUT``): the FP64
    oracle on `--cpu-sample-fields` fields of the workload through the first
    `--cpu-sample-layers` layers, forward + MSE loss + backward, with the
    OpenMP thread count the parent put in OMP_NUM_THREADS.  Writes the
    wall time and the oracle's outputs to OUT (npz)."""
    import numpy as np

    import oracle
    import workloads
    wl_def = workloads.DiffractiveNetWorkload(batch=args.batch, n=args.n, layers=args.layers)
    u0_np, masks_np, target_np = load_inputs(wl_def)
    k, nl = args.cpu_sample_fields, args.cpu_sample_layers
    oracle.build()
    u0 = u0_np[:k].astype(np.complex128)
    phis = [m.astype(np.float64) for m in masks_np[:nl]]
    T = target_np.astype(np.float64)
    d, lam, z = wl_def.d, wl_def.wavelength, wl_def.z
    meth = oracle.DI if args.method == "di" else oracle.ASM
    t0 = time.perf_counter()
    us = oracle.stack_forward(u0, phis, d, d, lam, z, meth, 2)
    _, g = oracle.mse_intensity(us[-1], T)
    _, grads = oracle.stack_backward(us, phis, g, d, d, lam, z, meth, 2)
    dt = time.perf_counter() - t0
    np.savez(args.cpu_child, seconds=dt, u_out=us[-1], grads=np.stack(grads))
    return 0


def cpu_baseline(args, wl_def, method="ASM"):
    """The FP64 oracle timed on the host cores on a bounded sample of the
    same workload, in fresh CPU-only child processes started before this
    process touches the GPU: once with every host thread (one field per
    thread, the first `--cpu-sample-layers` layers, fwd + bwd) and once with
    one thread (one field, two layers).  Returns the cpu_baseline record and
    the all-threads sample's oracle outputs (for the parity check)."""
    import subprocess
    import tempfile

    import numpy as np
    threads = host_threads()
    nl = max(1, min(args.cpu_sample_layers, wl_def.layers))
    k = min(args.cpu_sample_fields or threads, wl_def.batch)
    runs = {}
    for tag, nthr, kk, ll in (("all", threads, k, nl), ("one", 1, 1, min(2, nl))):
        print(f"[bench] cpu baseline: oracle on {kk} fields x {ll} layers, {nthr} threads",
              file=sys.stderr, flush=True)
        fd, out = tempfile.mkstemp(suffix=".npz", prefix=f"toprop_cpu_{tag}_")
        os.close(fd)
        env = dict(os.environ, OMP_NUM_THREADS=str(nthr))
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", out, "--batch", str(args.batch),
               "--n", str(args.n), "--layers", str(args.layers), "--method", args.method,
               "--cpu-sample-fields", str(kk), "--cpu-sample-layers", str(ll)]
        subprocess.run(cmd, env=env, check=True)
        with np.load(out) as zf:
            runs[tag] = (float(zf["seconds"]), kk, ll, zf["u_out"], zf["grads"])
        os.unlink(out)
    dt, _, _, u_ref, g_ref = runs["all"]
    dt1 = runs["one"][0]
    props, props1 = 2 * k * nl, 2 * runs["one"][2]
    shape = f"{wl_def.n}^2 -> {2 * wl_def.n}^2"
    cpu = {"value": round(props / dt, 3), "unit": "propagations/s", "cores": min(k, threads),
           "kind": "oracle", "host_cpu": host_cpu_model(), "host_threads": threads,
           "sample": f"{k} of {wl_def.batch} fields through the first {nl} of {wl_def.layers} "
                     f"layers, fwd+bwd with MSE loss ({props} FP64 propagations at the same "
                     f"{shape} shape, {dt:.1f} s; OpenMP over fields, one field per thread)",
           "single_thread": {"value": round(props1 / dt1, 4), "unit": "propagations/s", "cores": 1,
                             "sample": f"1 field through {runs['one'][2]} layers, fwd+bwd "
                                       f"({props1} propagations, {dt1:.1f} s)"}}
    return cpu, (k, nl, u_ref, g_ref)


def parity_on_sample(sample, u0_np, masks_np, target_np, opt):
    """The library on the oracle's sample (same fields, masks, target and
    loss): relative L2 errors of the output field and the mask gradients."""
    import numpy as np
    import torch

    from paper_2411_18591_amd.diffnet import DiffractiveNet
    k, nl, u_ref, g_ref = sample
    dev = torch.device("cuda", 0)
    net = DiffractiveNet(torch.from_numpy(u0_np[:k]).to(dev), torch.from_numpy(masks_np[:nl]).to(dev),
                         torch.from_numpy(target_np).to(dev), opt)
    net.step()
    torch.cuda.synchronize()

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {"output_field_rel_l2": rel(net.u[nl].cpu().numpy(), u_ref),
            "mask_gradients_rel_l2": rel(net.gmask.cpu().numpy(), g_ref),
            "sample": f"the oracle's sample: {k} fields, {nl} layers", "bar": "c64 field <= 2e-5"}


if __name__ == "__main__":
    sys.exit(main())
