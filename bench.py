#!/usr/bin/env python3
"""Benchmark of the IMEX PD-ARS radiation step on one MI355X.

Headline workload (a "step" is one full PD-ARS radiation step: both fused stage
kernels, transport + local implicit source, over the whole grid): the 3-D 256^3
dynamic-diffusion grid (periodic; uniform v = 0.01 c along x; 8 x-slabs with
tau_cell in {0.1, 10, 1000}; Gaussian temperature bump of 16 cells; chat = c/50;
300 steps), in FP64, with the mixed-precision step on the same inputs beside it.
Inputs are synthetic and resident in HBM before any timed region. Prints one
JSON line.

Timing protocol
  warm-up   --warmup steps, then more steps until at least --warmup-seconds of
            GPU time have passed (steady clocks), on a scratch copy of the state
  value     cells * K / median over --repeats calls of rhd_step(K steps), each
            call started from the workload's initial state (reset outside the
            timed region) and bracketed by one hipEvent pair on the library's
            stream (the error-word readback at the end of the call included)
  roofline  algorithmic HBM bytes of the dominant stage kernel per launch over
            its average duration, from a separate rhd_step_timed call of K steps
            (per-launch hipEvents on the library's stream; not part of `value`)
  valu      the same kernel against the FP64 vector peak (78.6 TFLOP/s), with the
            FP64 FLOPs per launch of the committed rocprofv3 counter summary (null
            when the kernel sources have changed since the counters were taken,
            like roofline.traffic)
  cpu_baseline  the CPU oracle (OpenMP over cells) on the first --cpu-steps steps
            of the same workload, rate per step extrapolated (rank 0, N = 1)
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
PROFILE = os.path.join(ROOT, "profiles", "k_stage_c3_256cubed_fp64.md")
HEADLINE = "3-D 256^3 dynamic diffusion, periodic, v = 0.01 c, chat = c/50, 300 steps"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("rhd_stage.hpp", "rhd_forward.hip", "rhd_device.hpp", "rhd_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2404_08247_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_per_launch(kind, kernel):
    """A per-launch counter figure of `kernel` from the committed counter summary
    (kind: "traffic_bytes_per_launch" = HBM bytes, "fp64_flops_per_launch" = FP64
    VALU FLOPs), or None if that summary was taken on different kernel sources."""
    try:
        txt = open(PROFILE).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if line.startswith("kernel_source_sha256:"):
            vals["hash"] = line.split(":", 1)[1].strip()
        elif line.startswith(kind + " "):
            k, v = line[len(kind) + 1:].rsplit(":", 1)
            vals[k.strip()] = float(v)
    if vals.get("hash") != kernel_source_hash():
        return None
    return vals.get(kernel)


def stage_bytes_per_cell(ndim):
    """Compulsory float64 HBM traffic per cell of each stage kernel.
    Stage 1 reads y^n (nvar) + rho + kappa and writes y^{n+1/2} (nvar);
    stage 2 reads y^{n+1/2} (nvar) + y^n (nvar) + rho + kappa and writes y^{n+1}."""
    nvar = 2 + 2 * ndim
    return 8 * (nvar + 2 + nvar), 8 * (2 * nvar + 2 + nvar)


def cpu_model():
    """Model name of the host CPU with its family / model numbers (some virtual
    machines report only a generic name) and the logical CPUs visible."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if fields:
                        break
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                fields.setdefault(k, v)
    except OSError:
        return "unknown"
    name = fields.get("model name", "unknown")
    fam, mod = fields.get("cpu family"), fields.get("model")
    if fam is not None and mod is not None:
        name += f" (family {fam}, model {mod})"
    return f"{name}, {os.cpu_count()} logical CPUs visible"


def _wall(torch, fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t


def event_timed(torch, S, y, y0, dt, nsteps, repeats):
    """`repeats` calls of rhd_step(nsteps) on y, each from y0 (copied in outside
    the timed region), each timed by one hipEvent pair on the solver's stream and
    by the host clock around it. Returns (event seconds, wall seconds) lists."""
    ev_s, wall_s = [], []
    for _ in range(repeats):
        y.copy_(y0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(S.stream)
        S.step(y, dt, nsteps)
        e1.record(S.stream)
        torch.cuda.synchronize()
        wall_s.append(time.perf_counter() - t0)
        ev_s.append(e0.elapsed_time(e1) * 1e-3)
    return ev_s, wall_s


def warm_up(torch, S, y, y0, dt, nsteps, seconds):
    """nsteps steps, then batches of steps until `seconds` of wall time have passed."""
    y.copy_(y0)
    t0 = time.perf_counter()
    if nsteps > 0:
        S.step(y, dt, nsteps)
    torch.cuda.synchronize()
    batch = max(1, nsteps)
    while time.perf_counter() - t0 < seconds:
        y.copy_(y0)
        S.step(y, dt, batch)
        torch.cuda.synchronize()


def measure(torch, rhd, w, dev, to, steps, warmup, warmup_s, repeats, label):
    """Throughput of rhd_step on workload w (the protocol of the module docstring).
    Returns (line item, solver, state after the last timed call, y0 on device)."""
    rho, kap = to(w.rho), to(w.kappa_P)
    y0 = to(w.y0)
    y = y0.clone()
    S = rhd.Solver(w.params, rho, kap, None, 0, dev)
    S._keep = (rho, kap)
    warm_up(torch, S, y, y0, w.dt, warmup, warmup_s)
    ev, wall = event_timed(torch, S, y, y0, w.dt, steps, repeats)
    med = statistics.median(ev)
    item = {"value": w.ncells * steps / med, "unit": "cell-updates/s",
            "ms_per_step": med / steps * 1e3, "steps_per_call": steps, "calls": repeats,
            "call_ms_event": [t * 1e3 for t in ev], "call_ms_wall": [t * 1e3 for t in wall]}
    print(f"[bench] {label}: {med / steps * 1e3:.4f} ms/step (median of {repeats} calls of "
          f"{steps} steps; spread {min(ev) / steps * 1e3:.4f}..{max(ev) / steps * 1e3:.4f})",
          file=sys.stderr, flush=True)
    return item, S, y, y0


def stage_times(S, y, y0, dt, steps):
    """Average stage-1 / stage-2 kernel durations (s) over a separate call."""
    y.copy_(y0)
    ms1, ms2 = S.step_timed(y, dt, steps)
    return ms1 / steps * 1e-3, ms2 / steps * 1e-3


def bench_c1(torch, rhd, W, dev, to, repeats):
    """1-D 256 cells, reflecting walls, FP64, 1000 steps (launch-latency bound)."""
    w = W.config1()
    item, S, _, _ = measure(torch, rhd, w, dev, to, w.nsteps, 50, 0.3, repeats, "c1 fp64")
    item["us_per_step"] = item["ms_per_step"] * 1e3
    item["workload"] = "1-D 256 cells, reflecting, FP64, chat = c, 1000 steps"
    return item


def bench_c2(torch, rhd, W, dev, to, repeats):
    """3-D 128^3 static mixed-regime grid, FP64, 200 steps."""
    w = W.config2(precision="fp64")
    item, S, y, y0 = measure(torch, rhd, w, dev, to, w.nsteps, 20, 0.5, repeats, "c2 fp64")
    t1, t2 = stage_times(S, y, y0, w.dt, w.nsteps)
    item["stage_us"] = [t1 * 1e6, t2 * 1e6]
    item["workload"] = "3-D 128^3 static mixed-regime grid, periodic, FP64, chat = c/100, 200 steps"
    return item


def bench_c5_forward(torch, rhd, W, dev, to, repeats):
    """3-D 320^3 mixed precision, 100 forward steps (no checkpoint copies)."""
    w = W.config5(precision="mixed")
    item, S, y, y0 = measure(torch, rhd, w, dev, to, w.nsteps, 5, 0.5, repeats, "c5 mixed forward")
    item["workload"] = "3-D 320^3 turbulent velocity field, periodic, mixed precision, chat = c/100, 100 steps"
    del S, y, y0
    torch.cuda.empty_cache()
    return item


def bench_options(torch, rhd, W, dev, to, nsteps=50):
    """The 128^3 FP64 workload with each optional part of the step switched on
    (one at a time), and the Marshak wave (60 cells, 5451 steps at CFL 10): rate
    and time per step, and the ratio to the plain step's time."""
    base = W.config2(precision="fp64")
    rng = np.random.default_rng(77)
    kE = base.kappa_P * 10.0 ** rng.uniform(-0.5, 0.5, base.kappa_P.shape)
    kF = base.kappa_P * 10.0 ** rng.uniform(-0.5, 0.5, base.kappa_P.shape)
    jS = rng.uniform(0.0, 0.1, base.kappa_P.shape) * base.y0[0] / (200 * base.dt)
    Ein = 2.0 * base.y0[0].max()
    inflow = dict(bc=(2, 0, 0), inflow_E=Ein, inflow_F=0.3 * Ein)
    cases = {
        "plain": ({}, None, False),
        "rk2ssp": ({"scheme": "rk2ssp"}, None, False),
        "hll_eps_2cells": ({"hll_eps_cells": 2.0}, None, False),
        "kappa_F_order2": ({}, kF, False),
        "kappa_E_and_source": ({}, None, True),
        "T_pow_-3_inflow_x": (dict(kappa_T_power=-3.0, newton_maxit=400, **inflow), None, False),
    }
    out = {"workload": f"3-D 128^3 static mixed-regime grid, FP64, {nsteps} steps per option"}
    t_plain = None
    for name, (over, kf, kes) in cases.items():
        p = dict(base.params, **over)
        S = rhd.Solver(p, to(base.rho), to(base.kappa_P), None if kf is None else to(kf), 0, dev)
        if kes:
            kEd, jd = to(kE), to(jS)
            S.set_kappa_E(kEd)
            S.set_radiation_source(jd)
        y = to(base.y0)
        S.step(y, base.dt, 3)
        dt_s = _wall(torch, lambda: S.step(y, base.dt, nsteps))
        if t_plain is None:
            t_plain = dt_s
        out[name] = {"value": base.ncells * nsteps / dt_s, "unit": "cell-updates/s",
                     "ms_per_step": dt_s / nsteps * 1e3, "time_vs_plain": dt_s / t_plain}
        print(f"[bench] option {name}: {dt_s / nsteps * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        del S
    w = W.marshak(cfl=10.0)
    S = rhd.Solver(w.params, to(w.rho), to(w.kappa_P), None, 0, dev)
    y = to(w.y0)
    S.step(y, w.dt, 10)
    y = to(w.y0)
    dt_s = _wall(torch, lambda: S.step(y, w.dt, w.nsteps))
    out["marshak_60_cfl10"] = {"steps": w.nsteps, "seconds": dt_s,
                               "us_per_step": dt_s / w.nsteps * 1e6}
    print(f"[bench] marshak: {dt_s:.3f} s for {w.nsteps} steps", file=sys.stderr, flush=True)
    return out


def bench_hydro(torch, rhd, W, dev, to, nsteps=20):
    """Operator-split radiation hydrodynamics on the 3-D 128^3 workload with a
    moving gas (rough density, velocities up to 0.5 c_s): hydro steps alone, and
    split steps with 4 radiation subcycles per hydro step."""
    w = W.config2(precision="fp64")
    rng = np.random.default_rng(91)
    p = w.params
    cv = p["kB_over_mu"] / (p["gamma"] - 1.0)
    T = w.y0[4] / (w.rho * cv)
    rho = w.rho * (1.0 + 0.3 * rng.uniform(-1, 1, w.rho.shape))
    cs = np.sqrt(p["gamma"] * p["kB_over_mu"] * T)
    y = w.y0.copy()
    v = [0.5 * cs * rng.uniform(-1, 1, rho.shape) for _ in range(3)]
    for k in range(3):
        y[5 + k] = rho * v[k]
    y[4] = rho * cv * T + 0.5 * rho * sum(vk ** 2 for vk in v)
    rd = to(rho)
    S = rhd.Solver(p, rd, to(w.kappa_P), None, 0, dev)
    yd = to(y)
    smax = S.hydro_signal_speed(yd)
    dt_h = 0.3 * p["dx"] / smax
    nsub = 4
    S.hydro_step(yd, dt_h, 2)
    t_h = _wall(torch, lambda: S.hydro_step(yd, dt_h, nsteps))
    rd.copy_(to(rho))
    yd.copy_(to(y))
    S.rhd_step(yd, dt_h, nsub, 1)
    t_s = _wall(torch, lambda: S.rhd_step(yd, dt_h, nsub, nsteps))
    cells = w.ncells
    print(f"[bench] hydro: {t_h / nsteps * 1e3:.3f} ms/step; split (1 hydro + {nsub} radiation): "
          f"{t_s / nsteps * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    return {"workload": "3-D 128^3 mixed-regime grid with moving gas (|v| <= 0.5 c_s, density "
                        "+-30 %), FP64, hydro CFL 0.3",
            "hydro": {"value": cells * nsteps / t_h, "unit": "cell-updates/s",
                      "ms_per_step": t_h / nsteps * 1e3},
            "split": {"value": cells * nsteps / t_s, "unit": "cell-updates/s (hydro steps)",
                      "ms_per_step": t_s / nsteps * 1e3, "radiation_subcycles": nsub}}


def bench_adjoint(torch, rhd, W, dev, to, config=4):
    """Adjoint workloads: config 4, 2-D 512^2 FP64 (200 steps, checkpoints every 20,
    J = sum of E over the central 64^2 patch), or config 5, 3-D 320^3 mixed precision
    (100 steps, checkpoints every 10, J over the central 64^3 block). Forward with
    checkpoint copies, then the full backward (recompute + reverse of every
    segment), gradients with respect to kappa and the initial temperature."""
    from paper_2404_08247_amd import autograd as AG
    w = W.config4() if config == 4 else W.config5()
    p = w.params
    nd = w.ndim
    cv = p["kB_over_mu"] / (p["gamma"] - 1)
    ke = (w.y0[2 + nd:] ** 2).sum(axis=0) / (2 * w.rho)
    T0 = to((w.y0[1 + nd] - ke) / (w.rho * cv))
    rho, kap = to(w.rho), to(w.kappa_P)
    mom, mask = to(w.y0[2 + nd:]), to(w.objective_mask.astype(np.float64))
    w.y0 = None
    S = rhd.Solver(p, rho, kap, None, w.ckpt_every, dev)
    kap.requires_grad_(True)
    T = T0.clone().requires_grad_(True)
    F = torch.zeros((nd,) + tuple(T0.shape), dtype=T0.dtype, device=dev)
    AG.patch_energy_gradients(p, T0, mom, rho, kap, mask, w.dt, 4, 2, S)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y0 = AG.initial_state(T, T, F, mom, rho, p)
    yN = AG.RHDFunction.apply(y0, kap, S, w.dt, w.nsteps, w.ckpt_every)
    J = (yN[0] * mask).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gT, gk = torch.autograd.grad(J, [T, kap])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd, bwd = t1 - t0, t2 - t1
    print(f"[bench] c{config} adjoint: forward {fwd * 1e3:.1f} ms, backward {bwd * 1e3:.1f} ms",
          file=sys.stderr, flush=True)
    desc = ("2-D 512^2, FP64, periodic, chat = c, 200 steps, checkpoints every 20" if config == 4 else
            "3-D 320^3, mixed precision (float32 transport stencil and transport adjoint, FP64 "
            "source and its transposed-Jacobian solve), periodic, chat = c/100, 100 steps, "
            "checkpoints every 10")
    out = {"workload": desc, "forward_s": fwd, "backward_s": bwd, "adjoint_forward_ratio": bwd / fwd,
           "forward_cell_updates_per_s": w.ncells * w.nsteps / fwd,
           "J": float(J.item()), "grad_norm_kappa": float(gk.norm().item()),
           "grad_norm_T0": float(gT.norm().item())}
    del S, yN, y0, gT, gk, J
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300,
                    help="steps per timed rhd_step call (the workload's 300 by default)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--warmup-seconds", type=float, default=1.0,
                    help="minimum warm-up time before the timed calls")
    ap.add_argument("--repeats", type=int, default=5, help="timed calls (the median is reported)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--cpu-steps", type=int, default=10,
                    help="oracle steps of the CPU-baseline sample on the headline workload (0 = skip)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra line items (same as --extras none)")
    ap.add_argument("--extras", default="mixed,c1,c2,c5,adjoint,adjoint5,options,hydro",
                    help="comma list of extra line items: mixed (the headline workload in mixed "
                         "precision), c1, c2, c5 (forward), adjoint (config 4), adjoint5 (config 5), "
                         "options, hydro, or none")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the timed region, copy a MIB-mebibyte buffer once (a plain copy "
                         "kernel of known size, to scale the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; the multi-GPU path (halo exchange over xGMI) "
              "is a design, not implemented. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.repeats < 1:
        print("bench.py: --steps and --repeats must be >= 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_08247_amd import rhd, workloads as W

    dev = torch.device("cuda:0")
    w = W.config3(precision=args.precision)
    print(f"[bench] workload {w.name} cells={w.ncells} steps={args.steps} warmup={args.warmup} "
          f"repeats={args.repeats}", file=sys.stderr, flush=True)

    def to(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    if args.calibrate_copy > 0:
        nb = args.calibrate_copy * (1 << 20)
        a = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {nb} bytes done", file=sys.stderr, flush=True)
        del a, b

    head, S, y, y0 = measure(torch, rhd, w, dev, to, args.steps, args.warmup, args.warmup_seconds,
                             args.repeats, f"c3 {args.precision}")
    t1, t2 = stage_times(S, y, y0, w.dt, args.steps)
    cells = w.ncells
    b1, b2 = stage_bytes_per_cell(w.ndim)
    tt = "double" if args.precision == "fp64" else "float"
    if t2 >= t1:
        kname, kb, kt = "k_stage<3,STAGE2>", b2, t2
    else:
        kname, kb, kt = "k_stage<3,STAGE1>", b1, t1
    traffic = measured_per_launch("traffic_bytes_per_launch", kname) if args.precision == "fp64" else None
    flops = measured_per_launch("fp64_flops_per_launch", kname) if args.precision == "fp64" else None
    achieved = kb * cells / kt / 1e9
    print(f"[bench] stage1 {t1 * 1e6:.1f} us  stage2 {t2 * 1e6:.1f} us  (rhd_step_timed, "
          f"{args.steps} steps)", file=sys.stderr, flush=True)

    extras = {}
    want = set() if args.no_extras else set(args.extras.split(","))
    if "mixed" in want:
        other = "mixed" if args.precision == "fp64" else "fp64"
        wm = W.config3(precision=other)
        item, Sm, ym, _ = measure(torch, rhd, wm, dev, to, args.steps, args.warmup,
                                  args.warmup_seconds, args.repeats, f"c3 {other}")
        m1, m2 = stage_times(Sm, ym, to(wm.y0), wm.dt, args.steps)
        # both states now hold K steps from the same initial state
        a, b = (ym, y) if other == "mixed" else (y, ym)
        errs = [float(((a[v] - b[v]).abs().max() / b[v].abs().max()).item()) for v in range(a.shape[0])]
        item["stage_us"] = [m1 * 1e6, m2 * 1e6]
        ref = head if other == "mixed" else item
        mix = item if other == "mixed" else head
        extras["mixed_vs_fp64"] = {
            "workload": HEADLINE + " (same inputs, same protocol)", other: item,
            "speedup_mixed_over_fp64": ref["ms_per_step"] / mix["ms_per_step"],
            "max_rel_err_vs_fp64_per_field": errs,
            "error_note": f"L-inf of (mixed - FP64) over max |FP64| per field after {args.steps} steps"}
        del Sm, ym
        torch.cuda.empty_cache()
    if "c1" in want:
        extras["c1"] = bench_c1(torch, rhd, W, dev, to, args.repeats)
    if "c2" in want:
        extras["c2"] = bench_c2(torch, rhd, W, dev, to, args.repeats)
    del S, y, y0
    torch.cuda.empty_cache()
    if "c5" in want:
        extras["c5_forward"] = bench_c5_forward(torch, rhd, W, dev, to, 3)
    if "adjoint" in want:
        extras["adjoint"] = bench_adjoint(torch, rhd, W, dev, to, 4)
    if "adjoint5" in want:
        extras["adjoint_c5"] = bench_adjoint(torch, rhd, W, dev, to, 5)
    if "options" in want:
        extras["options"] = bench_options(torch, rhd, W, dev, to)
    if "hydro" in want:
        extras["hydro_coupling"] = bench_hydro(torch, rhd, W, dev, to)

    cpu = None
    if args.cpu_steps > 0:
        import oracle
        wc = W.config3(precision="fp64")
        tc = time.perf_counter()
        _, st, _ = oracle.step(wc.params, wc.y0, wc.rho, wc.kappa_P, None, wc.dt, args.cpu_steps)
        tcpu = time.perf_counter() - tc
        cpu = {"value": wc.ncells * args.cpu_steps / tcpu, "unit": "cell-updates/s",
               "cores": oracle.num_threads(), "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"first {args.cpu_steps} of the 300 steps of the same 256^3 workload in "
                         f"FP64 (OpenMP over cells), {tcpu:.1f} s; rate per step extrapolated to "
                         f"the full run"}
        print(f"[bench] cpu oracle: {args.cpu_steps} steps in {tcpu:.1f} s", file=sys.stderr,
              flush=True)

    line = {
        "metric": "IMEX RHD cell-updates/s, FP64 vs mixed; adjoint/forward time ratio",
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": HEADLINE, "cells": cells, "precision": args.precision,
                   "steps_per_call": args.steps, "timed_calls": args.repeats,
                   "statistic": "median of hipEvent-timed calls",
                   "call_ms_event": head["call_ms_event"], "call_ms_wall": head["call_ms_wall"]},
        "roofline": {"bound": "hbm", "kernel": f"k_stage<3,{kname[-7:-1]},{tt}>",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated)",
                     "algorithmic_bytes_per_launch": kb * cells, "bytes_per_cell": kb,
                     "avg_launch_us": kt * 1e6, "stage_us": [t1 * 1e6, t2 * 1e6]},
        "valu": None if flops is None else {
            "bound": "alu", "kernel": kname, "fp64_flops_per_launch": flops,
            "achieved": flops / kt / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": flops / kt / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "flops_source": "rocprofv3 SQ_INSTS_VALU_FLOPS_FP64 per dispatch (profiles/)"},
        "cpu_baseline": cpu,
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
