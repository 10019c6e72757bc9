"""Benchmark of the free-surface LBM time step on one MI355X.

Workload: the 512 x 320 x 512 sloshing tank (84 M cells, liquid depth 192 with a
cosine surface of amplitude 12, walls on all faces, g_y = -2e-5, tau = 0.55,
FSL rule), synthetic and seeded.  A step is one full time step: the fused
stream/collide/interface sweep and the conversion kernels.  Each precision form
(FP64, FP32 on shifted populations, FP16 storage of shifted populations) runs
`warmup` untimed and `steps` timed steps from the same initial state; the
velocity and fill errors of each form against the FP64 run are reported after
the same number of steps (relative L2 / L-infinity norms over cells that are
liquid or interface in both runs).

Printed: one JSON line.  `value` is the MLUPS (million active-cell updates per
second, active = liquid + interface) of the headline form (FP16 storage,
FP32 compute).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STORAGE_BYTES = {"fp64": 8, "fp32": 4, "fp16s": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16s": "f32"}
HEADLINE = "fp16s"
RULE_NAME = {0: "FSK", 1: "FSL", 2: "FSK with the shear-rate boundary term", 3: "FSL with the shear-rate boundary term"}
SWEEP_KERNEL = {"fp64": "k_sweep<FormF64, 1, false>", "fp32": "k_sweep<FormF32, 1, false>",
                "fp16s": "k_sweep_h2<1>"}


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("fslbm_device.hpp", "fslbm_internal.hpp", "fslbm_sweep.hip"):
        h.update(open(os.path.join(ROOT, "paper_1409_5645_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(form: str, n_cells: int):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source and a lattice of n_cells cells
    (else None)."""
    path = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != sweep_source_hash() or form not in d.get("forms", {}):
        return None
    if d.get("cells") != n_cells:
        return None
    return d["forms"][form].get("bytes_per_launch")


def errors(ref: dict, other: dict) -> dict:
    """Relative L2 and L-inf of u and phi (Eq. l2error, maxerror) over cells
    active in both runs; flag mismatch count."""
    import torch
    act = (ref["flags"] != 0) & (other["flags"] != 0)
    out = {"flag_mismatch": int((ref["flags"] != other["flags"]).sum().item())}
    for name in ("u", "phi"):
        a, b = other[name], ref[name]
        if name == "u":
            a, b = a[:, act], b[:, act]
        else:
            a, b = a[act], b[act]
        d = (a - b).double()
        out[f"{name}_l2"] = float(torch.sqrt((d * d).sum() / (b.double() * b.double()).sum()).item())
        out[f"{name}_linf"] = float((d.abs().max() / b.abs().max()).item())
    return out


def run_form(w, form, steps, warmup, rule, log, roof_steps=500):
    """Warm-up, then two timed regions on the context's stream: `steps` steps
    with nothing but the step kernels in the queue (the whole-step rate), and
    min(steps, roof_steps) more with HIP events around every sweep launch (its
    average duration for the roofline).  The events of the second region cost
    a few microseconds per step, so they stay out of the first."""
    import torch
    from paper_1409_5645_amd import fslbm
    t0 = time.time()
    s = fslbm.Sim.from_workload(w, precision=form)
    st0 = s.stats()
    log(f"[{form}] init {time.time() - t0:.1f}s, active {st0['liquid'] + st0['interface']}")
    s.step(warmup, rule)
    torch.cuda.synchronize()
    stream = s.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps, rule)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    st1 = s.stats()
    f = s.fields(("u", "phi", "flags"), device=True)
    # sweep launches timed with HIP events
    n_roof = max(1, min(steps, roof_steps))
    s.timing(True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.step(n_roof, rule)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_roof = e0.elapsed_time(e1)
    sweep_ms, nsweeps = s.timing(False)
    n_act = 0.5 * ((st0["liquid"] + st0["interface"]) + (st1["liquid"] + st1["interface"]))
    ms = ms_total / steps
    sweep_avg = sweep_ms / max(nsweeps, 1)
    alg_bytes = n_act * 38 * STORAGE_BYTES[form] + w.params.n_cells * 1
    res = {
        "mlups": n_act / (ms * 1e-3) / 1e6,
        "mlups_all_cells": w.params.n_cells / (ms * 1e-3) / 1e6,
        "ms_per_step": ms,
        "sweep_ms": sweep_avg,
        "sweep_share": sweep_avg / ms,
        "sweep_timed_steps": n_roof,
        "ms_per_step_with_sweep_events": ms_roof / n_roof,
        "active_cells": n_act,
        "alg_bytes_per_sweep": alg_bytes,
        "sweep_gbs": alg_bytes / (sweep_avg * 1e-3) / 1e9,
        "step_gbs": alg_bytes / (ms * 1e-3) / 1e9,
        "mass_drift": (st1["total_mass"] - st0["total_mass"]) / st0["total_mass"],
        "conversions_last_step": st1["filled"] + st1["emptied_converted"],
    }
    log(f"[{form}] {ms:.3f} ms/step, sweep {sweep_avg:.3f} ms, {res['mlups']:.0f} MLUPS, "
        f"{res['sweep_gbs']:.0f} GB/s alg. sweep, {res['step_gbs']:.0f} GB/s over the step")
    s.close()
    del s
    torch.cuda.empty_cache()
    return res, f


def adjoint_leg(log, T=400, config="slosh128"):
    """Adjoint window of T steps with frozen cell classes on the 128 x 96 x 128
    sloshing tank: FP32 (headline) and FP64 gradients of
    L = sum over interface cells of |u_T - u*|^2 + (phi_T - phi*)^2 with respect
    to f0, P_b and g; u*, phi* from a seed-generated target run (P_b and g scaled
    by 1 + 0.01 xi, f0 + 1e-4 w xi).  Cost = (window forward with checkpoints +
    backward) / (T plain frozen steps)."""
    import torch
    from paper_1409_5645_amd import fslbm, workloads as W
    w = W.config(config, seed=0)
    p = w.params
    rng = np.random.default_rng(11)
    xi1, xi2 = rng.normal(size=2)
    base_sim = fslbm.Sim.from_workload(w)
    base = base_sim.fields(("f", "mass", "phi", "flags"), device=True)
    base_sim.close()
    dev = base["f"].device
    iface = base["flags"] == 1
    act = (base["flags"] != 0).to(torch.float64)
    wq = torch.tensor([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=torch.float64, device=dev)
    gen = torch.Generator(device=dev).manual_seed(11)
    f_t = base["f"] + 1e-4 * wq[:, None] * torch.randn(base["f"].shape, dtype=torch.float64, device=dev,
                                                       generator=gen) * act
    tgt = fslbm.Sim(p, w.flags)
    tgt.set_state(f_t, base["mass"], base["phi"])
    tgt.set_forcing([v * (1 + 0.01 * xi2) for v in p.g], p.rho_gas * (1 + 0.01 * xi1))
    tgt.window(T, 1)
    tg = tgt.fields(("u", "phi"), device=True)
    tgt.close()
    C = torch.tensor([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (1, 1, 0),
                      (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1), (0, 1, 1),
                      (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=torch.float64, device=dev)

    def loss(fT, phiT, g):
        u = (C.T @ fT - g[:, None]) + 0.5 * g[:, None]
        return ((u - tg["u"]) ** 2).sum(0)[iface].sum() + ((phiT - tg["phi"]) ** 2)[iface].sum()

    out = {}
    for form in ("fp64", "fp32"):
        sim = fslbm.Sim(p, w.flags, precision=form, freeze=True)
        # T plain frozen steps
        sim.set_state(base["f"], base["mass"], base["phi"])
        sim.step(20, 1)
        sim.set_state(base["f"], base["mass"], base["phi"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(T, 1)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        def timed(K):
            f0 = base["f"].clone().requires_grad_(True)
            P_b = torch.tensor(p.rho_gas / 3.0, dtype=torch.float64, device=dev, requires_grad=True)
            g = torch.tensor(p.g, dtype=torch.float64, device=dev, requires_grad=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fT, mT, phiT = fslbm.window_apply(sim, T, 1, f0, base["mass"], base["phi"], P_b, g, K=K)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L = loss(fT, phiT, g)
            L.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            return {"L": float(L.detach()), "dL_dPb": float(P_b.grad), "dL_dg": g.grad.cpu().tolist(),
                    "f0_grad": f0.grad, "t_window_fwd_ms": (t1 - t0) * 1e3, "t_backward_ms": (t2 - t1) * 1e3}

        timed(0)  # warms the allocator
        res = timed(0)  # the default spacing (every record when it fits in memory)
        res["K"] = sim.last_window_K
        res["t_plain_ms"] = t_plain * 1e3
        res["cost_ratio"] = (res["t_window_fwd_ms"] + res["t_backward_ms"]) / res["t_plain_ms"]
        # sqrt(T) checkpointing: memory ~2 sqrt(T) states, one recompute pass
        ks = int(np.ceil(np.sqrt(T)))
        timed(ks)
        sq = timed(ks)
        res["sqrt_T"] = {"K": ks, "t_window_fwd_ms": sq["t_window_fwd_ms"], "t_backward_ms": sq["t_backward_ms"],
                         "cost_ratio": (sq["t_window_fwd_ms"] + sq["t_backward_ms"]) / res["t_plain_ms"],
                         "same_gradient": bool(torch.equal(sq["f0_grad"], res["f0_grad"]))}
        del sq
        out[form] = res
        sim.close()
        log(f"[adjoint {form}] plain {res['t_plain_ms']:.1f} ms, window fwd {res['t_window_fwd_ms']:.1f} ms, "
            f"bwd {res['t_backward_ms']:.1f} ms, cost x{res['cost_ratio']:.2f} (default spacing K={res['K']}; "
            f"sqrt(T) x{res['sqrt_T']['cost_ratio']:.2f}), dL/dP_b {res['dL_dPb']:.6e}")
    a, b = out["fp32"], out["fp64"]
    err = {"f0": float(torch.linalg.norm(a["f0_grad"] - b["f0_grad"]) / torch.linalg.norm(b["f0_grad"])),
           "P_b": abs(a["dL_dPb"] - b["dL_dPb"]) / abs(b["dL_dPb"]),
           "g": float(np.linalg.norm(np.subtract(a["dL_dg"], b["dL_dg"])) / np.linalg.norm(b["dL_dg"]))}
    for r in out.values():
        del r["f0_grad"]
    torch.cuda.empty_cache()
    return {"workload": f"sloshing tank {p.nx}x{p.ny}x{p.nz}, T = {T} steps with frozen cell classes, FSL, "
                        f"default checkpoint spacing (every step's record when it fits in half the free memory, "
                        f"else ceil(sqrt T))",
            "cost_ratio": out["fp32"]["cost_ratio"], "cost_ratio_sqrt_T": out["fp32"]["sqrt_T"]["cost_ratio"],
            "fp32_grad_err_vs_fp64": err, "forms": out}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def device_facts(torch) -> dict:
    """Name, compute units, memory and clocks of device 0 as the runtime reports them."""
    pr = torch.cuda.get_device_properties(0)
    facts = {"name": pr.name, "compute_units": pr.multi_processor_count,
             "memory_gib": round(pr.total_memory / 2 ** 30, 1)}
    for key in ("gcnArchName", "clock_rate", "memory_clock_rate", "l2_cache_size"):
        v = getattr(pr, key, None)
        if v is not None:
            facts[key] = v
    return facts


def cpu_baseline(w_full, log, budget_s=12.0, rule=1):
    """The serial FP64 oracle on a z-slab of the same tank (same x-y profile,
    walls on all faces), timed on one host core."""
    import oracle
    from paper_1409_5645_amd import workloads as W
    p = w_full.params
    nz = 16
    m = w_full.meta
    w = W.sloshing(p.nx, p.ny, nz, depth=m["depth"], amp=m["amp"], seed=m["seed"], gy=p.g[1], tau=p.tau,
                   Lambda=p.Lambda, wavelength=m["wavelength"])
    o = oracle.Oracle.from_workload(w)
    n_act = int((w.flags != 0).sum())
    t0 = time.time()
    o.step(1, rule)
    t1 = time.time() - t0
    n = max(1, int(budget_s / max(t1, 1e-3)) - 1)
    t0 = time.time()
    o.step(n, rule)
    dt = time.time() - t0
    mlups = n_act * n / dt / 1e6
    log(f"[cpu oracle] {n} steps of {p.nx}x{p.ny}x{nz}: {mlups:.2f} MLUPS")
    return {"value": mlups, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "cpu": f"{cpu_model()}, {os.cpu_count()} logical cores present, 1 used",
            "sample": f"{n} {RULE_NAME[rule]} steps (after 1 untimed) of a {p.nx}x{p.ny}x{nz} z-slab of the same tank "
                      f"({n_act} active cells), serial FP64 oracle, 1 thread"}


def copy_calibration(nbytes: int) -> None:
    """A plain device copy of a known size, five dispatches: the reference for
    the HBM traffic counters (rocprofv3 --pmc FETCH_SIZE, and in a run of its
    own WRITE_SIZE).  Every dispatch reads and writes exactly nbytes, so a
    counter divided by nbytes is the factor by which it reports bytes on this
    GPU."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    reps = 5
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "dispatches": reps, "check": float(b[-1])}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)  # the run length of the tank configurations
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--roof-steps", type=int, default=500,
                    help="steps of the second timed region (HIP events around each sweep launch)")
    ap.add_argument("--forms", default="fp64,fp32,fp16s")
    ap.add_argument("--config", default="slosh512")
    ap.add_argument("--rule", type=int, default=1)
    ap.add_argument("--sigma", type=float, default=0.0)  # surface tension (0: none)
    ap.add_argument("--plic", type=int, default=0)  # interface position / height functions (0, 1, 2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="NBYTES",
                    help="only run the counter-calibration copy of NBYTES bytes (e.g. 1073741824) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)

    def log(msg):
        if not args.quiet:
            print(msg, file=sys.stderr, flush=True)

    import torch
    from paper_1409_5645_amd import fslbm, workloads as W
    if not os.path.exists(fslbm.LIB_PATH):
        from paper_1409_5645_amd import build
        build.build()
    t0 = time.time()
    w = W.config(args.config, seed=0)
    if args.sigma != 0.0 or args.plic != 0:
        import dataclasses
        w = dataclasses.replace(w, params=dataclasses.replace(w.params, sigma=args.sigma, plic=args.plic))
    log(f"workload {w.name} {w.params.nx}x{w.params.ny}x{w.params.nz} generated in {time.time() - t0:.1f}s "
        f"{w.counts()}")
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    results, fieldsets = {}, {}
    for form in forms:
        results[form], fieldsets[form] = run_form(w, form, args.steps, args.warmup, args.rule, log,
                                                   roof_steps=args.roof_steps)
    if "fp64" in fieldsets:
        for form in forms:
            if form != "fp64":
                results[form]["err_vs_fp64"] = errors(fieldsets["fp64"], fieldsets[form])
    fieldsets.clear()
    torch.cuda.empty_cache()

    head = HEADLINE if HEADLINE in results else forms[-1]
    r = results[head]
    traffic = traffic_for(head, w.params.n_cells)
    roof = {"bound": "hbm", "achieved": r["sweep_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": r["sweep_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": SWEEP_KERNEL[head],
            "bytes_per_launch": r["alg_bytes_per_sweep"], "avg_launch_ms": r["sweep_ms"],
            "timed_launches": r["sweep_timed_steps"],
            # the sweep's algorithmic bytes over the whole step (interface and
            # conversion kernels included)
            "step_frac": r["step_gbs"] / HBM_PEAK_GBS}
    for form in forms:
        results[form]["roofline_frac"] = results[form]["sweep_gbs"] / HBM_PEAK_GBS
        results[form]["step_roofline_frac"] = results[form]["step_gbs"] / HBM_PEAK_GBS
    line = {
        "metric": "MLUPS + % HBM roofline per form (FP64/FP32/FP16-store, FSL) at stated err vs FP64",
        "value": r["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "storage": "f16" if head == "fp16s" else DTYPE[head],
        "data": "synthetic",
        "config": {"workload": f"sloshing tank {w.params.nx}x{w.params.ny}x{w.params.nz} "
                               f"(depth {w.meta['depth']:g}, amplitude {w.meta['amp']:g}, seed 0), {RULE_NAME[args.rule]} rule, "
                               f"tau {w.params.tau}, g_y {w.params.g[1]:g}"
                               + (f", sigma {w.params.sigma:g}" if w.params.sigma else "")
                               + (f", plic {w.params.plic}" if w.params.plic else ""),
                   "cells": w.params.n_cells, "active_cells": r["active_cells"], "form": head},
        "roofline": roof,
        "err_after_steps": args.warmup + args.steps,  # errors vs FP64 compare the final states
        "forms": results,
        "device": device_facts(torch),
    }
    if not args.no_adjoint:
        line["adjoint"] = adjoint_leg(log)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, log, rule=args.rule)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
