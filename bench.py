#!/usr/bin/env python3
"""Throughput of the fused D2Q9 collide-and-stream step with the Ehrenfest
limiter on the periodic double shear layer (4096 x 4096, nu = 1e-5, LBGK,
top 0.1 % of sites by nonequilibrium entropy sent to equilibrium each step),
and of its adjoint.

One JSON line on stdout:
  value     whole-step throughput in MLUPS (million lattice-site updates per
            second), inputs resident in HBM, timed over --steps steps of
            lbm_step (graph replays of 16 steps, eager launches for the rest);
  roofline  the fused step kernel's algorithmic bytes (read 9 populations,
            write 9, per site) over its average duration from HIP events
            recorded around each launch inside the timed region, against
            the MI355X HBM peak of 8 TB/s (from a separate profiled run
            of the same length), and the whole step's bytes over its time;
  forms     the same workload with FP64 and shifted FP16/BF16 storage, each
            run for the same number of steps as the FP32 line, with the
            relative L2 error of rho and u against the FP64 run;
  adjoint   the 512^2 lid-driven cavity (MRT with a per-site shear rate,
            Ehrenfest k = 9), 8192 steps forward and the adjoint with
            checkpoints every 256 steps, in FP32 and FP64; the FP32
            gradients' error against the FP64 ones;
  adjoint_scale  forward and adjoint of the shear-layer workload (FP32,
            128 steps, checkpoints every 16), with the adjoint kernel's
            bytes over its event-timed duration;
  elbm_8192 the 8192^2 ELBM workload (positivity, Ehrenfest 0.1 %, FP16
            shifted storage): forward MLUPS and branch statistics, forward +
            adjoint over 32 steps, and the workspace of its full 5000-step
            adjoint;
  median3d_256  the 256^3 D3Q27 Taylor-Green vortex with the 27-site median
            filter (FP32), at the workload's delta = 1e-3 and at delta = 0
            (every site ranks its neighbourhood): MLUPS and the step kernel's
            algorithmic bytes (27 populations read and written) over its
            event-timed duration;
  nonlocal_4096  the 4096^2 shear layer with the general nonlocal filter
            (binomial 3 x 3 smoothing of f_neq, FP32): MLUPS and the step
            kernel against HBM;
  cpu_baseline  the FP64 oracle timed on this host: two full steps on all
            threads, and one step of a 1024-row band on one thread.
Progress goes to stderr.
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

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the FP32 step kernel on this workload (periodic
# one-site kernel, LBGK + Ehrenfest): rocprofv3 FETCH_SIZE and WRITE_SIZE
# medians over 45 launches, scaled by what the counters read for a device
# copy of 1,207,959,552 bytes (FETCH x 2.0, WRITE x 1.0); summary in
# profiles/hbm_traffic_k_step_shear_layer_4096_f32.md.  Retake after any
# change of the kernel.
HBM_TRAFFIC_F32 = 648_124_928 + 607_071_936
ELEM = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
METRIC = "MLUPS and % HBM roofline, D2Q9 fwd+adjoint, FP64 vs FP32/FP16-storage at stated err"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(w: dict, storage: str, steps: int, warmup: int) -> tuple:
    import torch

    from lbm_inputs import generators as G
    from paper_1110_0270_amd import lbm as B

    cfg = B.make_config(**{**w, "storage": storage})
    sim = B.Simulation(cfg)
    rho, ux, uy = G.double_shear_layer(w["nx"])
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    sim.set_equilibrium(t(rho), t(ux), t(uy))
    sim.step(warmup)
    # the timed steps: lbm_step as a caller runs it (groups of 16 steps replay
    # the graphs captured at lbm_init, the rest launch eagerly)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sim.stats(allow_status=(B.LBM_OK, B.LBM_EDIVERGED, B.LBM_ESELECT))
    mom = sim.moments()
    # the step kernel's duration: HIP events at the kernel's own start and
    # end on the library's stream, over the same number of further steps
    kern_ms, prof_total_ms = sim.profile_step(steps)
    torch.cuda.synchronize()
    n_sites = w["nx"] * w["ny"]
    ms_step = (t1 - t0) * 1e3 / steps
    kern_avg = kern_ms / steps
    alg_bytes = 2 * 9 * ELEM[storage] * n_sites
    res = {
        "storage": storage,
        "ms_per_step": ms_step,
        "mlups": n_sites / (ms_step * 1e-3) / 1e6,
        "whole_step_gbs": alg_bytes / (ms_step * 1e-3) / 1e9,
        "kernel_ms": kern_avg,
        "kernel_gbs": alg_bytes / (kern_avg * 1e-3) / 1e9,
        "profiled_ms_per_step": prof_total_ms / steps,
        "alg_bytes_per_launch": alg_bytes,
        "n_selected": int(st.n_selected),
        "select_fallbacks": int(st.select_fallbacks),
        "candidates_per_step": round(st.select_candidates / max(1, steps + warmup), 1),
        "diverged_step": int(st.diverged_step),
        "mass": st.mass,
    }
    del sim
    torch.cuda.empty_cache()
    return res, mom


def rel_l2(a, b) -> float:
    return float(((a - b).norm() / b.norm().clamp(min=1e-300)).item())


def velocity_loss_grad(f, tx, ty):
    """L = sum_x |u(x) - u_t(x)|^2 of the final state and dL/df:
    dL/df_i = 2 (u - u_t) . (v_i - u) / rho (velocity i = 3 (b+1) + (a+1))."""
    import torch
    rho = f.sum(0)
    v = torch.tensor([[(i % 3) - 1, (i // 3) - 1] for i in range(9)], dtype=f.dtype,
                     device=f.device)
    ux = (v[:, 0].view(9, 1, 1) * f).sum(0) / rho
    uy = (v[:, 1].view(9, 1, 1) * f).sum(0) / rho
    ex, ey = ux - tx, uy - ty
    loss = float((ex * ex + ey * ey).sum())
    g = 2 * (ex * (v[:, 0].view(9, 1, 1) - ux) + ey * (v[:, 1].view(9, 1, 1) - uy)) / rho
    return loss, g.contiguous()


def run_adjoint(w: dict, storage: str, steps: int, K: int, init: str, dldomega: bool) -> dict:
    """Forward `steps` steps with checkpoints every K, then the adjoint of the
    velocity misfit to the seeded Fourier target."""
    import torch

    from lbm_inputs import generators as G
    from paper_1110_0270_amd import lbm as B

    nx, ny = w["nx"], w["ny"]
    cfg = B.make_config(**{**w, "storage": storage, "checkpoint_every": K, "max_steps": steps})
    sim = B.Simulation(cfg)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    if init == "uniform_rest":
        rho, ux, uy = G.uniform_rest(nx, ny)
    else:
        rho, ux, uy = G.double_shear_layer(nx)
    om = t(G.smooth_omega_field(nx, ny, seed=w.get("omega_seed", 41))) if w.get("omega_field") else None
    sim.set_equilibrium(t(rho), t(ux), t(uy))
    if om is not None:
        sim.set_omega(om)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)              # recorded rollout (HIP-graph groups between checkpoints)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tx, ty = G.fourier_target(nx, ny, seed=w.get("target_seed", 4))
    loss, g = velocity_loss_grad(sim.populations(), t(tx), t(ty))
    g0 = torch.empty_like(g)
    gw = torch.empty((ny, nx), dtype=torch.float64, device="cuda") if dldomega else None
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    adj_kern, _ = sim.profile_backward(g, g0, gw)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    # the step kernel's average duration, from events on a separate
    # unrecorded run of the same lattice (events force eager launches)
    nk = min(steps, 256)
    cfg_k = B.make_config(**{**w, "storage": storage, "checkpoint_every": 0, "max_steps": 0})
    sim_k = B.Simulation(cfg_k)
    sim_k.set_equilibrium(t(rho), t(ux), t(uy))
    if om is not None:
        sim_k.set_omega(om)
    fwd_kern, _ = sim_k.profile_step(nk)
    del sim_k
    n = nx * ny
    fwd_s, bwd_s = t1 - t0, t3 - t2
    res = {
        "storage": storage, "steps": steps, "checkpoint_every": K, "loss": loss,
        "fwd_ms": fwd_s * 1e3, "bwd_ms": bwd_s * 1e3,
        "fwd_mlups": n * steps / fwd_s / 1e6, "bwd_mlups": n * steps / bwd_s / 1e6,
        "fwd_adjoint_mlups": n * steps / (fwd_s + bwd_s) / 1e6,
        "fwd_kernel_us": fwd_kern / nk * 1e3, "adjoint_kernel_us": adj_kern / steps * 1e3,
        "workspace_gb": sim.workspace.numel() / 1e9,
    }
    out = (res, g0, gw)
    del sim
    torch.cuda.empty_cache()
    return out


def run_median3d(steps: int, warmup: int, delta=None) -> dict:
    """The 256^3 D3Q27 Taylor-Green workload with the 27-site median filter
    (FP32 storage): throughput, the step kernel against HBM (27 populations
    of 4 B read and written per site) and the fraction of updates the filter
    changed.  delta overrides the workload's acceptance threshold."""
    import torch

    from lbm_inputs import generators as G
    from lbm_inputs.workloads import workload
    from paper_1110_0270_amd import lbm as B

    w = workload("median3d_256")
    if delta is not None:
        w["med_delta"] = delta
    n = w["nx"] * w["ny"] * w["nz"]
    rho, ux, uy, uz = G.taylor_green_3d(w["nx"], w["ny"], w["nz"], u0=w["u0"])
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    sim = B.Simulation(B.make_config(**{**w, "storage": "f32"}))
    sim.set_equilibrium3d(t(rho), t(ux), t(uy), t(uz))
    del rho, ux, uy, uz
    sim.step(warmup)
    c0 = sim.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern_ms, _ = sim.profile_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = sim.counters()
    st = sim.stats()
    alg = 2 * 27 * 4 * n
    us = kern_ms / steps * 1e3
    res = {"workload": "median3d_256", "storage": "f32", "med_delta": w["med_delta"],
           "steps": steps, "warmup": warmup, "mlups": n * steps / (t1 - t0) / 1e6,
           "kernel_us": us, "alg_bytes_per_launch": alg, "kernel_gbs": alg / (us * 1e-6) / 1e9,
           "kernel_frac_of_hbm_peak": alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
           "median_per_update": (c1[1] - c0[1]) / (n * steps),
           "diverged_step": int(st.diverged_step), "mass_per_site": st.mass / n}
    del sim
    torch.cuda.empty_cache()
    log(f"[bench] median3d 256^3 f32 delta={w['med_delta']:g}: {res['mlups']:.0f} MLUPS, kernel "
        f"{us:.0f} us = {res['kernel_gbs']:.0f} GB/s, median on {res['median_per_update']:.4f} of updates")
    return res


def run_nonlocal(steps: int, warmup: int) -> dict:
    """The 4096^2 shear layer with the general nonlocal filter (binomial 3 x 3
    smoothing of f_neq), FP32 storage: throughput and the step kernel against
    HBM (9 populations of 4 B read and written per site)."""
    import torch

    from lbm_inputs import generators as G
    from lbm_inputs.workloads import workload
    from paper_1110_0270_amd import lbm as B

    w = workload("nonlocal_4096")
    n = w["nx"] * w["ny"]
    r0, ux, uy = G.double_shear_layer(w["nx"])
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    sim = B.Simulation(B.make_config(**{**w, "storage": "f32"}))
    sim.set_equilibrium(t(r0), t(ux), t(uy))
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern_ms, _ = sim.profile_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sim.stats()
    alg = 2 * 9 * 4 * n
    us = kern_ms / steps * 1e3
    res = {"workload": "nonlocal_4096", "storage": "f32", "steps": steps, "warmup": warmup,
           "mlups": n * steps / (t1 - t0) / 1e6, "kernel_us": us, "alg_bytes_per_launch": alg,
           "kernel_gbs": alg / (us * 1e-6) / 1e9,
           "kernel_frac_of_hbm_peak": alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
           "diverged_step": int(st.diverged_step), "mass_per_site": st.mass / n}
    del sim
    torch.cuda.empty_cache()
    log(f"[bench] nonlocal 4096^2 f32: {res['mlups']:.0f} MLUPS, kernel {us:.1f} us = "
        f"{res['kernel_gbs']:.0f} GB/s")
    return res


def _cpu_model() -> str:
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def cpu_baseline(w: dict, steps: int) -> dict:
    """The FP64 oracle on this host: `steps` full steps of the workload on
    all the threads torch uses, and one step of a 1024-row band of it (a
    1024 x 4096 periodic lattice of the same fields) on one thread."""
    import torch

    import oracle as O
    from lbm_inputs import generators as G

    lat = O.Lattice("D2Q9")
    rho, ux, uy = G.double_shear_layer(w["nx"])
    g = O.init_equilibrium(lat, rho, ux, uy)
    cfg = O.Config(nx=w["nx"], ny=w["ny"], bc="periodic", nu=w["nu"], ehrenfest=True,
                   ehr_k=w["ehr_k"], ehr_delta=w["ehr_delta"])
    threads = torch.get_num_threads()
    with torch.no_grad():
        t0 = time.perf_counter()
        for _ in range(steps):
            g, _ = O.step(lat, cfg, g)
        dt = time.perf_counter() - t0
        band = 1024
        gb = g[:, 512:512 + band, :].contiguous()        # holds the lower shear layer
        cb = cfg.with_(ny=band, ehr_k=-(-w["ehr_k"] * band // w["ny"]))
        torch.set_num_threads(1)
        try:
            t2 = time.perf_counter()
            O.step(lat, cb, gb)
            dt1 = time.perf_counter() - t2
        finally:
            torch.set_num_threads(threads)
    return {"value": w["nx"] * w["ny"] * steps / dt / 1e6, "unit": "MLUPS",
            "cores": threads, "kind": "oracle",
            "sample": f"{steps} full steps of the {w['nx']}x{w['ny']} workload, FP64, "
                      f"{dt:.1f} s on {threads} threads",
            "cpu_model": _cpu_model(),
            "single_thread": {"value": w["nx"] * band / dt1 / 1e6, "unit": "MLUPS", "cores": 1,
                              "sample": f"1 step of a {band}x{w['nx']} band of the workload "
                                        f"(periodic, Ehrenfest k scaled to the band), {dt1:.1f} s"}}


def run_elbm_8192(steps: int, warmup: int, adj_steps: int, adj_K: int) -> dict:
    """The 8192^2 periodic ELBM workload (positivity fallback and rule,
    Ehrenfest on 0.1 %, FP16 shifted storage): forward throughput and the
    ELBM branch statistics, then forward + adjoint over adj_steps steps, and
    the workspace the full 5000-step adjoint needs with checkpoints every
    71 steps (about sqrt(5000): checkpoint store and segment store equal)."""
    import torch

    from lbm_inputs import generators as G
    from lbm_inputs.workloads import workload
    from paper_1110_0270_amd import lbm as B

    w = workload("elbm_8192")
    n = w["nx"] * w["ny"]
    r0, ux, uy = G.spectral_velocity(w["nx"], seed=w["seed"])
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    rho, uxd, uyd = t(r0), t(ux), t(uy)
    del r0, ux, uy
    sim = B.Simulation(B.make_config(**{**w, "storage": "f16s", "checkpoint_every": 0}))
    sim.set_equilibrium(rho, uxd, uyd)
    sim.step(warmup)
    c0 = sim.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern_ms, _ = sim.profile_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = sim.counters()
    st = sim.stats(allow_status=(B.LBM_OK, B.LBM_EDIVERGED, B.LBM_ESELECT))
    upd = n * steps
    res = {
        "workload": "elbm_8192", "storage": "f16s", "steps": steps, "warmup": warmup,
        "mlups": upd / (t1 - t0) / 1e6,
        "kernel_us": kern_ms / steps * 1e3,
        "kernel_gbs": 2 * 9 * 2 * n / (kern_ms / steps * 1e-3) / 1e9,
        "positivity_per_update": (c1[0] - c0[0]) / upd,
        "elbm_noroot_per_update": (c1[2] - c0[2]) / upd,
        "elbm_fp64_solve_per_update": (c1[3] - c0[3]) / upd,
        "elbm_nonpositive_per_update": (c1[4] - c0[4]) / upd,
        "elbm_newton_iters_per_update": (c1[5] - c0[5]) / upd,
        "n_selected": int(st.n_selected), "diverged_step": int(st.diverged_step),
        "mass_per_site": st.mass / n,
    }
    del sim
    torch.cuda.empty_cache()
    log(f"[bench] elbm 8192^2 f16s: {res['mlups']:.0f} MLUPS, kernel {res['kernel_us']:.0f} us")
    if adj_steps > 0:
        sim = B.Simulation(B.make_config(**{**w, "storage": "f16s", "checkpoint_every": adj_K,
                                            "max_steps": adj_steps}))
        sim.set_equilibrium(rho, uxd, uyd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(adj_steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tx, ty = G.fourier_target(w["nx"], w["ny"], seed=w["target_seed"])
        loss, g = velocity_loss_grad(sim.populations(), t(tx), t(ty))
        del tx, ty
        g0 = torch.empty_like(g)
        gw = torch.empty((w["ny"], w["nx"]), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        adj_kern, _ = sim.profile_backward(g, g0, gw)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        adj_bytes = n * (9 * (4 + 4 + 2) + 2 * 4)
        res["adjoint"] = {
            "steps": adj_steps, "checkpoint_every": adj_K, "loss": loss,
            "fwd_ms": (t1 - t0) * 1e3, "bwd_ms": (t3 - t2) * 1e3,
            "fwd_adjoint_mlups": n * adj_steps / (t3 - t2 + t1 - t0) / 1e6,
            "adjoint_kernel_us": adj_kern / adj_steps * 1e3,
            "adjoint_kernel_gbs": adj_bytes / (adj_kern / adj_steps * 1e-3) / 1e9,
            "adjoint_alg_bytes_per_launch": adj_bytes,
            "grad_finite": bool(torch.isfinite(g0).all()) and bool(torch.isfinite(gw).all()),
            "workspace_gb": sim.workspace.numel() / 1e9,
        }
        del sim, g, g0, gw
        torch.cuda.empty_cache()
        log(f"[bench] elbm 8192^2 adjoint: fwd+adjoint {res['adjoint']['fwd_adjoint_mlups']:.0f} "
            f"MLUPS, adjoint kernel {res['adjoint']['adjoint_kernel_us']:.0f} us")
    full = B.make_config(**{**w, "storage": "f16s", "checkpoint_every": 71, "max_steps": 5000})
    res["full_adjoint_5000_steps_workspace_gb"] = B.lbm_workspace_bytes(full) / 1e9
    return res


def cavity_study(steps: int, checkpoints: list) -> dict:
    """The 256^2 lid-driven cavity at Re 5000 (lid 0.1): LBGK, ELBM, MRT and
    LBGK with the median filter, each in FP64 and FP32, from rest;
    throughput, divergence (checked every 100 steps), total entropy, ELBM
    branch and iteration counts, and the FP32 run's error against the FP64
    one at the checkpoints, next to an FP64 control whose relaxation rate is
    rounded to FP32 (the flow's own sensitivity to a perturbation of that
    size)."""
    import numpy as np
    import torch

    from lbm_inputs import generators as G
    from lbm_inputs.workloads import workload
    from paper_1110_0270_amd import lbm as B

    w = workload("cavity_256")
    omega = 1.0 / (3.0 * w["nu"] + 0.5)
    runs = {"lbgk": {}, "elbm": {"collision": "elbm"}, "mrt": {"collision": "mrt"},
            "lbgk_median": {"median": True, "med_delta": 1e-3}}
    forms = {"f64": {"storage": "f64"}, "f32": {"storage": "f32"},
             "f64_omega_rounded_to_f32": {"storage": "f64", "nu": None,
                                          "omega": float(np.float32(omega))}}
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    rho, ux, uy = (t(a) for a in G.uniform_rest(w["nx"], w["ny"]))
    n = w["nx"] * w["ny"]
    cps = [c for c in checkpoints if c <= steps]
    out = {"workload": "cavity_256", "steps": steps, "nu": w["nu"], "omega": omega,
           "checkpoints": cps, "runs": {}}
    for name, over in runs.items():
        res, moms = {}, {}
        for form, fo in forms.items():
            sim = B.Simulation(B.make_config(**{**w, **over, **fo, "check_interval": 100}))
            sim.set_equilibrium(rho, ux, uy)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done, div, snaps = 0, -1, {}
            for c in cps:
                sim.step(c - done)
                done = c
                st = sim.stats(allow_status=(B.LBM_OK, B.LBM_EDIVERGED, B.LBM_ESELECT))
                div = int(st.diverged_step)
                if div >= 0:
                    break
                snaps[c] = torch.stack(sim.moments()[1:])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c = sim.counters()
            res[form] = {"mlups": n * done / dt / 1e6, "steps_run": done, "diverged_step": div,
                         "entropy": st.entropy, "mass_drift": st.mass / n - 1.0,
                         "median_corrections_per_update": c[1] / (n * done),
                         "elbm_noroot_per_update": c[2] / (n * done),
                         "elbm_fp64_solves_per_update": c[3] / (n * done),
                         "elbm_iterations_per_update": c[5] / (n * done)}
            moms[form] = snaps
            del sim
        for form in ("f32", "f64_omega_rounded_to_f32"):
            res[form]["rel_l2_u_vs_f64"] = {
                c: rel_l2(moms[form][c], moms["f64"][c]) for c in cps
                if c in moms[form] and c in moms["f64"]}
        out["runs"][name] = res
        log(f"[study] cavity {name}: " + ", ".join(
            f"{k} {v['mlups']:.0f} MLUPS div {v['diverged_step']}" for k, v in res.items()))
    return out


def precision_study(w: dict, checkpoints: list) -> dict:
    """Error of the FP32, FP16-shifted and BF16-shifted forms against FP64
    over a long run of the shear-layer workload, next to an FP64 control
    started from the FP32-rounded initial state (its error is what the
    flow's own amplification makes of one rounding of the initial state)."""
    import torch

    from lbm_inputs import generators as G
    from paper_1110_0270_amd import lbm as B

    rho, ux, uy = G.double_shear_layer(w["nx"])
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    rounded = None
    runs = {}
    for form in ("f64", "f32", "f64_from_f32_init", "f16s", "bf16s"):
        storage = "f64" if form.startswith("f64") else form
        sim = B.Simulation(B.make_config(**{**w, "storage": storage}))
        if form == "f64_from_f32_init":
            sim.set_populations(rounded)
        else:
            sim.set_equilibrium(t(rho), t(ux), t(uy))
        if form == "f32":
            rounded = sim.populations()
        done, snaps = 0, {}
        t0 = time.perf_counter()
        for c in checkpoints:
            sim.step(c - done)
            done = c
            st = sim.stats(allow_status=(B.LBM_OK, B.LBM_EDIVERGED, B.LBM_ESELECT))
            snaps[c] = {"mom": sim.moments(), "sel": set(sim.selected()),
                        "mass": st.mass, "entropy": st.entropy,
                        "diverged_step": int(st.diverged_step)}
        torch.cuda.synchronize()
        log(f"[study] {form}: {checkpoints[-1]} steps in {time.perf_counter() - t0:.1f} s")
        runs[form] = snaps
        del sim
        torch.cuda.empty_cache()
    ref = runs["f64"]
    out = {"workload": "shear_layer_4096", "reference": "f64", "checkpoints": checkpoints,
           "forms": {}}
    for form, snaps in runs.items():
        rows = []
        for c in checkpoints:
            a, b = snaps[c], ref[c]
            du = torch.stack(a["mom"][1:]) - torch.stack(b["mom"][1:])
            sa, sb = a["sel"], b["sel"]
            rows.append({
                "step": c,
                "rel_l2_u": rel_l2(torch.stack(a["mom"][1:]), torch.stack(b["mom"][1:])),
                "max_abs_u": float(du.abs().max()),
                "rel_l2_rho_minus_1": rel_l2(a["mom"][0] - 1.0, b["mom"][0] - 1.0),
                "max_abs_rho": float((a["mom"][0] - b["mom"][0]).abs().max()),
                "selection_jaccard": len(sa & sb) / max(1, len(sa | sb)),
                "mass_drift": a["mass"] / (w["nx"] * w["ny"]) - 1.0,
                "entropy": a["entropy"],
                "diverged_step": a["diverged_step"],
            })
        out["forms"][form] = rows
    return out


def c5_study(steps: int, K: int, checkpoints: list) -> dict:
    """The 8192^2 ELBM workload at its stated length: FP16 shifted storage,
    `steps` steps forward with checkpoints every K, then the adjoint of the
    velocity misfit to the seeded Fourier target with recompute.  Next to
    it, the same forward run in FP64 (the reference), in FP32, and in FP64
    from the FP16-rounded initial state (the control: what the flow's own
    amplification makes of one FP16 rounding of the initial state), with the
    velocity error against FP64 at the checkpoints and the limiter
    statistics of each run."""
    import torch

    from lbm_inputs import generators as G
    from lbm_inputs.workloads import workload
    from paper_1110_0270_amd import lbm as B

    w = workload("elbm_8192")
    n = w["nx"] * w["ny"]
    r0, ux, uy = G.spectral_velocity(w["nx"], seed=w["seed"])
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    rho, uxd, uyd = t(r0), t(ux), t(uy)
    del r0, ux, uy
    cps = [c for c in checkpoints if c <= steps]
    if not cps or cps[-1] != steps:
        cps.append(steps)
    # the FP16-stored initial state, in FP64
    sim = B.Simulation(B.make_config(**{**w, "storage": "f16s", "checkpoint_every": 0}))
    sim.set_equilibrium(rho, uxd, uyd)
    rounded = sim.populations()
    del sim
    torch.cuda.empty_cache()

    def forward(form: str, sim, t_start: float) -> dict:
        snaps, done = {}, 0
        c0 = sim.counters()
        for c in cps:
            while done < c:
                m = min(500, c - done)
                sim.step(m)
                done += m
                torch.cuda.synchronize()
                log(f"[c5] {form}: step {done}, {time.perf_counter() - t_start:.1f} s")
            mom = sim.moments(dtype=torch.float32)
            st = sim.stats(allow_status=(B.LBM_OK, B.LBM_EDIVERGED, B.LBM_ESELECT))
            snaps[c] = {"u": torch.stack(mom[1:]), "sel": set(sim.selected()),
                        "mass": st.mass, "entropy": st.entropy,
                        "diverged_step": int(st.diverged_step)}
            del mom
        c1 = sim.counters()
        upd = n * steps
        return {"snaps": snaps, "limiters": {
            "positivity_per_update": (c1[0] - c0[0]) / upd,
            "elbm_noroot_per_update": (c1[2] - c0[2]) / upd,
            "elbm_fp64_solve_per_update": (c1[3] - c0[3]) / upd,
            "elbm_nonpositive_per_update": (c1[4] - c0[4]) / upd,
            "elbm_newton_iters_per_update": (c1[5] - c0[5]) / upd}}

    runs, out = {}, {"workload": "elbm_8192", "nx": w["nx"], "ny": w["ny"], "steps": steps,
                     "checkpoint_every": K, "checkpoints": cps, "reference": "f64", "forms": {}}
    for form in ("f64", "f64_from_f16_init", "f32"):
        storage = "f64" if form.startswith("f64") else form
        sim = B.Simulation(B.make_config(**{**w, "storage": storage, "checkpoint_every": 0}))
        if form == "f64_from_f16_init":
            sim.set_populations(rounded)
        else:
            sim.set_equilibrium(rho, uxd, uyd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs[form] = forward(form, sim, t0)
        runs[form]["mlups"] = n * steps / (time.perf_counter() - t0) / 1e6
        del sim
        torch.cuda.empty_cache()
    del rounded

    # FP16 with recording, then the adjoint
    cfg = B.make_config(**{**w, "storage": "f16s", "checkpoint_every": K, "max_steps": steps})
    sim = B.Simulation(cfg)
    sim.set_equilibrium(rho, uxd, uyd)
    del rho, uxd, uyd
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs["f16s"] = forward("f16s", sim, t0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tx, ty = G.fourier_target(w["nx"], w["ny"], seed=w["target_seed"])
    loss, g = velocity_loss_grad(sim.populations(), t(tx), t(ty))
    del tx, ty
    g0 = torch.empty_like(g)
    gw = torch.empty((w["ny"], w["nx"]), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    log(f"[c5] f16s: loss {loss:.6g}, backward over {steps} steps ...")
    t2 = time.perf_counter()
    adj_kern, _ = sim.profile_backward(g, g0, gw)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    log(f"[c5] f16s: backward {t3 - t2:.1f} s")
    adjoint = {
        "loss": loss, "fwd_s": t1 - t0, "bwd_s": t3 - t2,
        "fwd_mlups": n * steps / (t1 - t0) / 1e6,
        "bwd_mlups": n * steps / (t3 - t2) / 1e6,
        "fwd_adjoint_mlups": n * steps / (t3 - t2 + t1 - t0) / 1e6,
        "adjoint_kernel_us": adj_kern / steps * 1e3,
        "grad_finite": bool(torch.isfinite(g0).all()) and bool(torch.isfinite(gw).all()),
        "grad_f0_l2": float(g0.norm()), "grad_omega_l2": float(gw.norm()),
        "workspace_gb": sim.workspace.numel() / 1e9,
        "device_peak_gb": torch.cuda.max_memory_allocated() / 1e9,
    }
    del sim, g, g0, gw
    torch.cuda.empty_cache()

    ref = runs["f64"]["snaps"]
    for form, r in runs.items():
        rows = []
        for c in cps:
            a, b = r["snaps"][c], ref[c]
            rows.append({
                "step": c,
                "rel_l2_u": rel_l2(a["u"].double(), b["u"].double()),
                "max_abs_u": float((a["u"] - b["u"]).abs().max()),
                "selection_jaccard": len(a["sel"] & b["sel"]) / max(1, len(a["sel"] | b["sel"])),
                "mass_drift": a["mass"] / n - 1.0,
                "entropy": a["entropy"],
                "diverged_step": a["diverged_step"],
            })
        out["forms"][form] = {"error_vs_f64": rows, "limiters": r["limiters"]}
        if "mlups" in r:
            out["forms"][form]["forward_mlups"] = r["mlups"]
    out["forms"]["f16s"]["adjoint"] = adjoint
    return out


def hopf_study(res: list, L: int, steps_factor: float, record_frac: float) -> dict:
    """The first Hopf bifurcation of the lid-driven cavity (section 8): an
    L x L lattice with diffusive Maxwell walls, entropic equilibria, LBGK
    with the median filter (delta 1e-3), lid u0 = 0.1, from rest, FP64; for
    each Re (nu = u0 L / Re) steps_factor L / u0 steps, u_x at the probe
    node (L/16, 13L/16) (from the bottom-left corner) recorded over the final
    record_frac of them, and E_u of eq. energy, sqrt(L / (u0 n)) times the
    l2 norm of the recorded signal minus its mean.  E_u^2 grows linearly in
    Re past the bifurcation: a least-squares line through the points above
    the noise floor places it where the line crosses zero.  Also: the probe
    signal's dominant frequency, the enstrophy at the end, throughput.  The
    Reynolds numbers run at once, each lattice on a stream of its own (one
    small lattice leaves most of the GPU idle)."""
    import numpy as np
    import torch

    from lbm_inputs import generators as G
    from paper_1110_0270_amd import lbm as B

    u0 = 0.1
    n_steps = int(round(steps_factor * L / u0))
    n_rec = max(2, int(round(record_frac * n_steps)))
    n_main = n_steps - n_rec
    px, py = L // 16, (13 * L) // 16
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    rho, ux, uy = (t(a) for a in G.uniform_rest(L, L))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in res]
    sims = []
    for re, st in zip(res, streams):
        with torch.cuda.stream(st):
            cfg = B.make_config(lattice="D2Q9", nx=L, ny=L, bc="diffusive", u_lid=u0,
                                nu=u0 * L / re, equilibrium="entropic", median=True,
                                med_delta=1e-3, storage="f64")
            sim = B.Simulation(cfg)
            sim.set_equilibrium(rho, ux, uy)
        sims.append(sim)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, chunk = 0, 250000
    while done < n_main:
        m = min(chunk, n_main - done)
        for sim, st in zip(sims, streams):
            with torch.cuda.stream(st):
                sim.step(m)
        torch.cuda.synchronize()
        done += m
        log(f"[hopf] step {done} of {n_steps}, {time.perf_counter() - t0:.1f} s")
    t1 = time.perf_counter()
    sigs = [torch.empty((n_rec, 2), dtype=torch.float64, device="cuda") for _ in res]
    torch.cuda.synchronize()
    for k in range(n_rec):
        for sim, st, sig in zip(sims, streams, sigs):
            with torch.cuda.stream(st):
                sim.step(1)
                _, mx, my = sim.moments()
                sig[k, 0] = mx[py, px]
                sig[k, 1] = my[py, px]
        if (k + 1) % 10000 == 0:
            log(f"[hopf] recorded {k + 1} of {n_rec} steps, {time.perf_counter() - t1:.1f} s")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    rows = []
    for re, sim, st, sig in zip(res, sims, streams, sigs):
        with torch.cuda.stream(st):
            stt = sim.stats(allow_status=(B.LBM_OK, B.LBM_EDIVERGED))
            cnt = sim.counters()
        u = sig[:, 0].cpu().numpy()
        e_u = float(math.sqrt(L / (u0 * n_rec)) * np.linalg.norm(u - u.mean()))
        spec = np.abs(np.fft.rfft(u - u.mean()))
        kmax = int(np.argmax(spec[1:]) + 1) if spec.size > 1 else 0
        rows.append({
            "Re": re, "nu": u0 * L / re, "E_u": e_u, "E_u2": e_u * e_u,
            "u_mean": float(u.mean()), "v_mean": float(sig[:, 1].mean()),
            "u_std": float(u.std()),
            # cycles per step, and per L / u0 (the flow's time unit)
            "dominant_frequency_per_step": kmax / n_rec,
            "dominant_frequency_per_L_over_u0": kmax / n_rec * L / u0,
            "enstrophy": stt.enstrophy, "diverged_step": int(stt.diverged_step),
            # sites the median filter changed, per fluid-site update
            "median_per_update": cnt[1] / ((L - 2) * (L - 2) * n_steps),
        })
        log(f"[hopf] Re {re}: E_u {e_u:.4g}, enstrophy {stt.enstrophy:.4g}, "
            f"median {rows[-1]['median_per_update']:.3g} per update")
    del sims
    torch.cuda.empty_cache()
    # least-squares line of E_u^2 over Re through the points above the noise
    # floor (E_u^2 above a tenth of the largest)
    e2 = np.array([r["E_u2"] for r in rows])
    rr = np.array([r["Re"] for r in rows], dtype=float)
    fit = None
    on = e2 > 0.1 * e2.max()
    if on.sum() >= 2:
        slope, icpt = np.polyfit(rr[on], e2[on], 1)
        fit = {"points": int(on.sum()), "slope": float(slope), "intercept": float(icpt),
               "re_critical": float(-icpt / slope) if slope != 0 else None}
    return {"workload": "hopf_cavity", "L": L, "u0": u0, "steps": n_steps,
            "recorded_steps": n_rec, "probe": [px, py], "median_delta": 1e-3,
            "equilibrium": "entropic", "storage": "f64", "runs": rows, "fit": fit,
            "lattices_at_once": len(res),
            "mlups_all_lattices": len(res) * L * L * n_main / (t1 - t0) / 1e6,
            "main_s": t1 - t0, "record_s": t2 - t1}


def _round(x):
    if isinstance(x, dict):
        return {k: _round(v) for k, v in x.items()}
    if isinstance(x, float):
        return float(f"{x:.6g}")
    return x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--forms", default="f64,f16s,bf16s")
    ap.add_argument("--study", default="", help="'precision': error of the storage forms "
                    "against FP64 over a long shear-layer run; 'cavity': the four 256^2 "
                    "cavity runs in FP64 and FP32; 'c5': the 8192^2 ELBM workload, "
                    "FP16 forward plus adjoint over --study-steps steps, with FP64, "
                    "FP32 and FP64-control forward runs; 'hopf': the first Hopf "
                    "bifurcation of the diffusive-wall cavity (one JSON document each)")
    ap.add_argument("--study-checkpoints", default="100,1000,5000,10000,20000")
    ap.add_argument("--study-steps", type=int, default=50000)
    ap.add_argument("--study-re", default="7000,7500,8000,8500",
                    help="Reynolds numbers of --study hopf")
    ap.add_argument("--study-l", type=int, default=100, help="lattice side of --study hopf")
    ap.add_argument("--study-steps-factor", type=float, default=5000.0,
                    help="--study hopf runs this many L / u0 (5000 in the paper)")
    ap.add_argument("--study-record-frac", type=float, default=0.01,
                    help="final fraction of the --study hopf run recorded at the probe")
    ap.add_argument("--study-k", type=int, default=71,
                    help="checkpoint interval of --study c5 (about sqrt of its 5000 steps)")
    ap.add_argument("--adjoint-steps", type=int, default=8192)
    ap.add_argument("--scale-adjoint-steps", type=int, default=128)
    ap.add_argument("--elbm-steps", type=int, default=50)
    ap.add_argument("--elbm-adjoint-steps", type=int, default=32)
    ap.add_argument("--median3d-steps", type=int, default=50,
                    help="timed steps of the 256^3 D3Q27 median workload (0: skip)")
    ap.add_argument("--nonlocal-steps", type=int, default=200,
                    help="timed steps of the 4096^2 nonlocal-filter workload (0: skip)")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--median", action="store_true",
                    help="the headline workload with the median entropy filter on (delta 1e-3)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run 10 device copies of this many bytes (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.study == "cavity":
        cps = [1000, 5000, 10000, 20000, 50000]
        print(json.dumps(_round(cavity_study(args.study_steps, cps))), flush=True)
        return
    if args.study == "hopf":
        res = [float(x) for x in args.study_re.split(",")]
        print(json.dumps(_round(hopf_study(res, args.study_l, args.study_steps_factor,
                                           args.study_record_frac))), flush=True)
        return
    if args.study == "c5":
        cps = [int(x) for x in args.study_checkpoints.split(",")]
        print(json.dumps(_round(c5_study(args.study_steps, args.study_k, cps))), flush=True)
        return
    if args.study == "precision":
        from lbm_inputs.workloads import workload
        cps = [int(x) for x in args.study_checkpoints.split(",")]
        print(json.dumps(_round(precision_study(workload("shear_layer_4096"), cps))), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 10
        # a copy reads and writes the buffer once: the rate that a streaming
        # kernel moving the same bytes can reach
        print(json.dumps({"copy_bytes": args.copy_probe, "launches": 11, "us_per_copy": round(us, 1),
                          "read_plus_write_gbs": round(2 * args.copy_probe / us / 1e3, 1)}))
        return

    import torch

    from lbm_inputs.workloads import workload

    w = workload("shear_layer_4096")
    if args.median:
        w.update(median=True, med_delta=1e-3)
    log(f"[bench] {w['nx']}x{w['ny']} D2Q9 LBGK + Ehrenfest k={w['ehr_k']}"
        f"{' + median' if args.median else ''}, storage {args.storage}")
    main_res, main_mom = run_form(w, args.storage, args.steps, args.warmup)
    log(f"[bench] {args.storage}: {main_res['mlups']:.0f} MLUPS, kernel {main_res['kernel_ms']*1e3:.1f} us "
        f"= {main_res['kernel_gbs']:.0f} GB/s")
    forms = {args.storage: main_res}
    moms = {args.storage: main_mom}
    for s in [x for x in args.forms.split(",") if x and x != args.storage]:
        r, m = run_form(w, s, args.steps, args.warmup)
        forms[s], moms[s] = r, m
        log(f"[bench] {s}: {r['mlups']:.0f} MLUPS, kernel {r['kernel_gbs']:.0f} GB/s")
    if "f64" in moms:
        # velocity after the timed steps against the FP64 run (a short-run
        # figure; the forms' stated errors over 20k steps come from
        # --study precision)
        ref = moms["f64"]
        for s, m in moms.items():
            forms[s]["rel_l2_u_vs_f64"] = rel_l2(torch.stack(m[1:]), torch.stack(ref[1:]))
            forms[s]["rel_l2_u_vs_f64_after_steps"] = args.steps + args.warmup
    del moms, main_mom

    adjoint = None
    if args.adjoint_steps > 0:
        wa = workload("cavity_adjoint_512")
        adjoint = {"workload": "cavity_adjoint_512", "nx": wa["nx"], "ny": wa["ny"],
                   "collision": "mrt", "omega_field": True, "limiters": "ehrenfest k=9 delta=1e-3"}
        grads = {}
        for s in ("f32", "f64"):
            r, g0, gw = run_adjoint(wa, s, args.adjoint_steps, wa["checkpoint_every"],
                                    "uniform_rest", True)
            adjoint[s] = r
            grads[s] = (g0, gw)
            log(f"[bench] adjoint 512^2 {s}: fwd {r['fwd_mlups']:.0f} MLUPS, adjoint "
                f"{r['bwd_mlups']:.0f} MLUPS, fwd+adjoint {r['fwd_adjoint_mlups']:.0f} MLUPS")
        adjoint["f32"]["grad_rel_l2_f0_vs_f64"] = rel_l2(grads["f32"][0], grads["f64"][0])
        adjoint["f32"]["grad_rel_l2_omega_vs_f64"] = rel_l2(grads["f32"][1], grads["f64"][1])
        del grads

    adjoint_scale = None
    if args.scale_adjoint_steps > 0:
        r, g0, gw = run_adjoint(w, "f32", args.scale_adjoint_steps, 16, "shear", True)
        del g0, gw
        n = w["nx"] * w["ny"]
        adj_bytes = n * (9 * (4 + 4 + 4) + 2 * 4)     # lambda in/out, f, omega-gradient RMW
        r["adjoint_alg_bytes_per_launch"] = adj_bytes
        r["adjoint_kernel_gbs"] = adj_bytes / (r["adjoint_kernel_us"] * 1e-6) / 1e9
        r["adjoint_frac_of_hbm_peak"] = r["adjoint_kernel_gbs"] / HBM_PEAK_GBS
        adjoint_scale = {"workload": "shear_layer_4096", **r}
        log(f"[bench] adjoint 4096^2 f32: fwd+adjoint {r['fwd_adjoint_mlups']:.0f} MLUPS, adjoint "
            f"kernel {r['adjoint_kernel_us']:.1f} us = {r['adjoint_kernel_gbs']:.0f} GB/s")

    elbm = None
    if args.elbm_steps > 0:
        elbm = run_elbm_8192(args.elbm_steps, 20, args.elbm_adjoint_steps, 8)

    median3d = None
    if args.median3d_steps > 0:
        median3d = {"delta_1e-3": run_median3d(args.median3d_steps, 10),
                    "delta_0": run_median3d(args.median3d_steps, 10, delta=0.0)}
    nonlocal_ = None
    if args.nonlocal_steps > 0:
        nonlocal_ = run_nonlocal(args.nonlocal_steps, 20)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host ...")
        cpu = cpu_baseline(w, args.cpu_steps)
        log(f"[bench] oracle: {cpu['value']:.2f} MLUPS on {cpu['cores']} threads")
    achieved = main_res["kernel_gbs"]
    line = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "shear_layer_4096", "lattice": "D2Q9", "nx": w["nx"],
                   "ny": w["ny"], "bc": "periodic", "collision": "lbgk", "nu": w["nu"],
                   "limiters": f"ehrenfest k={w['ehr_k']} delta={w['ehr_delta']}"
                               + (f", median delta={w['med_delta']}" if args.median else ""),
                   "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (HBM_TRAFFIC_F32 if args.storage == "f32" and not args.median
                                 else None),
                     "traffic_unit": "bytes per launch",
                     "kernel": "k_step (fused collide-stream"
                               + (", median filter in LDS)" if args.median else ")"),
                     "kernel_us": round(main_res["kernel_ms"] * 1e3, 2),
                     "alg_bytes_per_launch": main_res["alg_bytes_per_launch"],
                     # the whole step (step kernel, Ehrenfest selection and
                     # the gaps between kernels) against the same peak
                     "whole_step_gbs": round(main_res["whole_step_gbs"], 1),
                     "whole_step_frac": round(main_res["whole_step_gbs"] / HBM_PEAK_GBS, 4)},
        "forms": _round(forms),
        "adjoint": _round(adjoint),
        "adjoint_scale": _round(adjoint_scale),
        "elbm_8192": _round(elbm),
        "median3d_256": _round(median3d),
        "nonlocal_4096": _round(nonlocal_),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
