#!/usr/bin/env python3
"""Throughput of the fused D2Q9 collide-and-stream step with the Ehrenfest
limiter on the periodic double shear layer (4096 x 4096, nu = 1e-5, LBGK,
top 0.1 % of sites by nonequilibrium entropy sent to equilibrium each step).

One JSON line on stdout:
  value     whole-step throughput in MLUPS (million lattice-site updates per
            second), inputs resident in HBM, timed over --steps steps;
  roofline  the fused step kernel's algorithmic bytes (read 9 populations,
            write 9, per site) over its average duration from HIP events
            recorded around each launch inside the timed region, against
            the MI355X HBM peak of 8 TB/s;
  forms     the same workload with FP64 and shifted FP16/BF16 storage;
  cpu_baseline  the FP64 oracle timed on this host on two full steps.
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ELEM = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
METRIC = "MLUPS and % HBM roofline, D2Q9 fwd+adjoint, FP64 vs FP32/FP16-storage at stated err"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(w: dict, storage: str, steps: int, warmup: int) -> dict:
    import torch

    from lbm_inputs import generators as G
    from paper_1110_0270_amd import lbm as B

    cfg = B.make_config(**{**w, "storage": storage})
    sim = B.Simulation(cfg)
    rho, ux, uy = G.double_shear_layer(w["nx"])
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    sim.set_equilibrium(t(rho), t(ux), t(uy))
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern_ms, total_ms = sim.profile_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sim.stats(allow_status=(B.LBM_OK, B.LBM_EDIVERGED, B.LBM_ESELECT))
    n_sites = w["nx"] * w["ny"]
    ms_step = (t1 - t0) * 1e3 / steps
    kern_avg = kern_ms / steps
    alg_bytes = 2 * 9 * ELEM[storage] * n_sites
    res = {
        "storage": storage,
        "ms_per_step": ms_step,
        "mlups": n_sites / (ms_step * 1e-3) / 1e6,
        "kernel_ms": kern_avg,
        "kernel_gbs": alg_bytes / (kern_avg * 1e-3) / 1e9,
        "alg_bytes_per_launch": alg_bytes,
        "n_selected": int(st.n_selected),
        "select_fallbacks": int(st.select_fallbacks),
        "candidates_per_step": round(st.select_candidates / max(1, steps + warmup), 1),
        "diverged_step": int(st.diverged_step),
        "mass": st.mass,
    }
    del sim
    torch.cuda.empty_cache()
    return res


def cpu_baseline(w: dict, steps: int) -> dict:
    import torch

    import oracle as O
    from lbm_inputs import generators as G

    lat = O.Lattice("D2Q9")
    rho, ux, uy = G.double_shear_layer(w["nx"])
    g = O.init_equilibrium(lat, rho, ux, uy)
    cfg = O.Config(nx=w["nx"], ny=w["ny"], bc="periodic", nu=w["nu"], ehrenfest=True,
                   ehr_k=w["ehr_k"], ehr_delta=w["ehr_delta"])
    t0 = time.perf_counter()
    for _ in range(steps):
        g, _ = O.step(lat, cfg, g)
    dt = time.perf_counter() - t0
    return {"value": w["nx"] * w["ny"] * steps / dt / 1e6, "unit": "MLUPS",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{steps} full steps of the {w['nx']}x{w['ny']} workload, FP64, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--forms", default="f64,f16s,bf16s")
    ap.add_argument("--form-steps", type=int, default=300)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run 10 device copies of this many bytes (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_probe, "launches": 10}))
        return

    from lbm_inputs.workloads import workload

    w = workload("shear_layer_4096")
    log(f"[bench] {w['nx']}x{w['ny']} D2Q9 LBGK + Ehrenfest k={w['ehr_k']}, storage {args.storage}")
    main_res = run_form(w, args.storage, args.steps, args.warmup)
    log(f"[bench] {args.storage}: {main_res['mlups']:.0f} MLUPS, kernel {main_res['kernel_ms']*1e3:.1f} us "
        f"= {main_res['kernel_gbs']:.0f} GB/s")
    forms = {args.storage: main_res}
    for s in [x for x in args.forms.split(",") if x and x != args.storage]:
        r = run_form(w, s, args.form_steps, 100)
        forms[s] = r
        log(f"[bench] {s}: {r['mlups']:.0f} MLUPS, kernel {r['kernel_gbs']:.0f} GB/s")
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
                   "limiters": f"ehrenfest k={w['ehr_k']} delta={w['ehr_delta']}",
                   "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "k_step (fused collide-stream)",
                     "kernel_us": round(main_res["kernel_ms"] * 1e3, 2),
                     "alg_bytes_per_launch": main_res["alg_bytes_per_launch"]},
        "forms": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                      for kk, vv in v.items()} for k, v in forms.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
