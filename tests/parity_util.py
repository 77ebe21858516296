"""Shared helpers of the GPU parity tests: run the same seeded case through
the FP64 oracle and through the HIP library (via the C ABI)."""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

import oracle as O
from lbm_inputs import generators as G

DT = torch.float64
ORACLE_FIELDS = {f.name for f in dataclasses.fields(O.Config)}


def oracle_config(p: dict) -> O.Config:
    return O.Config(**{k: v for k, v in p.items() if k in ORACLE_FIELDS})


def lattice(p: dict) -> O.Lattice:
    return O.Lattice(p.get("lattice", "D2Q9"))


def random_state(p: dict, seed: int, amp: float = 0.05, umax: float = 0.08,
                 kind: str = "poly") -> torch.Tensor:
    """Equilibrium of random moments times (1 + uniform noise of size amp)."""
    lat = lattice(p)
    ny, nx = p["ny"], p["nx"]
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.uniform(-1, 1, (ny, nx))
    ux = umax * rng.uniform(-1, 1, (ny, nx))
    uy = umax * rng.uniform(-1, 1, (ny, nx)) if lat.name == "D2Q9" else np.zeros((ny, nx))
    f = O.init_equilibrium(lat, rho, ux, uy, kind)
    return f * (1.0 + torch.tensor(G.uniform_noise(f.shape, seed + 1000, amp)))


def make_sim(p: dict, storage: str = "f64"):
    from paper_1110_0270_amd import lbm as B
    cfg = B.make_config(**{**p, "storage": storage})
    return B.Simulation(cfg)


def gpu_run(p: dict, f0: torch.Tensor, n: int, storage: str = "f64", omega_field=None):
    """Run n steps on the GPU from f0 (CPU float64).  Returns (f_in, f_out,
    sim): f_in is the state as the library stores it (after rounding to the
    storage form), f_out the state after n steps, both as CPU float64."""
    sim = make_sim(p, storage)
    sim.set_populations(f0.to("cuda"))
    if omega_field is not None:
        sim.set_omega(omega_field.to("cuda"))
    f_in = sim.populations().cpu()
    sim.step(n)
    f_out = sim.populations().cpu()
    torch.cuda.synchronize()
    return f_in, f_out, sim


def oracle_run(p: dict, f0: torch.Tensor, n: int, omega_field=None):
    lat, cfg = lattice(p), oracle_config(p)
    g = f0.clone()
    infos = []
    for _ in range(n):
        g, info = O.step(lat, cfg, g, omega_field)
        infos.append(info)
    return g, infos


def rel_err(a: torch.Tensor, b: torch.Tensor, floor: float = 1e-3) -> float:
    """max_i |a_i - b_i| / max(|b_i|, floor)."""
    return float(((a - b).abs() / b.abs().clamp(min=floor)).max())


def near_tie_ok(gpu_sel, ora_sel, dS: torch.Tensor, k: int, rtol: float) -> bool:
    """Selected sets may differ only at sites whose Delta S lies within rtol
    (relative) of the k-th largest value."""
    a, b = set(int(i) for i in gpu_sel), set(int(i) for i in ora_sel)
    diff = a ^ b
    if not diff:
        return True
    flat = dS.flatten()
    kth = float(torch.sort(flat[torch.isfinite(flat)], descending=True).values[min(k, flat.numel()) - 1])
    return all(abs(float(flat[i]) - kth) <= rtol * abs(kth) for i in diff)
