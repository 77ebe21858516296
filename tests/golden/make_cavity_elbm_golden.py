"""Writes cavity_256_elbm_1000.npz: the FP64 oracle's 256^2 lid-driven
cavity at Re 5000 (lid 0.1, nu = 0.1 * 256 / 5000) with the ELBM collision,
from rest, after 500 and 1000 steps, at 2048 seeded sites plus the four
corners (all nine populations each), with the whole-lattice mass and
entropy.  A second oracle run from the rest state times (1 + a seeded
relative perturbation of 1e-16) measures how much the flow itself
amplifies rounding-sized differences by those steps (sens_500, sens_1000:
the largest relative difference of a population between the two runs).
Calls only the oracle; run it from the repository root:

    python tests/golden/make_cavity_elbm_golden.py
"""
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from lbm_inputs import generators as G  # noqa: E402
from lbm_inputs.workloads import workload  # noqa: E402

OUT = os.path.join(HERE, "cavity_256_elbm_1000.npz")
CHECKPOINTS = (500, 1000)


def sample_sites(n: int):
    rng = np.random.default_rng(97)
    idx = rng.choice(n * n, size=2048, replace=False)
    corners = np.array([0, n - 1, n * (n - 1), n * n - 1])
    return np.unique(np.concatenate([idx, corners]))


def main():
    w = workload("cavity_256")
    n = w["nx"]
    lat = O.Lattice("D2Q9")
    cfg = O.Config(nx=n, ny=n, bc="cavity", u_lid=w["u_lid"], nu=w["nu"], collision="elbm")
    g = O.init_equilibrium(lat, *G.uniform_rest(n, n), "entropic")
    h = g * (1 + 1e-16 * torch.tensor(np.random.default_rng(98).uniform(-1, 1, g.shape)))
    sites = sample_sites(n)
    out = {"sites": sites, "checkpoints": np.array(CHECKPOINTS)}
    with torch.no_grad():
        for t in range(1, CHECKPOINTS[-1] + 1):
            g, _ = O.step(lat, cfg, g)
            h, _ = O.step(lat, cfg, h)
            if t in CHECKPOINTS:
                st = O.stats(lat, g)
                sens = float(((g - h).abs() / g.abs().clamp(min=1e-3)).max())
                out[f"f_{t}"] = g.reshape(9, -1)[:, torch.tensor(sites)].numpy()
                out[f"mass_{t}"] = np.array(st["mass"])
                out[f"entropy_{t}"] = np.array(st["entropy"])
                out[f"sens_{t}"] = np.array(sens)
                print(f"step {t}: mass {st['mass']:.15g} entropy {st['entropy']:.15g} "
                      f"sensitivity {sens:.3e}", flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
