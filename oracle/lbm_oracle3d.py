"""FP64 CPU oracle of the D3Q27 step with the 27-site median entropy filter
and the nonlocal f_neq filter (Brownlee, Levesley, Packwood and Gorban,
arXiv:1110.0270, section 4).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the HIP library or its binding.

Populations are tensors of shape (27, nz, ny, nx) on a periodic lattice.
One step, all sites at once:

  stream (pull, periodic)                -- section 2, free flight
  moments, product equilibrium           -- section 6 (1D equilibria); the 3D
                                            equilibrium is their product, as
                                            the 2D one of section 8 is
  nonlocal f_neq filter (optional)       -- section 4, "General nonlocal filters"
  Delta S (Kullback), median filter      -- section 4, eq. DelS; "Median entropy
                                            filter", 27 neighbours -> 14th value
  LBGK collision, positivity (optional)  -- eq. CollisionIntegral; eq. LimGenF

Reading: the paper names no 3D velocity set; its 27-site neighbourhood is
that of D3Q27, the tensor product of D1Q3 (velocities (a, b, c) in
{-1, 0, 1}^3, weights w_a w_b w_c).  The entropy, Delta S, LBGK and
positivity functions are the 2D oracle's, which act on any site shape.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Optional

import torch

from .lbm_oracle import DT, kullback_dS, lbgk, phi_entropic, phi_poly, positivity, relaxation_rate

__all__ = ["Lattice3", "Config3", "equilibrium3", "moments3", "stream3", "median_filter3",
           "nonlocal_filter3", "stencil_offsets3", "step3", "run3", "stats3",
           "init_equilibrium3"]


class Lattice3:
    """D3Q27 in tensor order i = 9 (c + 1) + 3 (b + 1) + (a + 1) for the
    velocity (a, b, c); the opposite of i is 26 - i."""

    def __init__(self):
        w1 = (1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0)
        self.name = "D3Q27"
        self.vel = [(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)]
        self.Q = 27
        self.opp = [self.vel.index((-a, -b, -c)) for (a, b, c) in self.vel]
        self.vx = torch.tensor([v[0] for v in self.vel], dtype=DT)
        self.vy = torch.tensor([v[1] for v in self.vel], dtype=DT)
        self.vz = torch.tensor([v[2] for v in self.vel], dtype=DT)
        self.w = torch.tensor([w1[a + 1] * w1[b + 1] * w1[c + 1] for (a, b, c) in self.vel],
                              dtype=DT)

    def col(self, t: torch.Tensor) -> torch.Tensor:
        return t.view(27, 1, 1, 1)


@dataclass
class Config3:
    nx: int = 8
    ny: int = 8
    nz: int = 8
    equilibrium: str = "poly"     # poly | entropic
    nu: Optional[float] = None
    omega: Optional[float] = None
    median: bool = False
    med_delta: float = 1e-3
    positivity: bool = False
    # nonlocal filter coefficients d(y) over the 27 shifts y = (dz, dy, dx)
    # in tensor order 9 (dz + 1) + 3 (dy + 1) + (dx + 1); None: off
    nl_coef: Optional[tuple] = None

    def with_(self, **kw) -> "Config3":
        return replace(self, **kw)


def equilibrium3(rho, ux, uy, uz, kind: str = "poly") -> torch.Tensor:
    """f*_(a,b,c) = rho phi_a(ux) phi_b(uy) phi_c(uz) with the 1D factors of
    section 6 (polynomial or entropic)."""
    phi = phi_poly if kind == "poly" else phi_entropic
    px, py, pz = phi(ux), phi(uy), phi(uz)
    lat = Lattice3()
    return torch.stack([rho * px[a + 1] * py[b + 1] * pz[c + 1] for (a, b, c) in lat.vel])


def moments3(f: torch.Tensor):
    """rho = sum_i f_i and rho u = sum_i v_i f_i (section 2)."""
    lat = Lattice3()
    return (f.sum(0), (lat.col(lat.vx) * f).sum(0), (lat.col(lat.vy) * f).sum(0),
            (lat.col(lat.vz) * f).sum(0))


def init_equilibrium3(rho, ux, uy, uz, kind: str = "poly") -> torch.Tensor:
    t = lambda a: torch.as_tensor(a, dtype=DT)  # noqa: E731
    return equilibrium3(t(rho), t(ux), t(uy), t(uz), kind)


def stream3(g: torch.Tensor) -> torch.Tensor:
    """Free flight on the periodic lattice: f_i(x) <- g_i(x - v_i)."""
    lat = Lattice3()
    return torch.stack([torch.roll(g[i], shifts=(c, b, a), dims=(0, 1, 2))
                        for i, (a, b, c) in enumerate(lat.vel)])


def stencil_offsets3():
    """The 27 neighbourhood shifts (dz, dy, dx) in tensor order."""
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _neighbour(t: torch.Tensor, dz: int, dy: int, dx: int) -> torch.Tensor:
    """out[z, y, x] = t[z + dz, y + dy, x + dx] (periodic) on the last three dims."""
    return torch.roll(t, shifts=(-dz, -dy, -dx), dims=(-3, -2, -1))


def median_filter3(f, feq, dS, med_delta: float):
    """Median entropy filter over the 27-site neighbourhood (the site and its
    26 neighbours; section 4 gives the 14th of the 27 sorted values): where
    dS > med_delta and dS_med < dS, f -> f* + sqrt(dS_med / dS) (f - f*)
    (eq. entrHom with the median as threshold).  Returns (f_new, mask)."""
    vals = torch.stack([_neighbour(dS, *o) for o in stencil_offsets3()])
    med = vals.sort(dim=0).values[13]
    accept = (dS > med_delta) & (med < dS) & torch.isfinite(dS)
    ratio = torch.where(accept, med / torch.where(accept, dS, torch.ones_like(dS)),
                        torch.ones_like(dS))
    coef = torch.where(accept, torch.sqrt(ratio.clamp(min=0.0)), torch.ones_like(dS))
    return feq + coef.unsqueeze(0) * (f - feq), accept


def nonlocal_filter3(f, feq, coef):
    """The nonlocal filter of section 4 on the 27 shifts: f*(x) + sum_y d(y)
    f_neq(x + y), f_neq = f - f* (moments of x unchanged)."""
    offs = stencil_offsets3()
    if len(coef) != len(offs):
        raise ValueError("D3Q27 takes 27 filter coefficients")
    neq = f - feq
    acc = torch.zeros_like(neq)
    for c, o in zip(coef, offs):
        acc = acc + float(c) * _neighbour(neq, *o)
    return feq + acc


def step3(cfg: Config3, g: torch.Tensor):
    """One step from the post-collision lattice g (27, nz, ny, nx).
    Reading (as in 2D): the filters act on the pre-collision state; the
    nonlocal filter comes first and Delta S is that of the filtered state.
    Returns (g_next, info)."""
    pre = stream3(g)
    rho, jx, jy, jz = moments3(pre)
    feq = equilibrium3(rho, jx / rho, jy / rho, jz / rho, cfg.equilibrium)
    info = {}
    if cfg.nl_coef is not None:
        pre = nonlocal_filter3(pre, feq, cfg.nl_coef)
    if cfg.median:
        dS = kullback_dS(pre, feq)
        info["dS"] = dS
        pre, info["median_mask"] = median_filter3(pre, feq, dS, cfg.med_delta)
    post = lbgk(pre, feq, relaxation_rate(cfg))   # nu = (1/omega - 1/2) / 3
    if cfg.positivity:
        post, info["positivity_mask"] = positivity(post, feq)
    return post, info


def run3(cfg: Config3, g: torch.Tensor, n: int, keep_info: bool = False):
    infos = []
    for _ in range(n):
        g, info = step3(cfg, g)
        if keep_info:
            infos.append(info)
    return (g, infos) if keep_info else g


def stats3(g: torch.Tensor) -> dict:
    """Whole-lattice mass, momentum and entropy -sum f_i ln(f_i / w_i)."""
    lat = Lattice3()
    rho, jx, jy, jz = moments3(g)
    ent = -torch.xlogy(g, g / lat.col(lat.w)).sum(0)
    return {"mass": float(rho.sum()), "mom_x": float(jx.sum()), "mom_y": float(jy.sum()),
            "mom_z": float(jz.sum()), "entropy": float(ent.sum())}

