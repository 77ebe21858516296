"""FP64 CPU oracle for one step of the regularised lattice Boltzmann method of
Brownlee, Levesley, Packwood and Gorban, "Add-ons for Lattice Boltzmann
Methods: Regularization, Filtering and Limiters" (arXiv:1110.0270).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the HIP library or its binding.

Plain PyTorch CPU operations in float64, written for readability, not speed.
Populations are tensors of shape (Q, ny, nx); D1Q3 uses ny = 1.  One time
step, all sites at once (a Jacobi update from the state at time t), in the
order:

  stream (pull, boundaries)            -- section 2, eq. of free flight
  moments, equilibrium                 -- section 2; section 6 (1D equilibria);
                                          section 8 (2D product equilibrium)
  nonlocal f_neq filter (optional)     -- section 4, "General nonlocal filters"
  nonequilibrium entropy Delta S       -- section 4, Kullback entropy (eq. Kul, DelS)
  median entropy filter (optional)     -- section 4, "Median entropy filter"
  Ehrenfest selection (optional)       -- section 4, Ehrenfests' regularisation
  collision: LBGK | MRT | ELBM         -- eq. CollisionIntegral; section 5; section 3
  positivity rule (optional)           -- section 4, eq. LimGenF and StrLine

Readings of passages that the paper leaves open are marked "Reading:" where
they are used.  Autograd through `step` gives the exact (sub)gradient of the
step; the ELBM root carries its implicit-function derivative.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import Optional

import torch

DT = torch.float64

__all__ = [
    "Lattice", "Config", "relaxation_rate", "phi_poly", "phi_entropic",
    "equilibrium", "moments", "velocity", "stream", "entropy", "h_fn",
    "kullback_dS", "lbgk", "mrt_basis", "mrt_rates", "mrt_preset_rates", "mrt", "elbm_alpha",
    "elbm", "positivity", "median_filter", "ehrenfest_select", "ens_threshold",
    "ens_phi", "ensemble_limiter", "step", "run",
    "stats", "init_equilibrium", "ELBM_ROOT", "ELBM_CUTOFF", "ELBM_NOROOT",
    "ELBM_NONPOS", "wall_nodes", "diffusive_wall", "enstrophy", "hopf_energy",
    "nonlocal_filter", "stencil_offsets",
]


# ---------------------------------------------------------------------------
# Lattices.  Section 6 gives the D1Q3 velocities (-1, 0, 1); its polynomial
# equilibria at u = 0 fix the weights (1/6, 2/3, 1/6).  D2Q9 (section 5) has
# the nine velocities (a, b) in {-1,0,1}^2; the product equilibrium of
# section 8 fixes w_(a,b) = w_a w_b.  Index order ("tensor order"):
# i = 3 (b + 1) + (a + 1), so the opposite of i is Q - 1 - i.
# ---------------------------------------------------------------------------
class Lattice:
    def __init__(self, name: str):
        w1 = (1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0)
        if name == "D1Q3":
            vel = [(-1, 0), (0, 0), (1, 0)]
            w = list(w1)
        elif name == "D2Q9":
            vel = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
            w = [w1[a + 1] * w1[b + 1] for (a, b) in vel]
        else:
            raise ValueError(f"unknown lattice {name}")
        self.name = name
        self.Q = len(vel)
        self.vel = vel
        self.opp = [vel.index((-a, -b)) for (a, b) in vel]
        self.vx = torch.tensor([a for a, _ in vel], dtype=DT)
        self.vy = torch.tensor([b for _, b in vel], dtype=DT)
        self.w = torch.tensor(w, dtype=DT)

    def col(self, t: torch.Tensor) -> torch.Tensor:
        """Reshape a (Q,) tensor to broadcast against (Q, ...) populations."""
        return t.view(self.Q, *([1] * 2))


@dataclass
class Config:
    lattice: str = "D2Q9"
    nx: int = 16
    ny: int = 16
    bc: str = "periodic"          # periodic | bounceback | cavity | couette | diffusive
    u_lid: float = 0.0
    rho_wall: float = 1.0
    collision: str = "lbgk"       # lbgk | mrt | elbm
    equilibrium: str = "poly"     # poly | entropic (ELBM always uses entropic)
    nu: Optional[float] = None
    omega: Optional[float] = None
    mrt_basis: str = "M1"         # M1 (section 5, C1 rates) | M2 (C2 rates)
    s_e: float = 1.64
    s_eps: float = 1.54
    s_q: float = 1.9
    # M1 rate presets of sections 5, 7 and 8: given (s_e, s_eps, s_q as set) |
    # trt | mrt_trtq | mrt1 | shear
    mrt_preset: str = "given"
    ehrenfest: bool = False
    # what the selected sites receive: "equilibrium" (Ehrenfests' step) or
    # "mrt" (the MRT collision with mrt_basis and its rates: the MRT limiter
    # of section 5, on an LBGK lattice)
    sel_action: str = "equilibrium"
    ehr_k: int = 0
    ehr_delta: float = 0.0
    # ensemble-dependent and smooth limiters of section 4 (acting on the
    # pre-collision state): none | threshold (eqs. EntThresh, entrHom) |
    # smooth (eq. phiExamp) | double_monotone (eq. DoublMonSpec) | pointwise
    # (phi = 1 / (1 + alpha Delta S^k))
    ens_limiter: str = "none"
    ens_delta0: float = 0.1      # dissipation budget delta_0 of eq. LimEntLim
    ens_delta: float = 0.0       # lower bound delta of the threshold
    ens_alpha: float = 1.0
    ens_k: float = 1.0
    median: bool = False
    med_delta: float = 1e-3
    positivity: bool = False
    elbm_norm: str = "entropic"   # entropic | l1
    elbm_fallback: str = "positivity"  # positivity | ehrenfest
    elbm_eps: float = 1e-14
    elbm_max_iter: int = 32
    elbm_dS_cut: float = 1e-15
    # general nonlocal filter of section 4 (None: off): the coefficients
    # d(y) of the neighbourhood shifts y in tensor order, (dx) for D1Q3 and
    # 3 (dy + 1) + (dx + 1) for D2Q9
    nl_coef: Optional[tuple] = None

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


def relaxation_rate(cfg: Config) -> float:
    """omega from nu = c_s^2 (1/omega - 1/2), c_s^2 = 1/3.

    Reading: the paper's beta = eps/(2 nu + eps) (section 2) uses a different
    viscosity scale; the rate is bound here to the lattice viscosity
    nu = c_s^2 (1/omega - 1/2) whose decay the shear-wave test measures."""
    if cfg.omega is not None:
        return float(cfg.omega)
    return 1.0 / (3.0 * cfg.nu + 0.5)


# ---------------------------------------------------------------------------
# Equilibria (section 6: 1D polynomial and entropic equilibria; section 8:
# the 2D quasi-equilibrium is the product of the 1D ones).  phi(u) returns
# the three factors for a = -1, 0, +1 stacked on dim 0.
# ---------------------------------------------------------------------------
def phi_poly(u: torch.Tensor) -> torch.Tensor:
    return torch.stack([(1.0 - 3.0 * u + 3.0 * u * u) / 6.0,
                        (2.0 / 3.0) * (1.0 - 1.5 * u * u),
                        (1.0 + 3.0 * u + 3.0 * u * u) / 6.0])


def phi_entropic(u: torch.Tensor) -> torch.Tensor:
    s = torch.sqrt(1.0 + 3.0 * u * u)
    return torch.stack([(-3.0 * u - 1.0 + 2.0 * s) / 6.0,
                        (2.0 / 3.0) * (2.0 - s),
                        (3.0 * u - 1.0 + 2.0 * s) / 6.0])


def equilibrium(lat: Lattice, rho, ux, uy, kind: str = "poly") -> torch.Tensor:
    phi = phi_poly if kind == "poly" else phi_entropic
    px = phi(ux)
    if lat.name == "D1Q3":
        return rho.unsqueeze(0) * px
    py = phi(uy)
    return torch.stack([rho * px[a + 1] * py[b + 1] for (a, b) in lat.vel])


def moments(lat: Lattice, f: torch.Tensor):
    """rho = sum_i f_i and rho u = sum_i v_i f_i (section 2)."""
    rho = f.sum(0)
    jx = (lat.col(lat.vx) * f).sum(0)
    jy = (lat.col(lat.vy) * f).sum(0)
    return rho, jx, jy


def velocity(lat: Lattice, f: torch.Tensor):
    rho, jx, jy = moments(lat, f)
    return rho, jx / rho, jy / rho


def init_equilibrium(lat: Lattice, rho, ux, uy, kind="poly") -> torch.Tensor:
    """Populations at equilibrium for given macroscopic fields (ny, nx)."""
    t = lambda a: torch.as_tensor(a, dtype=DT)  # noqa: E731
    return equilibrium(lat, t(rho), t(ux), t(uy), kind)


# ---------------------------------------------------------------------------
# Free flight (section 2): f_i(x, t+1) = f_i(x - v_i, t), as a pull.
# Reading of "bounce back" (section 8): halfway bounce-back with every node a
# fluid node.  A population whose source x - v_i lies outside the domain is
# the opposite population of the same node; when the source lies above the
# top row of a cavity (the lid takes precedence at the two top corners), the
# moving wall adds 6 w_i rho_wall (v_i . u_wall), u_wall = (u_lid, 0).
# "couette" is the same lid over a bounce-back floor with periodic sides.
# ---------------------------------------------------------------------------
def stream(lat: Lattice, g: torch.Tensor, bc: str, u_lid: float = 0.0,
           rho_wall: float = 1.0) -> torch.Tensor:
    Q, ny, nx = g.shape
    ys = torch.arange(ny).view(ny, 1)
    xs = torch.arange(nx).view(1, nx)
    out = []
    for i, (a, b) in enumerate(lat.vel):
        shifted = torch.roll(g[i], shifts=(b, a), dims=(0, 1))
        if bc == "periodic":
            out.append(shifted)
            continue
        sx, sy = xs - a, ys - b
        outside = (sy < 0) | (sy >= ny)
        if bc != "couette":                 # couette: periodic in x
            outside = outside | (sx < 0) | (sx >= nx)
        outside = outside.expand(ny, nx)
        refl = g[lat.opp[i]]
        if bc == "diffusive":
            # the wall rule (diffusive_wall) replaces every such population
            out.append(torch.where(outside, refl, shifted))
            continue
        if bc in ("cavity", "couette"):
            from_lid = (sy >= ny).expand(ny, nx)
            lid = torch.tensor(6.0 * float(lat.w[i]) * rho_wall * a * u_lid, dtype=DT)
            refl = refl + torch.where(from_lid, lid, torch.zeros((), dtype=DT))
        elif bc != "bounceback":
            raise ValueError(bc)
        out.append(torch.where(outside, refl, shifted))
    return torch.stack(out)


# ---------------------------------------------------------------------------
# Diffusive Maxwell wall (section 8, "First Hopf bifurcation"): after the
# advection, at a wall site the populations pointing into the fluid become
# gamma f*_i(u_wall), gamma = (sum of the populations that reached the wall)
# / (sum of f*_i(u_wall) over the incoming directions), f* at unit density
# (density is a linear factor); wall sites do not collide.
# Reading: the lattice is nx x ny nodes; its outer ring of nodes is the wall
# (the lid is the top row y = ny - 1, moving with (u_lid, 0); the other
# walls rest).  At an edge site the incoming directions are those with
# v . n > 0 (n the inward normal: on the lid S, SW, SE, as printed); at a
# corner only the diagonal along n, which makes the rule bounce-back there
# (as the paper states).  Every population whose source lies outside the
# lattice takes gamma f*_i(u_wall) with the site's gamma: at an edge these
# are exactly the incoming ones; at a corner the others run along a wall or
# out of the lattice and never reach the fluid.  Corners rest (u_wall = 0;
# the diagonal's value does not depend on it).  f* is the step's
# equilibrium kind.
# ---------------------------------------------------------------------------
def wall_nodes(ny: int, nx: int) -> torch.Tensor:
    """Boolean (ny, nx) mask of the wall ring of a diffusive-wall lattice."""
    m = torch.zeros((ny, nx), dtype=torch.bool)
    m[0, :] = True
    m[-1, :] = True
    m[:, 0] = True
    m[:, -1] = True
    return m


def diffusive_wall(lat: Lattice, pre: torch.Tensor, u_lid: float, kind: str) -> torch.Tensor:
    """The wall rule on the streamed state `pre` (Q, ny, nx); interior sites
    are returned unchanged."""
    Q, ny, nx = pre.shape
    one = torch.ones((1, 1), dtype=DT)
    zero = torch.zeros((1, 1), dtype=DT)
    feq_lid = equilibrium(lat, one, one * u_lid, zero, kind)[:, 0, 0]
    feq_rest = equilibrium(lat, one, zero, zero, kind)[:, 0, 0]
    out = pre.clone()
    X, Y = nx - 1, ny - 1
    # (ys, xs, inward normal, f*(u_wall)) for the four edges and four corners
    parts = [
        (torch.full((nx - 2,), Y), torch.arange(1, X), (0, -1), feq_lid),    # lid
        (torch.full((nx - 2,), 0), torch.arange(1, X), (0, 1), feq_rest),    # floor
        (torch.arange(1, Y), torch.full((ny - 2,), 0), (1, 0), feq_rest),    # left
        (torch.arange(1, Y), torch.full((ny - 2,), X), (-1, 0), feq_rest),   # right
        (torch.tensor([0]), torch.tensor([0]), (1, 1), feq_rest),
        (torch.tensor([0]), torch.tensor([X]), (-1, 1), feq_rest),
        (torch.tensor([Y]), torch.tensor([0]), (1, -1), feq_rest),
        (torch.tensor([Y]), torch.tensor([X]), (-1, -1), feq_rest),
    ]
    for ys, xs, (n_x, n_y), feq_w in parts:
        corner = n_x != 0 and n_y != 0
        incoming = [i for i, (a, b) in enumerate(lat.vel)
                    if ((a, b) == (n_x, n_y) if corner else a * n_x + b * n_y > 0)]
        unknown = [i for i, (a, b) in enumerate(lat.vel) if a * n_x > 0 or b * n_y > 0]
        reached = sum(pre[lat.opp[i], ys, xs] for i in incoming)
        gamma = reached / sum(float(feq_w[i]) for i in incoming)
        for i in unknown:
            out[i, ys, xs] = gamma * feq_w[i]
    return out


def enstrophy(lat: Lattice, g: torch.Tensor, bc: str = "periodic") -> float:
    """Enstrophy (section 8, cavity study): the sum of the squared vorticity
    over the lattice divided by the number of sites.  Reading: vorticity
    du_y/dx - du_x/dy by central differences of the velocity at the sites
    with four neighbours inside the lattice (all sites of a periodic
    lattice, with wrap-around), and the sum is divided by the number of
    those sites."""
    rho, jx, jy = moments(lat, g)
    ux, uy = jx / rho, jy / rho
    # roll(a, -1, dims=1)[y, x] = a[y, x + 1]
    duy_dx = (torch.roll(uy, -1, dims=1) - torch.roll(uy, 1, dims=1)) / 2.0
    dux_dy = (torch.roll(ux, -1, dims=0) - torch.roll(ux, 1, dims=0)) / 2.0
    w = duy_dx - dux_dy
    if bc != "periodic":
        w = w[1:-1, 1:-1]
    return float((w * w).sum() / w.numel())


def hopf_energy(signal, L: float, u0: float) -> float:
    """E_u of eq. energy: the l2 norm of sqrt(L / (u0 n)) (s - mean(s)) over
    the n samples of the probe signal s."""
    s = torch.as_tensor(signal, dtype=DT)
    n = s.numel()
    return float(math.sqrt(L / (u0 * n)) * torch.linalg.vector_norm(s - s.mean()))


# ---------------------------------------------------------------------------
# Entropy and nonequilibrium entropy (section 3, eq. ELBMEntropy; section 4,
# eqs. Kul, KulSq, DelS).  Perfect entropy S(f) = -sum f_i ln(f_i / W_i) with
# W_i = w_i (the D1Q3 form with W = (1, 4, 1) differs by a multiple of rho).
# ---------------------------------------------------------------------------
def entropy(lat: Lattice, f: torch.Tensor) -> torch.Tensor:
    return -torch.xlogy(f, f / lat.col(lat.w)).sum(0)


_H_SERIES = [((-1.0) ** n) / (n * (n - 1)) for n in range(2, 17)]


def h_fn(x: torch.Tensor) -> torch.Tensor:
    """h(x) = (1 + x) ln(1 + x) - x for x >= -1, with h(-1) = 1 (0 ln 0 = 0;
    autograd takes h constant there, i.e. no derivative at a zero population).

    For |x| < 0.1 the Taylor series sum_{n>=2} (-1)^n x^n / (n (n-1)) is
    summed to n = 16 (truncation below 1e-16 relative), avoiding the
    cancellation of the direct form."""
    small = x.abs() < 0.1
    xs = torch.where(small, x, torch.zeros_like(x))
    acc = torch.zeros_like(x)
    for c in reversed(_H_SERIES[1:]):
        acc = (acc + c) * xs
    series = (acc + _H_SERIES[0]) * xs * xs
    edge = x <= -1.0
    xd = torch.where(small | edge, torch.full_like(x, 0.5), x)
    direct = (1.0 + xd) * torch.log1p(xd) - xd
    return torch.where(small, series, torch.where(edge, torch.ones_like(x), direct))


def kullback_dS(f: torch.Tensor, feq: torch.Tensor) -> torch.Tensor:
    """Delta S = sum_i f_i ln(f_i / f*_i) (eq. DelS), evaluated as
    sum_i f*_i h((f_i - f*_i) / f*_i), which is the same sum because f and f*
    share their density.  This form keeps full relative accuracy when Delta S
    is far below rounding of rho.  Reading: Delta S = +inf at a site with a
    negative population (the Kullback sum is undefined there)."""
    x = (f - feq) / feq
    terms = feq * h_fn(x)
    bad = ((f < 0) | (feq <= 0)).any(0)
    return torch.where(bad, torch.full_like(terms[0], math.inf), terms.sum(0))


# ---------------------------------------------------------------------------
# Collisions.
# ---------------------------------------------------------------------------
def lbgk(f, feq, omega):
    """F(f) = f + alpha beta (f* - f) with alpha beta = omega
    (eq. CollisionIntegral)."""
    return f + omega * (feq - f)


def mrt_basis(kind: str) -> torch.Tensor:
    """Change-of-basis matrix rebuilt from its defining velocity polynomials
    (section 5), columns in tensor order.

    M1 rows: rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy, i.e. 1,
    -4 + 3 v^2, 4 - 21/2 v^2 + 9/2 v^4, v_x, (-5 + 3 v^2) v_x, v_y,
    (-5 + 3 v^2) v_y, v_x^2 - v_y^2, v_x v_y.
    M2 rows: 1, v_x, v_y, v_x^2 + v_y^2, v_x^2 - v_y^2, v_x v_y, v_x^2 v_y,
    v_x v_y^2, v_x^2 v_y^2 (the listed basis; the printed M2 has its last two
    cubic rows interchanged, which the C2 rates make immaterial)."""
    lat = Lattice("D2Q9")
    vx, vy = lat.vx, lat.vy
    v2 = vx * vx + vy * vy
    one = torch.ones_like(vx)
    if kind == "M1":
        rows = [one, -4 + 3 * v2, 4 - 10.5 * v2 + 4.5 * v2 * v2, vx,
                (-5 + 3 * v2) * vx, vy, (-5 + 3 * v2) * vy, vx * vx - vy * vy,
                vx * vy]
    elif kind == "M2":
        rows = [one, vx, vy, v2, vx * vx - vy * vy, vx * vy, vx * vx * vy,
                vx * vy * vy, vx * vx * vy * vy]
    else:
        raise ValueError(kind)
    return torch.stack(rows)


def mrt_rates(kind: str, s_e: float, s_eps: float, s_q: float, s_nu):
    """Diagonal of C1 = diag(1, s_e, s_eps, 1, s_q, 1, s_q, s_nu, s_nu) or
    C2 = diag(1, 1, 1, 1, s_nu, s_nu, 1, 1, 1) (section 5).  s_nu may be a
    tensor (per-site shear rate); the result then has shape (9, *s_nu.shape).
    Reading: s_nu is the shear rate (the text names the second-order rates
    both ways; the TRT paragraph ties s_nu to shear viscosity)."""
    s_nu = torch.as_tensor(s_nu, dtype=DT)
    one = torch.ones_like(s_nu)
    if kind == "M1":
        c = [one, s_e * one, s_eps * one, one, s_q * one, one, s_q * one, s_nu, s_nu]
    else:
        c = [one, one, one, one, s_nu, s_nu, one, one, one]
    return torch.stack(c)


def mrt_preset_rates(preset: str, s_nu, s_e: float = 1.64, s_eps: float = 1.54,
                     s_q: float = 1.9):
    """(s_e, s_eps, s_q) of the M1 (C1) rate presets, as functions of the
    shear rate s_nu (a number or a per-site tensor):
      trt      s_e = s_eps = s_nu, s_q = 8 (2 - s_nu) / (8 - s_nu)  (section 5,
               TRT; Reading: the printed "8(2=s_nu)" is 8(2 - s_nu))
      mrt_trtq s_e = 1.64, s_eps = 1.54, s_q as for trt (section 8, the
               cavity study's MRT with the TRT third-order rate)
      mrt1     s_e = 1.64, s_eps = 1.54, s_q = 1.9 (section 8, MRT1)
      shear    s_e = 1.64, s_eps = 1.54, s_q = 3 (2 - s_nu) / (3 - s_nu)
               (section 7, the shear-wave MRT)
      given    the rates as configured."""
    s_nu = torch.as_tensor(s_nu, dtype=DT)
    if preset == "given":
        return s_e, s_eps, s_q
    if preset == "trt":
        return s_nu, s_nu, 8.0 * (2.0 - s_nu) / (8.0 - s_nu)
    if preset == "mrt_trtq":
        return 1.64, 1.54, 8.0 * (2.0 - s_nu) / (8.0 - s_nu)
    if preset == "mrt1":
        return 1.64, 1.54, 1.9
    if preset == "shear":
        return 1.64, 1.54, 3.0 * (2.0 - s_nu) / (3.0 - s_nu)
    raise ValueError(preset)


def mrt(f, feq, M, rates):
    """F(f) = f + M^{-1} C M (f* - f) (section 5), applied in moment space.
    `rates` has shape (9,) or (9, ny, nx)."""
    Minv = torch.linalg.inv(M)
    Q = f.shape[0]
    d = (feq - f).reshape(Q, -1)
    m = M @ d
    r = rates.reshape(Q, -1) if rates.dim() > 1 else rates.view(Q, 1)
    return f + (Minv @ (r * m)).reshape(f.shape)


# ---------------------------------------------------------------------------
# ELBM (section 3): alpha is the nontrivial root of S(f + alpha (f* - f)) =
# S(f), found by successive parabolas from the LBGK estimate alpha = 2.
# With Delta = f* - f and entropic f*, S_f(alpha) = S(f + alpha Delta) - S(f)
# and its derivatives are evaluated in a cancellation-free form that uses
# the exact identities sum_i Delta_i = 0 and sum_i Delta_i ln(f*_i/W_i) = 0:
#   S_f   = -sum f_i h(alpha Delta_i / f_i) - alpha sum Delta_i ln(f_i / f*_i)
#   S_f'  = -sum Delta_i ln((f_i + alpha Delta_i) / f*_i)
#   S_f'' = -sum Delta_i^2 / (f_i + alpha Delta_i)
# ---------------------------------------------------------------------------
def _sf_parts(f, D, feq, alpha):
    x = alpha * D / f
    lnr = torch.log1p(-D / feq)                       # ln(f_i / f*_i)
    sf = -(f * h_fn(x)).sum(0) - alpha * (D * lnr).sum(0)
    d1 = -(D * (torch.log1p(x.clamp(min=-1.0)) + lnr)).sum(0)
    d2 = -(D * D / (f + alpha * D)).sum(0)
    return sf, d1, d2


# branch codes shared by elbm_alpha's outputs
ELBM_ROOT, ELBM_CUTOFF, ELBM_NOROOT, ELBM_NONPOS = 0, 1, 2, 3


def elbm_alpha(f, feq, *, eps=1e-14, max_iter=32, dS_cut=1e-15,
               norm="entropic", fallback="positivity"):
    """Per-site alpha for ELBM.  f, feq: (Q, n).  Returns (alpha, branch).

    Steps (section 3, "ELBM algorithm" and "Numerical method"):
      * Delta S < dS_cut (1e-15 in the paper): plain LBGK, alpha = 2.
      * alpha_max = min over Delta_i < 0 of f_i / (-Delta_i), the largest
        alpha keeping f + alpha Delta >= 0.  If S_f(alpha_max) >= 0 there is
        no nontrivial root: the positivity rule takes alpha = alpha_max, the
        Ehrenfest rule alpha = 1.
      * Otherwise iterate from alpha_0 = 2 (Reading: (1 + alpha_max)/2 when 2
        is not below alpha_max): stop when |S_f / S_f'| * ||Delta|| < eps
        (eq. ConvergenceTwo with the Newton estimate eq. Stopping), else move
        to the greater root of the second-order Taylor parabola, written as
        2 S_f / (-S_f' + sqrt(S_f'^2 - 2 S_f S_f'')).  Reading: a negative
        discriminant takes a Newton step; a step leaving (1, alpha_max) is
        replaced by bisection towards the violated bound.
      * After convergence, if S_f(alpha) < 0 take one double-length Newton
        step alpha - 2 S_f / S_f' to land below the root.
    Reading: ||Delta|| is the entropic norm sqrt(sum Delta_i^2 / f*_i) (the
    square root of the quadratic form of the second differential), or L1;
    eps = 1e-14 (no value is printed).  Reading: a site with a non-positive
    population has no entropy; it takes alpha = 1."""
    with torch.no_grad():
        fd, qd = f.detach(), feq.detach()
        D = qd - fd
        n = fd.shape[1]
        dS = kullback_dS(fd, qd)
        nonpos = (fd <= 0).any(0)
        cut = (dS < dS_cut) & ~nonpos
        ratio = torch.where(D < 0, fd / (-D).clamp(min=1e-300), torch.full_like(fd, math.inf))
        amax = ratio.min(0).values
        finite = torch.isfinite(amax)
        a_probe = torch.where(finite, amax, torch.full_like(amax, 2.0))
        sf_max, _, _ = _sf_parts(fd, D, qd, a_probe)
        noroot = ~cut & ~nonpos & finite & (sf_max >= 0)
        active = ~cut & ~nonpos & ~noroot
        nrm = torch.sqrt((D * D / qd).sum(0)) if norm == "entropic" else D.abs().sum(0)
        alpha = torch.where(amax > 2.0, torch.full_like(amax, 2.0), 0.5 * (1.0 + amax))
        todo = active.clone()
        for _ in range(max_iter):
            if not bool(todo.any()):
                break
            sf, d1, d2 = _sf_parts(fd, D, qd, alpha)
            stop = (sf / d1).abs() * nrm < eps
            todo = todo & ~stop
            disc = d1 * d1 - 2.0 * sf * d2
            par = 2.0 * sf / (-d1 + torch.sqrt(disc.clamp(min=0.0)))
            newton = -sf / d1
            delta = torch.where(disc >= 0, par, newton)
            anew = alpha + delta
            anew = torch.where(anew >= amax, 0.5 * (alpha + amax), anew)
            anew = torch.where(anew <= 1.0, 0.5 * (alpha + 1.0), anew)
            alpha = torch.where(todo, anew, alpha)
        sf, d1, _ = _sf_parts(fd, D, qd, alpha)
        alpha = torch.where(active & (sf < 0), alpha - 2.0 * sf / d1, alpha)
        fb = amax if fallback == "positivity" else torch.ones_like(amax)
        alpha = torch.where(noroot, fb, alpha)
        alpha = torch.where(cut, torch.full_like(alpha, 2.0), alpha)
        alpha = torch.where(nonpos, torch.ones_like(alpha), alpha)
        branch = torch.full((n,), ELBM_ROOT, dtype=torch.int64)
        branch[cut] = ELBM_CUTOFF
        branch[noroot] = ELBM_NOROOT
        branch[nonpos] = ELBM_NONPOS

    if not (torch.is_grad_enabled() and (f.requires_grad or feq.requires_grad)):
        return alpha, branch
    out = alpha.clone()
    # Implicit derivative at the root: d alpha = -(d_f S_f) / (d_alpha S_f).
    ridx = torch.nonzero(branch == ELBM_ROOT).flatten()
    if ridx.numel() > 0:
        fr, qr, ar = f[:, ridx], feq[:, ridx], alpha[ridx]
        sf, _, _ = _sf_parts(fr, qr - fr, qr, ar)
        _, d1, _ = _sf_parts(fr.detach(), (qr - fr).detach(), qr.detach(), ar)
        corr = -sf / d1
        out = out.index_put((ridx,), ar + (corr - corr.detach()))
    # Positivity fallback: alpha = alpha_max depends on f through the argmin.
    if fallback == "positivity":
        pidx = torch.nonzero(branch == ELBM_NOROOT).flatten()
        if pidx.numel() > 0:
            fp, qp = f[:, pidx], feq[:, pidx]
            Dp = qp - fp
            ratio = torch.where(Dp < 0, fp / (-Dp).clamp(min=1e-300),
                                torch.full_like(fp, math.inf))
            out = out.index_put((pidx,), ratio.min(0).values)
    return out, branch


def elbm(f, feq, omega, **kw):
    """ELBGK collision f + alpha beta (f* - f) with beta = omega / 2 and
    alpha from `elbm_alpha` (section 3).  f, feq: (Q, ny, nx)."""
    Q = f.shape[0]
    fl, ql = f.reshape(Q, -1), feq.reshape(Q, -1)
    alpha, branch = elbm_alpha(fl, ql, **kw)
    om = torch.as_tensor(omega, dtype=DT)
    beta = (om.reshape(-1) if om.dim() > 0 else om) / 2.0
    post = fl + alpha * beta * (ql - fl)
    return post.reshape(f.shape), alpha, branch


# ---------------------------------------------------------------------------
# Limiters (section 4).
# ---------------------------------------------------------------------------
def positivity(post, feq):
    """Positivity rule: a state with a negative component is replaced by the
    closest non-negative state on the line through it and f*, i.e.
    f* + phi (F - f*) with phi = min over F_i < 0 of f*_i / (f*_i - F_i).
    Reading: the component that attains the minimum is set to exactly 0;
    components with f*_i <= 0 are not eligible.  Returns (out, mask)."""
    neg = (post < 0) & (feq > 0)
    ratio = torch.where(neg, feq / (feq - post).clamp(min=1e-300), torch.full_like(post, math.inf))
    phi, arg = ratio.min(0)
    act = neg.any(0)
    phi_s = torch.where(act, phi, torch.ones_like(phi))
    out = feq + phi_s.unsqueeze(0) * (post - feq)
    onehot = torch.zeros_like(post, dtype=torch.bool).scatter_(0, arg.unsqueeze(0), True)
    out = torch.where(onehot & act.unsqueeze(0), torch.zeros_like(out), out)
    return torch.where(act.unsqueeze(0), out, post), act


def median_filter(lat: Lattice, cfg: Config, f, feq, dS, wall=None):
    """Median entropy filter (section 4): dS_med is the middle value of the
    neighbourhood of each site (itself included; 3 sites in 1D, 3x3 in 2D);
    where dS_med < dS the homothety f* + sqrt(dS_med / dS) (f - f*) is
    applied (eq. entrHom with the median as threshold).
    Reading: only neighbours inside the domain count (periodic directions
    wrap: both on a periodic lattice, x in the Couette channel);
    with n of them the median is the ceil(n/2)-th smallest (2nd of 3, 5th of
    9 as printed; 3rd of 6 and 2nd of 4 at walls).  Reading: the paper's
    delta (1e-3 in the Hopf study) is an acceptance threshold: only sites
    with dS > delta are filtered.  With diffusive walls (`wall`, the wall
    sites) only fluid sites filter and count as neighbours.
    Returns (f_new, mask)."""
    ny, nx = dS.shape
    offs = [(0, -1), (0, 0), (0, 1)] if lat.name == "D1Q3" else \
        [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    ys = torch.arange(ny).view(ny, 1)
    xs = torch.arange(nx).view(1, nx)
    vals, valid = [], []
    wrap_x = cfg.bc in ("periodic", "couette")    # Couette is periodic in x
    wrap_y = cfg.bc == "periodic"
    for dy, dx in offs:
        v = torch.roll(dS, shifts=(-dy, -dx), dims=(0, 1))   # v[y,x] = dS[y+dy, x+dx]
        sy, sx = ys + dy, xs + dx
        ok_y = torch.ones_like(sy, dtype=torch.bool) if wrap_y else (sy >= 0) & (sy < ny)
        ok_x = torch.ones_like(sx, dtype=torch.bool) if wrap_x else (sx >= 0) & (sx < nx)
        ok = (ok_y & ok_x).expand(ny, nx)
        if wall is not None:
            ok = ok & ~torch.roll(wall, shifts=(-dy, -dx), dims=(0, 1))
        vals.append(torch.where(ok, v, torch.full_like(v, math.inf)))
        valid.append(ok)
    stack = torch.stack(vals)
    n = torch.stack(valid).sum(0)
    # stable: among equal values the neighbour listed first holds the median
    # (decides only which neighbour a gradient flows to)
    srt = stack.sort(dim=0, stable=True).values
    rank = (n + 1) // 2 - 1                                   # ceil(n/2) - 1
    med = srt.gather(0, rank.unsqueeze(0)).squeeze(0)
    accept = (dS > cfg.med_delta) & (med < dS) & torch.isfinite(dS)
    if wall is not None:
        accept = accept & ~wall
    ratio = torch.where(accept, med / torch.where(accept, dS, torch.ones_like(dS)),
                        torch.ones_like(dS))
    # Reading (gradients only): a zero median maps the site onto f*; the
    # derivative of sqrt at 0 is infinite, so none is taken through it.
    pos = ratio > 0
    root = torch.sqrt(torch.where(pos, ratio, torch.ones_like(ratio)))
    coef = torch.where(accept, torch.where(pos, root, torch.zeros_like(root)), torch.ones_like(dS))
    return feq + coef.unsqueeze(0) * (f - feq), accept


def stencil_offsets(lat: Lattice):
    """The neighbourhood shifts y = (dy, dx) of the nonlocal filter in tensor
    order: 3 in 1D, the 3 x 3 block in 2D."""
    if lat.name == "D1Q3":
        return [(0, dx) for dx in (-1, 0, 1)]
    return [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def nonlocal_filter(lat: Lattice, f, feq, coef):
    """General nonlocal filter (section 4, "General nonlocal filters"): with
    f_neq = f - f*, every site takes f*(x) + sum_y d(y) f_neq(x + y), the sum
    over the neighbourhood shifts y (stencil_offsets) with the coefficients
    d(y) = coef.  Each f_neq(x + y) has zero density and momentum, so the
    filtered state keeps the moments (and f*) of x.
    Reading: the shifts must map the grid into itself, which on a finite
    lattice means a periodic one; the filter acts on the pre-collision state
    (after streaming), like the other filters of section 4."""
    offs = stencil_offsets(lat)
    if len(coef) != len(offs):
        raise ValueError(f"{lat.name} takes {len(offs)} filter coefficients")
    neq = f - feq
    acc = torch.zeros_like(neq)
    for c, (dy, dx) in zip(coef, offs):
        acc = acc + float(c) * torch.roll(neq, shifts=(-dy, -dx), dims=(1, 2))  # neq[., y+dy, x+dx]
    return feq + acc


def ens_threshold(dS: torch.Tensor, production: float, delta0: float) -> float:
    """Delta S_0 of eq. EntThresh over the lattice's own values (the
    histogram's density taken as the empirical distribution of Delta S):
    sum over sites with Delta S > Delta S_0 of (Delta S - Delta S_0) equals
    delta_0 times the LBGK entropy production `production`.  The left side
    falls continuously and piecewise linearly from sum Delta S (at 0) to 0
    (at the largest value); between consecutive values taken in descending
    order, with the j largest above the threshold, it is S_j - j s.
    Reading: sites with Delta S = +inf are left out."""
    v = torch.sort(dS[torch.isfinite(dS)].flatten(), descending=True).values
    rhs = delta0 * production
    if v.numel() == 0 or rhs <= 0:
        return float(v[0]) if v.numel() else 0.0
    cums = torch.cumsum(v, 0)
    if rhs >= float(cums[-1]):
        return 0.0
    nxt = torch.cat([v[1:], torch.zeros(1, dtype=v.dtype)])
    j = torch.arange(1, v.numel() + 1, dtype=v.dtype)
    lhs_at_next = cums - j * nxt         # the left side at the next value down
    i = int(torch.nonzero(lhs_at_next >= rhs)[0])
    return float((cums[i] - rhs) / (i + 1))


def ens_phi(cfg: "Config", dS: torch.Tensor, mean_dS: float, dS_t: float) -> torch.Tensor:
    """The coefficient phi of the limiter f* + phi (f - f*) at every site:
      threshold        sqrt(Delta S_t / Delta S) where Delta S >= Delta S_t
                       (eq. entrHom), else 1;
      smooth           (1 + r^(k - 1/2)) / (1 + r^k), r = Delta S /
                       (alpha E(Delta S))  (eq. phiExamp);
      double_monotone  (1 + (Delta S / Delta S_t)^k)^(-1/(2k))  (eq. DoublMonSpec);
      pointwise        1 / (1 + alpha Delta S^k)  (section 4, smooth limiters).
    Reading: a site with Delta S = +inf (a non-positive population) gets the
    common limit phi = 0, i.e. f*."""
    fin = torch.isfinite(dS)
    x = torch.where(fin, dS, torch.zeros_like(dS))
    if cfg.ens_limiter == "threshold":
        phi = torch.where(x >= dS_t, torch.sqrt(dS_t / torch.where(x > 0, x, torch.ones_like(x))),
                          torch.ones_like(x))
        phi = torch.where(x >= dS_t, phi, torch.ones_like(x))
    elif cfg.ens_limiter == "smooth":
        r = x / (cfg.ens_alpha * mean_dS)
        phi = (1 + r ** (cfg.ens_k - 0.5)) / (1 + r ** cfg.ens_k)
    elif cfg.ens_limiter == "double_monotone":
        phi = (1 + (x / dS_t) ** cfg.ens_k) ** (-1.0 / (2 * cfg.ens_k))
    elif cfg.ens_limiter == "pointwise":
        phi = 1.0 / (1.0 + cfg.ens_alpha * x ** cfg.ens_k)
    else:
        raise ValueError(cfg.ens_limiter)
    return torch.where(fin, phi, torch.zeros_like(phi))


def ensemble_limiter(cfg: "Config", f, feq, dS, omega):
    """Section 4, "Monitoring total dissipation": the LBGK entropy production
    of the step in quadratic approximation, [1 - (2 beta - 1)^2] sum Delta S
    with beta = omega / 2 (per site under an omega field), the threshold
    Delta S_t = max(Delta S_0, delta) from eq. EntThresh, the mean E(Delta S),
    and the limiter f* + phi (f - f*).  Returns (f_new, info) with the
    limiter's own production in the same approximation,
    sum (1 - phi^2) Delta S.  Reading: E(Delta S) and both sums are over the
    sites with finite Delta S.  delta_0 <= 0 fixes Delta S_t = delta (a
    pointwise threshold)."""
    om = torch.as_tensor(omega, dtype=DT)
    fin = torch.isfinite(dS)
    x = torch.where(fin, dS, torch.zeros_like(dS))
    c = 1.0 - (om - 1.0) ** 2
    production = float((c * x).sum())
    mean_dS = float(x.sum() / fin.sum().clamp(min=1))
    if cfg.ens_limiter not in ("threshold", "double_monotone"):
        dS_t = math.inf                  # the limiter has no threshold
    elif cfg.ens_delta0 > 0:
        dS_t = max(ens_threshold(dS.detach(), production, cfg.ens_delta0), cfg.ens_delta)
    else:
        dS_t = cfg.ens_delta
    phi = ens_phi(cfg, dS, mean_dS, dS_t)
    out = feq + phi.unsqueeze(0) * (f - feq)
    lim_production = float(((1.0 - phi.detach() ** 2) * x.detach()).sum())
    return out, {"lbgk_production": production, "limiter_production": lim_production,
                 "threshold": dS_t, "mean_dS": mean_dS, "phi": phi.detach()}


def ehrenfest_select(dS_flat: torch.Tensor, k: int, delta: float) -> torch.Tensor:
    """Ehrenfests' regularisation with a budget (section 4): the k sites with
    the highest Delta S > delta, ties broken by the lower linear index
    y * nx + x.  Returns the selected linear indices, sorted ascending."""
    idx = torch.nonzero(dS_flat > delta).flatten()
    if k <= 0 or idx.numel() == 0:
        return torch.zeros(0, dtype=torch.int64)
    order = torch.sort(-dS_flat[idx], stable=True).indices
    return torch.sort(idx[order[:k]]).values


# ---------------------------------------------------------------------------
# One step.
# ---------------------------------------------------------------------------
def step(lat: Lattice, cfg: Config, g: torch.Tensor,
         omega_field: Optional[torch.Tensor] = None):
    """One time step from the stored post-collision lattice g (Q, ny, nx).
    Returns (g_next, info).  Reading: the Ehrenfest step replaces the
    collision at the selected sites (f' = f*), and selection ranks the
    unfiltered Delta S; the median filter acts on the pre-collision state.
    Diffusive walls: the wall sites keep their streamed state after the wall
    rule (no collision, no limiter); they are neither selected nor counted
    as median neighbours."""
    pre = stream(lat, g, cfg.bc, cfg.u_lid, cfg.rho_wall)
    kind = "entropic" if cfg.collision == "elbm" else cfg.equilibrium
    wall = None
    if cfg.bc == "diffusive":
        if lat.name != "D2Q9" or cfg.ens_limiter != "none":
            raise ValueError("diffusive walls: D2Q9 without the ensemble limiters")
        pre = diffusive_wall(lat, pre, cfg.u_lid, kind)
        wall = wall_nodes(*pre.shape[1:])
    rho, jx, jy = moments(lat, pre)
    feq = equilibrium(lat, rho, jx / rho, jy / rho, kind)
    if cfg.nl_coef is not None:
        if cfg.bc != "periodic":
            raise ValueError("the nonlocal filter needs a periodic lattice")
        pre = nonlocal_filter(lat, pre, feq, cfg.nl_coef)
    omega = omega_field if omega_field is not None else relaxation_rate(cfg)
    info = {}
    dS = None
    if cfg.ehrenfest or cfg.median or cfg.ens_limiter != "none":
        dS = kullback_dS(pre, feq)
        info["dS"] = dS.detach()
    walls_pre = pre
    if cfg.median:
        pre, acc = median_filter(lat, cfg, pre, feq, dS, wall)
        info["median_mask"] = acc
    if cfg.ens_limiter != "none":
        pre, info["ensemble"] = ensemble_limiter(cfg, pre, feq, dS, omega)
    sel = None
    if cfg.ehrenfest:
        dS_sel = dS.detach() if wall is None else torch.where(wall, torch.zeros_like(dS), dS.detach())
        sel = ehrenfest_select(dS_sel.flatten(), cfg.ehr_k, cfg.ehr_delta)
        info["selected"] = sel
    def mrt_collision():
        se, seps, sq = mrt_preset_rates(cfg.mrt_preset, omega, cfg.s_e, cfg.s_eps, cfg.s_q)
        rates = mrt_rates(cfg.mrt_basis, se, seps, sq, omega)
        return mrt(pre, feq, mrt_basis(cfg.mrt_basis), rates)

    if cfg.collision == "lbgk":
        post = lbgk(pre, feq, omega)
    elif cfg.collision == "mrt":
        post = mrt_collision()
    elif cfg.collision == "elbm":
        post, alpha, branch = elbm(pre, feq, omega, eps=cfg.elbm_eps,
                                   max_iter=cfg.elbm_max_iter, dS_cut=cfg.elbm_dS_cut,
                                   norm=cfg.elbm_norm, fallback=cfg.elbm_fallback)
        info["alpha"] = alpha.detach().reshape(rho.shape)
        info["branch"] = branch.reshape(rho.shape)
        if wall is not None:
            info["branch"] = torch.where(wall, torch.full_like(info["branch"], -1), info["branch"])
    else:
        raise ValueError(cfg.collision)
    if cfg.positivity:
        # diagnostic only: where the collided state (before any Ehrenfest
        # step) has a negative population the rule acts
        info["positivity_collided"] = ((post < 0) & (feq > 0)).any(0)
        if wall is not None:
            info["positivity_collided"] = info["positivity_collided"] & ~wall
    selmask = torch.zeros(rho.numel(), dtype=torch.bool)
    if sel is not None and sel.numel() > 0:
        selmask[sel] = True
        selmask_q = selmask.view(1, *rho.shape)
        if cfg.sel_action == "mrt":
            # the MRT limiter: the MRT collision replaces LBGK's at the
            # selected sites (section 5)
            post = torch.where(selmask_q, mrt_collision(), post)
        else:
            post = torch.where(selmask_q, feq, post)
    if cfg.positivity:
        lim, act = positivity(post, feq)
        if cfg.sel_action != "mrt":
            # f* needs no positivity rule
            act = act & ~selmask.view(rho.shape)
        if wall is not None:
            act = act & ~wall
        post = torch.where(act.unsqueeze(0), lim, post)
        info["positivity_mask"] = act
    if wall is not None:
        post = torch.where(wall.unsqueeze(0), walls_pre, post)
    return post, info


def run(lat: Lattice, cfg: Config, g: torch.Tensor, n: int,
        omega_field: Optional[torch.Tensor] = None, keep_info: bool = False):
    infos = []
    for _ in range(n):
        g, info = step(lat, cfg, g, omega_field)
        if keep_info:
            infos.append(info)
    return (g, infos) if keep_info else g


def stats(lat: Lattice, g: torch.Tensor) -> dict:
    """Whole-lattice mass, momentum and entropy (sum over sites of
    -sum_i f_i ln(f_i / w_i)) in float64."""
    rho, jx, jy = moments(lat, g)
    return {"mass": float(rho.sum()), "mom_x": float(jx.sum()),
            "mom_y": float(jy.sum()), "entropy": float(entropy(lat, g).sum())}
