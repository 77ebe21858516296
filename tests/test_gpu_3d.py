"""GPU parity of the D3Q27 step (LBGK, the 27-site median entropy filter of
section 4, the positivity rule) against the FP64 oracle, called through the
C ABI.

Bars: FP64 storage, one step from identical states: elementwise
|gpu - oracle| <= 1e-12 max(|oracle|, 1e-3); 20 steps: 1e-10; the median
and positivity counters equal the oracle's masks.  FP32 and FP16 storage:
half an ulp of the stored deviation plus 8 FP32 roundings of the
population, except at sites whose median decision is a tie within FP32's
resolution of Delta S (1e-4 relative; a site whose own value is the
median decides alike in both), which are counted and kept rare.
The 70 x 13 x 19 lattice is ragged in every direction for both kernels
(64 x 8 tiles and 16-layer chunks of the median kernel; 256-site rows of
the plain one)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from lbm_inputs import generators as G
from tests.parity_util import gpu_run, make_sim, rel_err

pytestmark = pytest.mark.gpu

SIZE = dict(nx=70, ny=13, nz=19)
CASES = {
    "lbgk": dict(nu=0.01),
    "lbgk_entropic": dict(nu=1e-3, equilibrium="entropic"),
    "median": dict(nu=1e-3, median=True, med_delta=1e-5),
    "median_entropic_all": dict(nu=1e-3, equilibrium="entropic", median=True, med_delta=0.0),
    "positivity": dict(nu=1e-4, positivity=True, _amp=0.6),
    "median_positivity": dict(nu=1e-4, median=True, med_delta=1e-5, positivity=True, _amp=0.5),
}
FIELDS3 = {f.name for f in dataclasses.fields(O.Config3)}


def _params(name, size=SIZE):
    d = dict(CASES[name])
    amp = d.pop("_amp", 0.1)
    return {"lattice": "D3Q27", "bc": "periodic", **size, **d}, amp


def random_state3(p, seed, amp=0.1, umax=0.08):
    rng = np.random.default_rng(seed)
    shape = (p["nz"], p["ny"], p["nx"])
    rho = 1.0 + 0.1 * rng.uniform(-1, 1, shape)
    u = [umax * rng.uniform(-1, 1, shape) for _ in range(3)]
    f = O.init_equilibrium3(rho, *u, p.get("equilibrium", "poly"))
    return f * (1.0 + torch.tensor(G.uniform_noise(f.shape, seed + 1000, amp)))


def oracle3(p, f0, n):
    cfg = O.Config3(**{k: v for k, v in p.items() if k in FIELDS3})
    g, infos = f0.clone(), []
    for _ in range(n):
        g, info = O.step3(cfg, g)
        infos.append(info)
    return g, infos


@pytest.mark.parametrize("name", list(CASES))
def test_d3q27_one_step_fp64(name):
    p, amp = _params(name)
    f0 = random_state3(p, 71, amp)
    _, f_gpu, sim = gpu_run(p, f0, 1, "f64")
    f_ora, infos = oracle3(p, f0, 1)
    err = rel_err(f_gpu, f_ora)
    assert err <= 1e-12, f"max relative error {err:.3e}"
    c = sim.counters()
    if p.get("median"):
        assert c[1] == int(infos[0]["median_mask"].sum()) and c[1] > 0
    if p.get("positivity"):
        assert c[0] == int(infos[0]["positivity_mask"].sum()) and c[0] > 0


@pytest.mark.parametrize("name", ["median", "median_entropic_all", "median_positivity"])
def test_d3q27_twenty_steps_fp64(name):
    p, amp = _params(name)
    f0 = random_state3(p, 72, amp)
    _, f_gpu, sim = gpu_run(p, f0, 20, "f64")
    f_ora, infos = oracle3(p, f0, 20)
    err = rel_err(f_gpu, f_ora)
    assert err <= 1e-10, f"max relative error {err:.3e}"
    assert sim.counters()[1] == sum(int(i["median_mask"].sum()) for i in infos)


@pytest.mark.parametrize("shape", [(3, 2, 1), (1, 4, 2), (9, 1, 3), (2, 2, 2)])
def test_d3q27_degenerate_lattices_fp64(shape):
    """Extents of 1 and 2 (every neighbour wraps onto the same few sites)."""
    nx, ny, nz = shape
    p, amp = _params("median_positivity", dict(nx=nx, ny=ny, nz=nz))
    f0 = random_state3(p, 73, amp)
    _, f_gpu, _ = gpu_run(p, f0, 3, "f64")
    f_ora, _ = oracle3(p, f0, 3)
    assert rel_err(f_gpu, f_ora) <= 1e-12


ULP_BITS = {"f32": 23, "f16s": 10}
FP32_TERM = 8.0 * 2.0 ** -24


def _median_ties(p, f_in):
    """Sites whose median decision the oracle takes within 1e-4 relative of
    a tie (the median against Delta S, or Delta S against delta)."""
    cfg = O.Config3(**{k: v for k, v in p.items() if k in FIELDS3})
    pre = O.stream3(f_in)
    r, jx, jy, jz = O.moments3(pre)
    feq = O.equilibrium3(r, jx / r, jy / r, jz / r, cfg.equilibrium)
    dS = O.kullback_dS(pre, feq)
    vals = torch.stack([torch.roll(dS, shifts=(-a, -b, -c), dims=(0, 1, 2))
                        for (a, b, c) in O.stencil_offsets3()])
    med = vals.sort(0).values[13]
    # a site whose own value is the median (one in 27) decides exactly alike
    # in both precisions; only the others near a tie can flip
    near = ((med - dS).abs() <= 1e-4 * dS.abs()) & (med != dS)
    return near | ((dS - cfg.med_delta).abs() <= 1e-4 * dS.abs())


@pytest.mark.parametrize("storage", ["f32", "f16s"])
@pytest.mark.parametrize("name", ["lbgk", "median", "median_positivity", "median:tall"])
def test_d3q27_low_precision_one_step(storage, name):
    """tall: 70 x 20 x 40 spans two rows of 64 x 16 tiles and two 32-layer
    chunks of the FP32-arithmetic median kernel, both ragged."""
    name, _, size = name.partition(":")
    p, amp = _params(name, dict(nx=70, ny=20, nz=40) if size == "tall" else SIZE)
    f0 = random_state3(p, 74, amp)
    f_in, f_gpu, _ = gpu_run(p, f0, 1, storage)
    f_ora, _ = oracle3(p, f_in, 1)
    w = O.Lattice3().w.view(27, 1, 1, 1)
    g = f_ora - w if storage == "f16s" else f_ora
    mag = g.abs().clamp(min=2.0 ** -14)
    bound = 0.5 * torch.pow(2.0, torch.floor(torch.log2(mag)) - ULP_BITS[storage]) + \
        FP32_TERM * f_ora.abs().clamp(min=1.0)
    if p.get("positivity"):
        # the rule's factor f*_j / (f*_j - F_j) amplifies the rounding of F_j
        bound = bound * 16
    excess = (f_gpu - f_ora).abs() - bound
    bad = (excess > 0).any(0)
    if p.get("median"):
        ties = _median_ties(p, f_in)
        assert int(ties.sum()) <= 0.01 * ties.numel()
        bad = bad & ~ties
    assert not bool(bad.any()), f"{int(bad.sum())} sites beyond the storage bound"


def _spotty_state(p, seed, frac=0.03):
    """A uniform flow with 1e-4 noise (Delta S near 1e-9 after streaming) and
    strongly perturbed populations at a fraction of the sites: with delta
    between the two, half of the sites lie far below delta, while the
    neighbourhoods of the spots hold candidates whose median is often one
    of those small values."""
    rng = np.random.default_rng(seed)
    shape = (p["nz"], p["ny"], p["nx"])
    ones = np.ones(shape)
    f = O.init_equilibrium3(ones, 0.02 * ones, -0.01 * ones, 0.015 * ones, "poly")
    small = torch.tensor(G.uniform_noise(f.shape, seed + 1000, 1e-4))
    big = torch.tensor(G.uniform_noise(f.shape, seed + 2000, 0.3))
    spots = torch.tensor(rng.random(shape) < frac).unsqueeze(0)
    return f * (1.0 + torch.where(spots, big, small))


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_d3q27_median_small_neighbourhoods(storage):
    """delta = 1e-6 on the spotty state (about 6.7 k accepted sites of
    17 k, 1.3 k of them with a median below delta).  Against the oracle:
    FP64 at 1e-12 with the median counter equal to the oracle's mask; FP32
    within the storage bound away from near-tie median decisions."""
    p, _ = _params("median")
    p["med_delta"] = 1e-6
    f0 = _spotty_state(p, 76)
    f_in, f_gpu, sim = gpu_run(p, f0, 1, storage)
    f_ora, infos = oracle3(p, f_in, 1)
    n_med = int(infos[0]["median_mask"].sum())
    assert n_med > 0
    if storage == "f64":
        assert rel_err(f_gpu, f_ora) <= 1e-12
        assert sim.counters()[1] == n_med
    else:
        mag = f_ora.abs().clamp(min=2.0 ** -14)
        bound = 0.5 * torch.pow(2.0, torch.floor(torch.log2(mag)) - ULP_BITS["f32"]) + \
            FP32_TERM * f_ora.abs().clamp(min=1.0)
        bad = (((f_gpu - f_ora).abs() - bound) > 0).any(0) & ~_median_ties(p, f_in)
        assert not bool(bad.any()), f"{int(bad.sum())} sites beyond the storage bound"


def test_d3q27_set_equilibrium3d_and_stats():
    p = {"lattice": "D3Q27", "bc": "periodic", **SIZE, "nu": 0.01, "equilibrium": "entropic"}
    rho, ux, uy, uz = G.taylor_green_3d(p["nx"], p["ny"], p["nz"], u0=0.05)
    uz = uz + 0.01 * np.sin(2 * np.pi * np.arange(p["nx"]) / p["nx"])
    sim = make_sim(p, "f64")
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")  # noqa: E731
    sim.set_equilibrium3d(t(rho), t(ux), t(uy), t(uz))
    f = sim.populations().cpu()
    want = O.init_equilibrium3(rho, ux, uy, uz, "entropic")
    assert rel_err(f, want) <= 1e-14
    sim.step(2)
    st = sim.stats()
    ref = O.stats3(sim.populations().cpu())
    for k in ("mass", "mom_x", "mom_y", "mom_z", "entropy"):
        assert abs(getattr(st, k) - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), k
    assert st.enstrophy == 0.0


def _window_oracle(p, f_in, site):
    """The oracle's result at one site of a large periodic lattice: the 5^3
    block around it (wrapped) stepped as a periodic lattice of its own;
    its centre sees exactly the populations and neighbour Delta S values of
    the full lattice."""
    nz, ny, nx = f_in.shape[1:]
    z, y, x = site
    iz = [(z + d) % nz for d in range(-2, 3)]
    iy = [(y + d) % ny for d in range(-2, 3)]
    ix = [(x + d) % nx for d in range(-2, 3)]
    blk = f_in[:, iz][:, :, iy][:, :, :, ix].clone()
    cfg = O.Config3(**{k: v for k, v in p.items() if k in FIELDS3})
    out, _ = O.step3(cfg, blk)
    return out[:, 2, 2, 2]


@pytest.mark.timeout(600)
def test_d3q27_median_full_size_sampled_fp32():
    """The 256^3 Taylor-Green workload in FP32 with the median filter, the
    launch configuration the benchmark times: 200 sampled sites against the
    oracle, mass and momentum conserved."""
    n = 256
    p = {"lattice": "D3Q27", "bc": "periodic", "nx": n, "ny": n, "nz": n, "nu": 1e-5,
         "median": True, "med_delta": 0.0}
    rho, ux, uy, uz = G.taylor_green_3d(n, u0=0.05)
    sim = make_sim(p, "f32")
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    sim.set_equilibrium3d(t(rho), t(ux), t(uy), t(uz))
    del rho, ux, uy, uz
    sim.step(4)
    s0 = sim.stats()
    f_in = sim.populations().cpu()          # the stored values, exactly
    sim.step(1)
    s1 = sim.stats()
    f_out = sim.populations().cpu()
    rng = np.random.default_rng(5)
    sites = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(200)]
    for s in sites:
        want = _window_oracle(p, f_in, s)
        got = f_out[:, s[0], s[1], s[2]]
        assert float((got - want).abs().max()) <= 2e-7, s
    assert abs(s1.mass - s0.mass) <= 1e-9 * s0.mass
    for k in ("mom_x", "mom_y", "mom_z"):
        assert abs(getattr(s1, k) - getattr(s0, k)) <= 1e-9 * s0.mass, k
    assert sim.counters()[1] > 0
