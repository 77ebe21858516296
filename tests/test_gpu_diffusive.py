"""GPU parity of the diffusive Maxwell wall (section 8, First Hopf
bifurcation) against the FP64 oracle: the wall rule on the outer ring of
nodes (the top row moving), wall nodes without collision, excluded from the
median neighbourhoods and from the Ehrenfest candidates; and the enstrophy
of the FP64 statistics.

FP64: one step from random states within 1e-12 relative (both tile shapes,
ragged), 200 steps of the 100^2 Hopf configuration from rest within 1e-10;
the median, no-root and non-positive counters equal the oracle's.  FP32 and
FP16 storage: the storage bound of the other parity tests."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from lbm_inputs import generators as G
from tests.parity_util import gpu_run, lattice, make_sim, oracle_config, oracle_run, \
    random_state, rel_err

pytestmark = pytest.mark.gpu

NARROW = dict(nx=70, ny=37)      # 64 x 4 tiles
WIDE = dict(nx=300, ny=13)       # 256 x 1 tiles
CASES = {
    "lbgk": dict(nu=0.01),
    "lbgk_entropic_median": dict(nu=1e-3, equilibrium="entropic", median=True, med_delta=1e-3),
    "elbm": dict(nu=1e-3, collision="elbm"),
    "mrt": dict(nu=0.01, collision="mrt"),
    "lbgk_ehrenfest_pos": dict(nu=1e-4, ehrenfest=True, ehr_k=12, ehr_delta=0.0,
                               positivity=True),
}


def _params(name, size):
    return {"lattice": "D2Q9", "bc": "diffusive", "u_lid": 0.1, **size, **CASES[name]}


def _kind(p):
    return "entropic" if p.get("collision") == "elbm" or p.get("equilibrium") == "entropic" \
        else "poly"


@pytest.mark.parametrize("size", ["narrow", "wide"])
@pytest.mark.parametrize("name", list(CASES))
def test_diffusive_one_step_fp64(name, size):
    p = _params(name, NARROW if size == "narrow" else WIDE)
    f0 = random_state(p, 61, amp=0.3 if "ehrenfest" in name else 0.1, kind=_kind(p))
    _, f_gpu, sim = gpu_run(p, f0, 1, "f64")
    f_ora, infos = oracle_run(p, f0, 1)
    err = rel_err(f_gpu, f_ora)
    assert err <= 1e-12, f"max relative error {err:.3e}"
    info = infos[0]
    c = sim.counters()
    if p.get("median"):
        assert c[1] == int(info["median_mask"].sum())
    if p.get("collision") == "elbm":
        assert c[2] == int((info["branch"] == O.ELBM_NOROOT).sum())
        assert c[4] == int((info["branch"] == O.ELBM_NONPOS).sum())
    if p.get("ehrenfest"):
        assert sorted(sim.selected()) == sorted(info["selected"].tolist())
        wall = O.wall_nodes(p["ny"], p["nx"]).flatten()
        assert not any(bool(wall[s]) for s in sim.selected())


ULP_BITS = {"f32": 23, "f16s": 10}
FP32_TERM = 8.0 * 2.0 ** -24


@pytest.mark.parametrize("storage", ["f32", "f16s"])
@pytest.mark.parametrize("name", ["lbgk", "lbgk_entropic_median", "elbm"])
def test_diffusive_low_precision_one_step(storage, name):
    p = _params(name, NARROW)
    f0 = random_state(p, 63, amp=0.1, kind=_kind(p))
    f_in, f_gpu, _ = gpu_run(p, f0, 1, storage)
    f_ora, _ = oracle_run(p, f_in, 1)
    lat = lattice(p)
    g = f_ora - lat.col(lat.w) if storage == "f16s" else f_ora
    mag = g.abs().clamp(min=2.0 ** -14)
    bound = 0.5 * torch.pow(2.0, torch.floor(torch.log2(mag)) - ULP_BITS[storage]) + \
        FP32_TERM * f_ora.abs().clamp(min=1.0)
    if p.get("collision") == "elbm":
        # the FP32 root solve resolves alpha to 5e-7
        pre = O.stream(lat, f_in, "diffusive")
        pre = O.diffusive_wall(lat, pre, 0.1, "entropic")
        r, jx, jy = O.moments(lat, pre)
        D = O.equilibrium(lat, r, jx / r, jy / r, "entropic") - pre
        bound = bound + 2 * 5e-7 * D.abs()
    excess = ((f_gpu - f_ora).abs() - bound).max()
    assert float(excess) <= 0, f"exceeds the storage bound by {float(excess):.3e}"


def _hopf_params(n=100, re=7500.0):
    u0 = 0.1
    return {"lattice": "D2Q9", "nx": n, "ny": n, "bc": "diffusive", "u_lid": u0,
            "nu": u0 * n / re, "equilibrium": "entropic", "median": True, "med_delta": 1e-3}


@pytest.mark.timeout(600)
def test_hopf_cavity_200_steps_fp64():
    """The 100^2 Hopf configuration (entropic equilibria, median filter
    delta 1e-3, lid 0.1, Re 7500) from rest, 200 steps, and its enstrophy."""
    p = _hopf_params()
    lat = lattice(p)
    rho, ux, uy = G.uniform_rest(p["nx"], p["ny"])
    f0 = O.init_equilibrium(lat, rho, ux, uy, "entropic")
    _, f_gpu, sim = gpu_run(p, f0, 200, "f64")
    f_ora, infos = oracle_run(p, f0, 200)
    err = rel_err(f_gpu, f_ora)
    assert err <= 1e-10, f"max relative error {err:.3e}"
    assert sim.counters()[1] == sum(int(i["median_mask"].sum()) for i in infos)
    ens_ora = O.enstrophy(lat, f_ora, "diffusive")
    ens_gpu = sim.stats().enstrophy
    assert ens_ora > 0 and abs(ens_gpu - ens_ora) <= 1e-11 * ens_ora, (ens_gpu, ens_ora)


@pytest.mark.parametrize("bc", ["periodic", "diffusive"])
def test_enstrophy_matches_oracle(bc):
    p = {"lattice": "D2Q9", "nx": 70, "ny": 37, "bc": bc, "u_lid": 0.1, "nu": 0.01}
    f0 = random_state(p, 65, amp=0.02)
    _, f_gpu, sim = gpu_run(p, f0, 3, "f64")
    ens = O.enstrophy(lattice(p), f_gpu, bc)
    assert abs(sim.stats().enstrophy - ens) <= 1e-12 * ens


def test_diffusive_rejects_unsupported_configurations():
    from paper_1110_0270_amd import lbm as B
    base = dict(lattice="D2Q9", nx=16, ny=16, bc="diffusive", u_lid=0.1, nu=0.01)
    for bad in (dict(checkpoint_every=4, max_steps=8), dict(ens_limiter="smooth"),
                dict(nx=2)):
        with pytest.raises(Exception):
            B.Simulation(B.make_config(**{**base, **bad}))
