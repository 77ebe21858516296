"""GPU parity of the ensemble-dependent and smooth limiters of section 4
(threshold limiter with Delta S_t from eq. EntThresh, the smooth limiter of
eq. phiExamp, the double-monotone limiter of eq. DoublMonSpec, the pointwise
1/(1 + alpha Delta S^k)) and of the dissipation monitor, against the FP64
oracle on the same seeded states.

FP64 storage: populations within 1e-12 relative after one step (1e-10 after
20), the step's threshold Delta S_t and mean E(Delta S) within 1e-12, the
LBGK production and the limiter's own within 1e-11.  FP32 and FP16 storage:
the storage bound of the other parity tests, from the stored state."""
import pytest
import torch

import oracle as O
from tests.parity_util import gpu_run, lattice, oracle_run, random_state, rel_err

pytestmark = pytest.mark.gpu

NARROW = dict(nx=70, ny=37)
WIDE = dict(nx=300, ny=13)
CASES = {
    "threshold": dict(bc="periodic", nu=1e-3, ens_limiter="threshold", ens_delta0=0.05),
    "threshold_floor": dict(bc="periodic", nu=1e-3, ens_limiter="threshold", ens_delta0=0.05,
                            ens_delta=2e-3),
    # delta_0 P exceeds sum Delta S: Delta S_0 = 0 and the floor delta rules
    "threshold_large_budget": dict(bc="periodic", nu=0.1, ens_limiter="threshold",
                                   ens_delta0=1.2, ens_delta=1e-4),
    "smooth": dict(bc="periodic", nu=1e-3, ens_limiter="smooth", ens_alpha=1.5, ens_k=1.0),
    "smooth_k2_cavity": dict(bc="cavity", u_lid=0.1, nu=1e-3, ens_limiter="smooth",
                             ens_alpha=2.0, ens_k=2.0),
    "double_monotone": dict(bc="periodic", nu=1e-3, ens_limiter="double_monotone",
                            ens_delta0=0.05, ens_k=2.0),
    "double_monotone_fixed": dict(bc="cavity", u_lid=0.1, nu=1e-3, ens_limiter="double_monotone",
                                  ens_delta0=0.0, ens_delta=1e-4, ens_k=0.5),
    "pointwise": dict(bc="periodic", nu=1e-3, ens_limiter="pointwise", ens_alpha=100.0,
                      ens_k=0.5),
    "threshold_ehrenfest_pos": dict(bc="cavity", u_lid=0.1, nu=1e-4, ens_limiter="threshold",
                                    ens_delta0=0.02, ehrenfest=True, ehr_k=9, ehr_delta=0.0,
                                    positivity=True, _amp=0.5),
    "elbm_threshold": dict(bc="periodic", nu=1e-4, collision="elbm", ens_limiter="threshold",
                           ens_delta0=0.05),
    "mrt_smooth_cavity": dict(bc="cavity", u_lid=0.1, nu=1e-3, collision="mrt",
                              mrt_preset="mrt1", ens_limiter="smooth", ens_alpha=1.2, ens_k=1.0),
}


def _params(name, size):
    p = {"lattice": "D2Q9", **size, **CASES[name]}
    amp = p.pop("_amp", 0.2)
    return p, amp


def _kind(p):
    return "entropic" if p.get("collision") == "elbm" else "poly"


def _check_monitor(sim, info):
    st = sim.stats()
    ens = info["ensemble"]
    thr = ens["threshold"]
    if thr == float("inf") or thr == 0.0:
        assert st.ens_threshold == thr
    else:
        assert abs(st.ens_threshold - thr) <= 1e-12 * abs(thr), (st.ens_threshold, thr)
    if ens["mean_dS"] > 0:
        assert abs(st.ens_mean - ens["mean_dS"]) <= 1e-12 * ens["mean_dS"]
    P, Lp = ens["lbgk_production"], ens["limiter_production"]
    assert abs(st.lbgk_production - P) <= 1e-11 * abs(P)
    assert abs(st.limiter_production - Lp) <= 1e-11 * max(abs(Lp), 1e-3 * abs(P))
    return st


@pytest.mark.parametrize("size", ["narrow", "wide"])
@pytest.mark.parametrize("name", list(CASES))
def test_ensemble_one_step_fp64(name, size):
    p, amp = _params(name, NARROW if size == "narrow" else WIDE)
    f0 = random_state(p, 41, amp=amp, kind=_kind(p))
    _, f_gpu, sim = gpu_run(p, f0, 1, "f64")
    f_ora, infos = oracle_run(p, f0, 1)
    err = rel_err(f_gpu, f_ora)
    assert err <= 1e-12, f"max relative error {err:.3e}"
    st = _check_monitor(sim, infos[0])
    if p.get("ens_limiter") == "threshold" and p.get("ens_delta", 0.0) == 0.0:
        # the budget is spent exactly (eq. EntThresh with Delta S_t = Delta S_0)
        assert abs(st.limiter_production - p["ens_delta0"] * st.lbgk_production) <= \
            1e-10 * st.lbgk_production
    if p.get("ehrenfest"):
        assert sim.selected() == infos[0]["selected"].tolist()


@pytest.mark.parametrize("name", ["threshold", "smooth", "double_monotone",
                                  "threshold_ehrenfest_pos", "elbm_threshold"])
def test_ensemble_twenty_steps_fp64(name):
    p, amp = _params(name, NARROW)
    f0 = random_state(p, 43, amp=amp, kind=_kind(p))
    _, f_gpu, sim = gpu_run(p, f0, 20, "f64")
    f_ora, infos = oracle_run(p, f0, 20)
    err = rel_err(f_gpu, f_ora)
    assert err <= 1e-10, f"max relative error {err:.3e}"
    _check_monitor(sim, infos[-1])


@pytest.mark.parametrize("name", ["threshold", "smooth", "double_monotone_fixed", "pointwise"])
def test_ensemble_d1q3_fp64(name):
    p = {"lattice": "D1Q3", "nx": 300, "ny": 1, **CASES[name]}
    p.pop("_amp", None)
    if p["bc"] == "cavity":
        p["bc"], p["u_lid"] = "bounceback", 0.0
    f0 = random_state(p, 45, amp=0.2)
    _, f_gpu, sim = gpu_run(p, f0, 1, "f64")
    f_ora, infos = oracle_run(p, f0, 1)
    assert rel_err(f_gpu, f_ora) <= 1e-12
    _check_monitor(sim, infos[0])


ULP_BITS = {"f32": 23, "f16s": 10}
FP32_TERM = 8.0 * 2.0 ** -24


@pytest.mark.parametrize("storage", ["f32", "f16s"])
@pytest.mark.parametrize("name", ["threshold", "smooth", "double_monotone", "pointwise",
                                  "wide:threshold"])
def test_ensemble_low_precision_one_step(storage, name):
    size = WIDE if name.startswith("wide:") else NARROW
    p, amp = _params(name.split(":")[-1], size)
    f0 = random_state(p, 47, amp=amp, kind=_kind(p))
    f_in, f_gpu, sim = gpu_run(p, f0, 1, storage)
    f_ora, infos = oracle_run(p, f_in, 1)
    lat = lattice(p)
    g = f_ora - lat.col(lat.w) if storage == "f16s" else f_ora
    mag = g.abs().clamp(min=2.0 ** -14)
    bound = 0.5 * torch.pow(2.0, torch.floor(torch.log2(mag)) - ULP_BITS[storage]) + \
        FP32_TERM * f_ora.abs().clamp(min=1.0)
    excess = ((f_gpu - f_ora).abs() - bound).max()
    assert float(excess) <= 0, f"exceeds the storage bound by {float(excess):.3e}"
    st = sim.stats()
    thr = infos[0]["ensemble"]["threshold"]
    if 0 < thr < float("inf"):
        assert abs(st.ens_threshold - thr) <= 1e-5 * thr
