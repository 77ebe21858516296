"""GPU parity of the adjoint (lbm_backward, called through the C ABI)
against the FP64 oracle's autograd gradient on the same seeded inputs.

Loss L = sum(w * f_T) with seeded weights w, so dL/df_T = w.  The library's
dL/df0 and per-site dL/d omega are compared with the oracle's gradients:
FP64 storage max |gpu - oracle| <= tol * max |oracle| with tol = 1e-11
(1e-9 through ELBM roots, which carry the root solve's 1e-14 tolerance
through the implicit derivative); FP32 storage 1e-4 (1e-3 ELBM), the
accumulated FP32 rounding of a few steps of forward recompute and adjoint;
FP16 shifted storage 5e-3 (the adjoint treats storage rounding as the
identity).
Rollouts span several checkpoint segments with a ragged last one, so the
recompute from checkpoints and the selection tape are exercised."""
import numpy as np
import pytest
import torch

import oracle as O
from tests.parity_util import lattice, make_sim, oracle_config, random_state

pytestmark = pytest.mark.gpu

NARROW = dict(nx=70, ny=37)
CASES = {
    "lbgk_periodic": dict(bc="periodic", omega=1.7),
    "lbgk_cavity_ehrenfest_pos": dict(bc="cavity", u_lid=0.1, omega=1.98, ehrenfest=True,
                                      ehr_k=9, ehr_delta=0.0, positivity=True, _amp=0.4),
    "lbgk_couette": dict(bc="couette", u_lid=0.05, nu=0.02),
    "lbgk_bounceback_entropic_eq": dict(bc="bounceback", nu=0.01, equilibrium="entropic"),
    "lbgk_positivity": dict(bc="periodic", omega=1.95, positivity=True, _amp=0.6),
    "mrt_m1_field_cavity": dict(bc="cavity", u_lid=0.1, collision="mrt", s_e=1.64,
                                s_eps=1.54, s_q=1.9, _field=True),
    "mrt_m2_periodic": dict(bc="periodic", nu=0.002, collision="mrt", mrt_basis="M2"),
    "mrt_ehrenfest_pos": dict(bc="cavity", u_lid=0.1, nu=1e-3, collision="mrt", s_e=1.64,
                              s_eps=1.64, s_q=1.9, ehrenfest=True, ehr_k=9, ehr_delta=1e-4,
                              positivity=True, _amp=0.3),
    "elbm_periodic": dict(bc="periodic", nu=1e-4, collision="elbm"),
    "elbm_field_cavity": dict(bc="cavity", u_lid=0.1, collision="elbm", _field=True),
    "elbm_far_positivity": dict(bc="periodic", nu=1e-4, collision="elbm", positivity=True,
                                _amp=0.6),
    "elbm_far_ehrenfest_rule": dict(bc="periodic", nu=1e-4, collision="elbm",
                                    elbm_fallback="ehrenfest", _amp=0.6),
    "elbm_ehrenfest": dict(bc="periodic", nu=1e-4, collision="elbm", ehrenfest=True,
                           ehr_k=12, ehr_delta=0.0, _amp=0.2),
    # more selected sites than the adjoint kernel reads into LDS: the mask path
    "lbgk_ehrenfest_k100_pos": dict(bc="periodic", omega=1.98, ehrenfest=True, ehr_k=100,
                                    ehr_delta=0.0, positivity=True, _amp=0.4),
    "d1q3_shock_ehrenfest": dict(lattice="D1Q3", nx=300, ny=1, bc="bounceback", nu=1e-4,
                                 ehrenfest=True, ehr_k=4, ehr_delta=0.0, _amp=0.2),
    "d1q3_elbm_periodic": dict(lattice="D1Q3", nx=300, ny=1, bc="periodic", nu=1e-4,
                               collision="elbm", _amp=0.2),
    # median entropy filter: the homothety's derivative through the site's
    # own Delta S and its median neighbour's
    "lbgk_median_periodic": dict(bc="periodic", nu=1e-3, median=True, med_delta=1e-5),
    "lbgk_median_cavity": dict(bc="cavity", u_lid=0.1, nu=1e-3, median=True, med_delta=1e-5),
    "mrt_median_field_cavity": dict(bc="cavity", u_lid=0.1, collision="mrt", s_e=1.64,
                                    s_eps=1.54, s_q=1.9, median=True, med_delta=1e-5,
                                    _field=True),
    "elbm_median": dict(bc="periodic", nu=1e-3, collision="elbm", median=True, med_delta=1e-5),
    "lbgk_median_ehrenfest_pos": dict(bc="periodic", omega=1.98, median=True, med_delta=1e-5,
                                      ehrenfest=True, ehr_k=9, ehr_delta=0.0, positivity=True,
                                      _amp=0.4),
    "d1q3_median_bb": dict(lattice="D1Q3", nx=300, ny=1, bc="bounceback", nu=1e-3,
                           median=True, med_delta=1e-5, _amp=0.1),
    # the MRT limiter (selected sites take the M2/C2 collision) and per-site
    # preset rates (dL/d omega through the TRT and shear-wave third-order
    # rates)
    "lbgk_mrt_limiter_pos": dict(bc="periodic", omega=1.98, ehrenfest=True, ehr_k=9,
                                 ehr_delta=0.0, sel_action="mrt", mrt_basis="M2",
                                 positivity=True, _amp=0.4),
    "lbgk_mrt_limiter_field_cavity": dict(bc="cavity", u_lid=0.1, ehrenfest=True, ehr_k=100,
                                          ehr_delta=0.0, sel_action="mrt", mrt_basis="M1",
                                          mrt_preset="trt", _field=True, _amp=0.2),
    "trt_field_cavity": dict(bc="cavity", u_lid=0.1, collision="mrt", mrt_preset="trt",
                             _field=True),
    "shear_field_periodic": dict(bc="periodic", collision="mrt", mrt_preset="shear",
                                 _field=True),
}


def _params(name):
    p = {"lattice": "D2Q9", **NARROW, **CASES[name]}
    amp = p.pop("_amp", 0.05)
    field = p.pop("_field", False)
    return p, amp, field


def _kind(p):
    return "entropic" if (p.get("collision") == "elbm" or p.get("equilibrium") == "entropic") else "poly"


def _omega_of(p):
    return O.relaxation_rate(oracle_config(p))


def _weights(shape, seed):
    return torch.tensor(np.random.default_rng(seed).normal(size=shape), dtype=torch.float64)


def _oracle_grad(p, f0, n, omega, w):
    """Gradients of sum(w * f_n) by the oracle's autograd; omega is a per-site
    tensor (a uniform one when the case has a scalar rate)."""
    lat, cfg = lattice(p), oracle_config(p)
    g0 = f0.clone().requires_grad_(True)
    om = omega.clone().requires_grad_(True)
    g = g0
    infos = []
    for _ in range(n):
        g, info = O.step(lat, cfg, g, om)
        infos.append(info)
    (g * w).sum().backward()
    return g.detach(), g0.grad, om.grad, infos


def _gpu_grad(p, f0, n, K, w, field, storage="f64", max_steps=None):
    sim = make_sim({**p, "checkpoint_every": K, "max_steps": max_steps or n,
                    "omega_field": field is not None}, storage)
    sim.set_populations(f0.to("cuda"))
    if field is not None:
        sim.set_omega(field.to("cuda"))
    sim.step(n)
    fT = sim.populations().cpu()
    g0 = torch.empty(sim.shape, dtype=torch.float64, device="cuda")
    gw = torch.empty((p["ny"], p["nx"]), dtype=torch.float64, device="cuda")
    sim.backward(w.to("cuda"), g0, gw)
    torch.cuda.synchronize()
    return sim, fT, g0.cpu(), gw.cpu()


def _field_for(p, field):
    if not field:
        return None
    from lbm_inputs import generators as G
    return torch.tensor(G.smooth_omega_field(p["nx"], p["ny"], seed=41), dtype=torch.float64)


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max().clamp(min=1e-300))


def _check_case(name, storage, n, K, tol64, tol32):
    p, amp, want_field = _params(name)
    field = _field_for(p, want_field)
    f0 = random_state(p, 23, amp=amp, kind=_kind(p))
    w = _weights(f0.shape, 29)
    omega = field if field is not None else torch.full((p["ny"], p["nx"]), _omega_of(p),
                                                       dtype=torch.float64)
    fT_o, g0_o, gw_o, infos = _oracle_grad(p, f0, n, omega, w)
    sim, fT, g0, gw = _gpu_grad(p, f0, n, K, w, field, storage)
    tol = tol64 if storage == "f64" else tol32
    e0, ew = _rel(g0, g0_o), _rel(gw, gw_o)
    assert e0 <= tol, f"dL/df0: {e0:.3e} > {tol:.0e}"
    assert ew <= tol, f"dL/domega: {ew:.3e} > {tol:.0e}"
    return sim, infos, fT, fT_o


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_fp64_matches_oracle_gradient(name):
    elbm = CASES[name].get("collision") == "elbm"
    sim, infos, fT, fT_o = _check_case(name, "f64", 5, 2, 1e-9 if elbm else 1e-11, None)
    # the branches the case is meant to exercise were taken
    if CASES[name].get("ehrenfest"):
        assert sum(int(i["selected"].numel()) for i in infos) > 0
    if CASES[name].get("positivity") and CASES[name].get("collision") != "elbm":
        assert sum(int(i["positivity_mask"].sum()) for i in infos) > 0
    if name.startswith("elbm_far"):
        assert any(bool((i["branch"] == O.ELBM_NOROOT).any()) for i in infos)
    if CASES[name].get("median"):
        assert sum(int(i["median_mask"].sum()) for i in infos) > 0
    # the backward pass leaves the final state in place
    assert torch.equal(sim.populations().cpu(), fT)


@pytest.mark.parametrize("name", ["lbgk_periodic", "mrt_m1_field_cavity",
                                  "lbgk_cavity_ehrenfest_pos", "elbm_periodic",
                                  "elbm_far_positivity", "lbgk_median_cavity",
                                  "elbm_median"])
def test_adjoint_fp32_storage(name):
    elbm = CASES[name].get("collision") == "elbm"
    _check_case(name, "f32", 4, 3, None, 1e-3 if elbm else 1e-4)


@pytest.mark.parametrize("n,K", [(1, 1), (6, 6), (7, 3), (9, 4)])
def test_adjoint_checkpoint_intervals(n, K):
    """Any interval gives the same gradient: full segments, one segment, and
    ragged last segments."""
    _check_case("mrt_ehrenfest_pos", "f64", n, K, 1e-11, None)


def test_adjoint_zero_steps_is_identity():
    p, amp, _ = _params("lbgk_periodic")
    f0 = random_state(p, 3, amp=amp)
    w = _weights(f0.shape, 5)
    sim, fT, g0, gw = _gpu_grad(p, f0, 0, 4, w, None, max_steps=4)
    assert torch.equal(g0, w)
    assert torch.equal(gw, torch.zeros_like(gw))


def test_adjoint_repeatable_and_after_more_steps():
    """Two backward calls on one rollout agree bit for bit; stepping further
    extends the recorded rollout."""
    p, amp, _ = _params("lbgk_cavity_ehrenfest_pos")
    f0 = random_state(p, 7, amp=amp)
    w = _weights(f0.shape, 9)
    sim = make_sim({**p, "checkpoint_every": 3, "max_steps": 8}, "f64")
    sim.set_populations(f0.to("cuda"))
    sim.step(2)
    sim.step(3)
    a = torch.empty(sim.shape, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    sim.backward(w.to("cuda"), a)
    sim.backward(w.to("cuda"), b)
    assert torch.equal(a, b)
    omega = torch.full((p["ny"], p["nx"]), _omega_of(p), dtype=torch.float64)
    _, g0_o, _, _ = _oracle_grad(p, f0, 5, omega, w)
    assert _rel(a.cpu(), g0_o) <= 1e-11


def test_adjoint_errors():
    from paper_1110_0270_amd import lbm as B
    p, amp, _ = _params("lbgk_periodic")
    f0 = random_state(p, 3, amp=amp).to("cuda")
    g = torch.empty_like(f0)
    sim = make_sim(p, "f64")                      # no checkpointing
    sim.set_populations(f0)
    sim.step(1)
    with pytest.raises(B.LBMError) as e:
        sim.backward(f0, g)
    assert e.value.status == B.LBM_ESTATE
    sim = make_sim({**p, "checkpoint_every": 2, "max_steps": 3}, "f64")
    sim.set_populations(f0)
    with pytest.raises(B.LBMError) as e:
        sim.step(4)                               # longer than max_steps
    assert e.value.status == B.LBM_ESTATE


def test_rollout_autograd_function():
    """LBMRollout (torch.autograd.Function over the library) returns the
    oracle's gradient for f0 and the omega field."""
    from paper_1110_0270_amd import lbm as B
    p, amp, _ = _params("mrt_m1_field_cavity")
    field = _field_for(p, True)
    f0 = random_state(p, 31, amp=amp)
    w = _weights(f0.shape, 37)
    sim = make_sim({**p, "checkpoint_every": 2, "max_steps": 4, "omega_field": True}, "f64")
    f0d = f0.to("cuda").requires_grad_(True)
    omd = field.to("cuda").requires_grad_(True)
    fT = B.LBMRollout.apply(f0d, omd, sim, 4)
    (fT * w.to("cuda")).sum().backward()
    _, g0_o, gw_o, _ = _oracle_grad(p, f0, 4, field, w)
    assert _rel(f0d.grad.cpu(), g0_o) <= 1e-11
    assert _rel(omd.grad.cpu(), gw_o) <= 1e-11


def test_rollout_backward_refuses_a_replaced_rollout():
    """The Simulation records one rollout: once a second LBMRollout.apply (or
    a further step) has replaced it, the first graph's backward raises
    instead of returning gradients of another rollout."""
    from paper_1110_0270_amd import lbm as B
    p, amp, _ = _params("lbgk_periodic")
    f0 = random_state(p, 3, amp=amp).to("cuda")
    sim = make_sim({**p, "checkpoint_every": 2, "max_steps": 6}, "f64")
    a = f0.clone().requires_grad_(True)
    fa = B.LBMRollout.apply(a, None, sim, 3)
    b = (1.01 * f0).requires_grad_(True)
    fb = B.LBMRollout.apply(b, None, sim, 2)
    with pytest.raises(RuntimeError, match="rollout"):
        fa.sum().backward()
    fb.sum().backward()                      # the current rollout still works
    assert b.grad is not None and bool(torch.isfinite(b.grad).all())
    c = f0.clone().requires_grad_(True)
    fc = B.LBMRollout.apply(c, None, sim, 2)
    sim.step(1)
    with pytest.raises(RuntimeError, match="rollout"):
        fc.sum().backward()


def test_adjoint_full_size_directional_derivative():
    """The cavity adjoint workload's configuration (512^2, MRT with an omega
    field, Ehrenfest k = 9) in FP64 over 48 steps, checkpoints every 16:
    <dL/df0, v> and <dL/domega, z> equal central differences of the
    library's own forward pass (the oracle cannot run this size)."""
    from lbm_inputs.workloads import workload
    wl = workload("cavity_adjoint_512")
    p = {k: wl[k] for k in ("lattice", "nx", "ny", "bc", "u_lid", "collision", "s_e", "s_eps",
                            "s_q", "ehrenfest", "ehr_k", "ehr_delta")}
    field = _field_for(p, True)
    f0 = random_state(p, 43, amp=0.05)
    rng = np.random.default_rng(47)
    w = torch.tensor(rng.normal(size=f0.shape))
    v = torch.tensor(rng.normal(size=f0.shape))
    z = torch.tensor(rng.normal(size=field.shape))
    n = 48
    sim, fT, g0, gw = _gpu_grad(p, f0, n, 16, w, field)
    wd = w.to("cuda")

    def loss(f, om):
        s = make_sim({**p, "omega_field": True}, "f64")
        s.set_populations(f.to("cuda"))
        s.set_omega(om.to("cuda"))
        s.step(n)
        return float((s.populations() * wd).sum())

    h = 1e-6
    fd = (loss(f0 + h * v, field) - loss(f0 - h * v, field)) / (2 * h)
    ad = float((g0 * v).sum())
    assert abs(ad - fd) <= 1e-6 * abs(ad)
    fdw = (loss(f0, field + h * z) - loss(f0, field - h * z)) / (2 * h)
    adw = float((gw * z).sum())
    assert abs(adw - fdw) <= 1e-6 * abs(adw)


def _cavity_copy(n=64):
    """The cavity adjoint workload's setup on an n x n copy: MRT with the
    seeded per-site shear rate, Ehrenfest k = 9, delta = 1e-3, fluid at rest,
    the seeded Fourier target velocity."""
    from lbm_inputs import generators as G
    from lbm_inputs.workloads import workload
    wl = workload("cavity_adjoint_512")
    p = {k: wl[k] for k in ("lattice", "bc", "u_lid", "collision", "s_e", "s_eps", "s_q",
                            "ehrenfest", "ehr_k", "ehr_delta")}
    p.update(nx=n, ny=n)
    field = torch.tensor(G.smooth_omega_field(n, n, seed=wl["omega_seed"]))
    rho, ux, uy = G.uniform_rest(n, n)
    f0 = O.init_equilibrium(lattice(p), rho, ux, uy)
    tx, ty = (torch.tensor(a) for a in G.fourier_target(n, n, seed=wl["target_seed"]))
    return p, field, f0, tx, ty


def _misfit(f, tx, ty):
    rho = f.sum(0)
    v = torch.tensor([[(i % 3) - 1, (i // 3) - 1] for i in range(9)], dtype=f.dtype,
                     device=f.device)
    ux = (v[:, 0].view(9, 1, 1) * f).sum(0) / rho
    uy = (v[:, 1].view(9, 1, 1) * f).sum(0) / rho
    return ((ux - tx.to(f.device)) ** 2 + (uy - ty.to(f.device)) ** 2).sum()


def _misfit_grad(fT, tx, ty):
    f = fT.clone().requires_grad_(True)
    _misfit(f, tx, ty).backward()
    return f.grad


def test_cavity_copy_velocity_misfit_matches_oracle():
    """64^2 copy of the cavity adjoint workload, 40 steps, checkpoints every
    16: gradients of the velocity misfit equal the oracle's autograd."""
    p, field, f0, tx, ty = _cavity_copy()
    n = 40
    lat, cfg = lattice(p), oracle_config(p)
    g0 = f0.clone().requires_grad_(True)
    om = field.clone().requires_grad_(True)
    g = g0
    for _ in range(n):
        g, _ = O.step(lat, cfg, g, om)
    _misfit(g, tx, ty).backward()
    sim = make_sim({**p, "checkpoint_every": 16, "max_steps": n, "omega_field": True}, "f64")
    sim.set_populations(f0.to("cuda"))
    sim.set_omega(field.to("cuda"))
    sim.step(n)
    dLdfT = _misfit_grad(sim.populations(), tx, ty)
    gf = torch.empty_like(dLdfT)
    gw = torch.empty((p["ny"], p["nx"]), dtype=torch.float64, device="cuda")
    sim.backward(dLdfT, gf, gw)
    assert _rel(gf.cpu(), g0.grad) <= 1e-11
    assert _rel(gw.cpu(), om.grad) <= 1e-11


def test_cavity_copy_8192_steps_central_differences():
    """64^2 copy of the cavity adjoint workload over the full 8192 steps in
    FP64 with checkpoints every 256: directional derivatives of the velocity
    misfit along seeded directions in f0 and omega equal central
    differences of the library's forward pass (h = 1e-6; the final
    Ehrenfest sets of the +-h runs are equal).  The rest state is perturbed
    by a seeded relative 1e-3: at rest the two lid corners tie exactly in
    Delta S at the first step, where the loss is not differentiable.  From
    the perturbed start the oracle's smallest selection margin over the
    8192 steps (k-th against (k+1)-th Delta S, or against delta) is 7e-5
    relative, far above what the 1e-8 perturbations move."""
    p, field, f0, tx, ty = _cavity_copy()
    f0 = f0 * (1 + 1e-3 * torch.tensor(np.random.default_rng(59).uniform(-1, 1, f0.shape)))
    n = 8192
    rng = np.random.default_rng(53)
    v = torch.tensor(rng.normal(size=f0.shape)) * 1e-2
    z = torch.tensor(rng.normal(size=field.shape)) * 1e-2
    sim = make_sim({**p, "checkpoint_every": 256, "max_steps": n, "omega_field": True}, "f64")
    sim.set_populations(f0.to("cuda"))
    sim.set_omega(field.to("cuda"))
    sim.step(n)
    dLdfT = _misfit_grad(sim.populations(), tx, ty)
    gf = torch.empty_like(dLdfT)
    gw = torch.empty((p["ny"], p["nx"]), dtype=torch.float64, device="cuda")
    sim.backward(dLdfT, gf, gw)
    sel_ref = sim.selected()

    def loss(f, om):
        s = make_sim({**p, "omega_field": True}, "f64")
        s.set_populations(f.to("cuda"))
        s.set_omega(om.to("cuda"))
        s.step(n)
        return float(_misfit(s.populations(), tx, ty)), s.selected()

    h = 1e-6
    (lp, sp), (lm, sm) = loss(f0 + h * v, field), loss(f0 - h * v, field)
    assert sp == sel_ref and sm == sel_ref
    ad = float((gf.cpu() * v).sum())
    assert abs(ad - (lp - lm) / (2 * h)) <= 1e-6 * abs(ad)
    (lp, sp), (lm, sm) = loss(f0, field + h * z), loss(f0, field - h * z)
    assert sp == sel_ref and sm == sel_ref
    adw = float((gw.cpu() * z).sum())
    assert abs(adw - (lp - lm) / (2 * h)) <= 1e-6 * abs(adw)


@pytest.mark.parametrize("name,storage,tol", [
    ("elbm_periodic", "f32", 1e-3),          # row-pipelined kernel keeps alpha in the recompute
    ("elbm_periodic", "f64", 1e-9),
    ("lbgk_cavity_ehrenfest_pos", "f32", 1e-4),
    ("lbgk_periodic", "f16s", 5e-3),          # 16-bit storage: row kernel, storage rounding
    ("mrt_m1_field_cavity", "f32", 1e-4),
])
def test_adjoint_row_tiles(name, storage, tol):
    """The adjoint on 300 x 13 lattices (256-site row tiles; periodic 16-bit
    and FP32 ELBM steps run the row-pipelined kernel), 6 steps with
    checkpoints every 4, against the oracle's FP64 gradient from the state
    the library stores."""
    p, amp, want_field = _params(name)
    p.update(nx=300, ny=13)
    field = _field_for(p, want_field)
    f0 = random_state(p, 67, amp=amp, kind=_kind(p))
    w = _weights(f0.shape, 71)
    sim = make_sim({**p, "checkpoint_every": 4, "max_steps": 6,
                    "omega_field": field is not None}, storage)
    sim.set_populations(f0.to("cuda"))
    f_in = sim.populations().cpu()
    if field is not None:
        sim.set_omega(field.to("cuda"))
    sim.step(6)
    g0 = torch.empty(sim.shape, dtype=torch.float64, device="cuda")
    gw = torch.empty((p["ny"], p["nx"]), dtype=torch.float64, device="cuda")
    sim.backward(w.to("cuda"), g0, gw)
    torch.cuda.synchronize()
    omega = field if field is not None else torch.full((p["ny"], p["nx"]), _omega_of(p),
                                                       dtype=torch.float64)
    _, g0_o, gw_o, _ = _oracle_grad(p, f_in, 6, omega, w)
    e0, ew = _rel(g0.cpu(), g0_o), _rel(gw.cpu(), gw_o)
    assert e0 <= tol, f"dL/df0: {e0:.3e}"
    assert ew <= tol, f"dL/domega: {ew:.3e}"
