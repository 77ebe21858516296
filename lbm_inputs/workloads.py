"""The synthetic workloads, as plain parameter sets.

Each entry names the lattice, the grid, the boundary, the collision, the
limiters with their parameters, the step count and the storage forms, plus
the name of the generator that produces its initial macroscopic fields.
Physical parameters are given as the kinematic viscosity nu (lattice units);
each implementation converts nu to its relaxation rate itself.
"""
from __future__ import annotations

import math

WORKLOADS = {
    # D1Q3 shock tube, 800 nodes, bounce-back ends, LBGK + Ehrenfest top-4.
    "shock_tube_1d": dict(
        lattice="D1Q3", nx=800, ny=1, bc="bounceback", u_lid=0.0,
        collision="lbgk", equilibrium="poly", nu=1e-9,
        ehrenfest=True, ehr_k=4, ehr_delta=1e-3,
        median=False, med_delta=1e-3, positivity=False,
        steps=400, storages=("f64",), init="shock_tube_1d", seed=1),
    # D2Q9 lid-driven cavity 256^2, Re 5000 at lid speed 0.1: nu = 0.1*256/5000.
    "cavity_256": dict(
        lattice="D2Q9", nx=256, ny=256, bc="cavity", u_lid=0.1,
        collision="lbgk", equilibrium="poly", nu=0.1 * 256 / 5000.0,
        ehrenfest=False, ehr_k=0, ehr_delta=0.0,
        median=False, med_delta=1e-3, positivity=False,
        s_e=1.64, s_eps=1.64, s_q=1.9,
        runs=("lbgk", "elbm", "mrt", "lbgk_median"),
        steps=50000, storages=("f64", "f32"), init="uniform_rest", seed=3),
    # D2Q9 periodic double shear layer 4096^2, LBGK + Ehrenfest on 0.1 % of sites.
    "shear_layer_4096": dict(
        lattice="D2Q9", nx=4096, ny=4096, bc="periodic", u_lid=0.0,
        collision="lbgk", equilibrium="poly", nu=1e-5,
        ehrenfest=True, ehr_k=math.ceil(0.001 * 4096 * 4096), ehr_delta=0.0,
        median=False, med_delta=1e-3, positivity=False,
        steps=20000, storages=("f64", "f32", "f16s", "bf16s"),
        init="double_shear_layer", seed=3),
    # D2Q9 cavity 512^2 adjoint: MRT with a per-site shear rate + Ehrenfest top-9.
    "cavity_adjoint_512": dict(
        lattice="D2Q9", nx=512, ny=512, bc="cavity", u_lid=0.1,
        collision="mrt", equilibrium="poly", nu=None,
        s_e=1.64, s_eps=1.64, s_q=1.9, omega_field=True, omega_seed=41,
        ehrenfest=True, ehr_k=9, ehr_delta=1e-3,
        median=False, med_delta=1e-3, positivity=False,
        steps=8192, checkpoint_every=256, storages=("f32",),
        target_seed=4, fd_copy_n=64, init="uniform_rest", seed=4),
    # D2Q9 periodic 8192^2 ELBM + positivity + Ehrenfest on 0.1 %, FP16 shifted.
    "elbm_8192": dict(
        lattice="D2Q9", nx=8192, ny=8192, bc="periodic", u_lid=0.0,
        collision="elbm", equilibrium="entropic", nu=1e-6,
        ehrenfest=True, ehr_k=math.ceil(0.001 * 8192 * 8192), ehr_delta=0.0,
        median=False, med_delta=1e-3, positivity=True,
        elbm_fallback="positivity",
        steps=5000, storages=("f16s",), checkpoint_every=256,
        init="spectral_velocity", seed=5, target_seed=4),
    # D3Q27 periodic 256^3 Taylor-Green vortex, LBGK + the 27-site median
    # entropy filter (delta 1e-3, the paper's value in its cavity study).
    "median3d_256": dict(
        lattice="D3Q27", nx=256, ny=256, nz=256, bc="periodic", u_lid=0.0,
        collision="lbgk", equilibrium="poly", nu=1e-5,
        ehrenfest=False, ehr_k=0, ehr_delta=0.0,
        median=True, med_delta=1e-3, positivity=False,
        steps=1000, storages=("f32",), init="taylor_green_3d", u0=0.05, seed=6),
    # D2Q9 periodic 4096^2 double shear layer, LBGK with the general nonlocal
    # filter: the binomial 3 x 3 smoothing (1 2 1; 2 4 2; 1 2 1) / 16 of the
    # nonequilibrium part, whose coefficients sum to 1.
    "nonlocal_4096": dict(
        lattice="D2Q9", nx=4096, ny=4096, bc="periodic", u_lid=0.0,
        collision="lbgk", equilibrium="poly", nu=1e-5,
        ehrenfest=False, ehr_k=0, ehr_delta=0.0,
        median=False, med_delta=1e-3, positivity=False,
        nl_coef=(1 / 16, 2 / 16, 1 / 16, 2 / 16, 4 / 16, 2 / 16, 1 / 16, 2 / 16, 1 / 16),
        steps=20000, storages=("f32",), init="double_shear_layer", seed=3),
}


def workload(name: str, **overrides) -> dict:
    """A copy of a workload's parameters with optional overrides."""
    w = dict(WORKLOADS[name])
    w.update(overrides)
    return w
