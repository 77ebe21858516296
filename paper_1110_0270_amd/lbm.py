"""Python binding of liblbm.so (argument marshalling only).

The functions here carry the names of the C ABI in include/lbm.h and pass
torch tensors to it as raw device pointers together with the current HIP
stream.  Every computation runs in the library's HIP kernels; if the
library is missing or cannot be loaded, importing a function fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_EWORKSPACE, LBM_EHIP = 0, -1, -2, -3
LBM_EDIVERGED, LBM_ESTATE, LBM_EUNSUPPORTED, LBM_ESELECT = -4, -5, -6, -7
LBM_D1Q3, LBM_D2Q9, LBM_D3Q27 = 1, 2, 3
LBM_BC_PERIODIC, LBM_BC_BOUNCEBACK, LBM_BC_CAVITY, LBM_BC_COUETTE, LBM_BC_DIFFUSIVE = 0, 1, 2, 3, 4
LBM_LBGK, LBM_MRT, LBM_ELBM = 0, 1, 2
LBM_EQ_POLY, LBM_EQ_ENTROPIC = 0, 1
LBM_MRT_M1, LBM_MRT_M2 = 0, 1
LBM_LIM_EHRENFEST, LBM_LIM_POSITIVITY, LBM_LIM_MEDIAN = 1, 2, 4
LBM_NORM_ENTROPIC, LBM_NORM_L1 = 0, 1
LBM_FB_POSITIVITY, LBM_FB_EHRENFEST = 0, 1
LBM_F64, LBM_F32, LBM_F16S, LBM_BF16S = 0, 1, 2, 3
LBM_RATES_GIVEN, LBM_RATES_TRT, LBM_RATES_MRT_TRTQ, LBM_RATES_MRT1, LBM_RATES_SHEAR = 0, 1, 2, 3, 4
LBM_SEL_EQUILIBRIUM, LBM_SEL_MRT = 0, 1
LBM_ENS_NONE, LBM_ENS_THRESHOLD, LBM_ENS_SMOOTH, LBM_ENS_DOUBLE_MONOTONE, LBM_ENS_POINTWISE = 0, 1, 2, 3, 4

EXPORTED = [
    "lbm_config_default", "lbm_workspace_bytes", "lbm_init", "lbm_set_equilibrium",
    "lbm_set_equilibrium3d",
    "lbm_set_populations", "lbm_get_populations", "lbm_set_omega", "lbm_step",
    "lbm_moments", "lbm_backward", "lbm_stats_get", "lbm_selected", "lbm_counters",
    "lbm_profile_step", "lbm_profile_backward", "lbm_step_noalloc", "lbm_destroy",
    "lbm_last_error",
]
# size of the static device array behind lbm_step_noalloc (LBM_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


class lbm_config(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("bc", ctypes.c_int), ("u_lid", ctypes.c_double), ("rho_wall", ctypes.c_double),
        ("collision", ctypes.c_int), ("equilibrium", ctypes.c_int),
        ("nu", ctypes.c_double), ("omega", ctypes.c_double), ("mrt_basis", ctypes.c_int),
        ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
        ("limiters", ctypes.c_uint), ("ehr_k", ctypes.c_longlong),
        ("ehr_delta", ctypes.c_double), ("med_delta", ctypes.c_double),
        ("elbm_norm", ctypes.c_int), ("elbm_fallback", ctypes.c_int),
        ("elbm_eps", ctypes.c_double), ("elbm_max_iter", ctypes.c_int),
        ("elbm_dS_cut", ctypes.c_double), ("elbm_f64_below", ctypes.c_double),
        ("storage", ctypes.c_int), ("rho0", ctypes.c_double),
        ("omega_field", ctypes.c_int), ("checkpoint_every", ctypes.c_int),
        ("max_steps", ctypes.c_longlong), ("check_interval", ctypes.c_int),
        ("mrt_preset", ctypes.c_int), ("sel_action", ctypes.c_int),
        ("ens_limiter", ctypes.c_int), ("ens_delta0", ctypes.c_double),
        ("ens_delta", ctypes.c_double), ("ens_alpha", ctypes.c_double),
        ("ens_k", ctypes.c_double), ("nz", ctypes.c_int), ("nl_filter", ctypes.c_int),
        ("nl_coef", ctypes.c_double * 27),
    ]


class lbm_stats(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
        ("entropy", ctypes.c_double), ("min_rho", ctypes.c_double),
        ("steps", ctypes.c_longlong), ("diverged_step", ctypes.c_longlong),
        ("n_selected", ctypes.c_longlong), ("select_fallbacks", ctypes.c_longlong),
        ("select_overflow", ctypes.c_longlong), ("select_candidates", ctypes.c_longlong),
        ("nonfinite", ctypes.c_int), ("ens_threshold", ctypes.c_double),
        ("ens_mean", ctypes.c_double), ("lbgk_production", ctypes.c_double),
        ("limiter_production", ctypes.c_double), ("enstrophy", ctypes.c_double),
        ("mom_z", ctypes.c_double),
    ]


_lib = None


def library() -> ctypes.CDLL:
    """Load liblbm.so once; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1110_0270_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, LL, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_size_t
    cfgp = ctypes.POINTER(lbm_config)
    sig = {
        "lbm_config_default": (None, [cfgp]),
        "lbm_workspace_bytes": (SZ, [cfgp]),
        "lbm_init": (I, [cfgp, P, SZ, P, ctypes.POINTER(P)]),
        "lbm_set_equilibrium": (I, [P, P, P, P, I]),
        "lbm_set_equilibrium3d": (I, [P, P, P, P, P, I]),
        "lbm_set_populations": (I, [P, P, I]),
        "lbm_get_populations": (I, [P, P, I]),
        "lbm_set_omega": (I, [P, P, I]),
        "lbm_step": (I, [P, LL]),
        "lbm_moments": (I, [P, P, P, P, I]),
        "lbm_backward": (I, [P, P, P, P, I]),
        "lbm_stats_get": (I, [P, ctypes.POINTER(lbm_stats)]),
        "lbm_selected": (I, [P, ctypes.POINTER(LL), LL, ctypes.POINTER(LL)]),
        "lbm_counters": (I, [P, ctypes.POINTER(ctypes.c_ulonglong), I]),
        "lbm_profile_step": (I, [P, LL, ctypes.POINTER(ctypes.c_double)]),
        "lbm_profile_backward": (I, [P, P, P, P, I, ctypes.POINTER(ctypes.c_double)]),
        "lbm_step_noalloc": (I, [cfgp, P, P, P]),
        "lbm_destroy": (None, [P]),
        "lbm_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LBMError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = library().lbm_last_error().decode()
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def _check(status: int, where: str):
    if status != LBM_OK:
        raise LBMError(status, where)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return LBM_F64
    if t.dtype == torch.float32:
        return LBM_F32
    raise ValueError("caller buffers must be float64 or float32")


def _stream_handle() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def lbm_config_default() -> lbm_config:
    c = lbm_config()
    library().lbm_config_default(ctypes.byref(c))
    return c


def lbm_workspace_bytes(cfg: lbm_config) -> int:
    n = library().lbm_workspace_bytes(ctypes.byref(cfg))
    if n == 0:
        raise LBMError(LBM_EINVAL, "lbm_workspace_bytes")
    return int(n)


def lbm_init(cfg: lbm_config, workspace: torch.Tensor):
    ctx = ctypes.c_void_p()
    _check(library().lbm_init(ctypes.byref(cfg), _ptr(workspace), workspace.numel(),
                              _stream_handle(), ctypes.byref(ctx)), "lbm_init")
    return ctx


def lbm_set_equilibrium(ctx, rho, ux, uy=None):
    _check(library().lbm_set_equilibrium(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _dtype_code(rho)),
           "lbm_set_equilibrium")


def lbm_set_equilibrium3d(ctx, rho, ux, uy, uz):
    _check(library().lbm_set_equilibrium3d(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(uz),
                                           _dtype_code(rho)), "lbm_set_equilibrium3d")


def lbm_set_populations(ctx, f):
    _check(library().lbm_set_populations(ctx, _ptr(f), _dtype_code(f)), "lbm_set_populations")


def lbm_get_populations(ctx, f):
    _check(library().lbm_get_populations(ctx, _ptr(f), _dtype_code(f)), "lbm_get_populations")


def lbm_set_omega(ctx, omega):
    _check(library().lbm_set_omega(ctx, _ptr(omega), _dtype_code(omega)), "lbm_set_omega")


def lbm_step(ctx, n: int):
    _check(library().lbm_step(ctx, int(n)), "lbm_step")


def lbm_moments(ctx, rho, ux, uy=None):
    _check(library().lbm_moments(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _dtype_code(rho)),
           "lbm_moments")


def lbm_backward(ctx, dL_dfT, dL_df0, dL_domega=None):
    _check(library().lbm_backward(ctx, _ptr(dL_dfT), _ptr(dL_df0), _ptr(dL_domega),
                                  _dtype_code(dL_dfT)), "lbm_backward")


def lbm_stats_get(ctx, allow_status=(LBM_OK,)) -> lbm_stats:
    st = lbm_stats()
    s = library().lbm_stats_get(ctx, ctypes.byref(st))
    if s not in allow_status:
        raise LBMError(s, "lbm_stats_get")
    return st


def lbm_selected(ctx, cap: int):
    arr = (ctypes.c_longlong * max(1, cap))()
    cnt = ctypes.c_longlong()
    _check(library().lbm_selected(ctx, arr, cap, ctypes.byref(cnt)), "lbm_selected")
    return [arr[i] for i in range(min(cnt.value, cap))], cnt.value


def lbm_counters(ctx, n: int = 8):
    arr = (ctypes.c_ulonglong * n)()
    _check(library().lbm_counters(ctx, arr, n), "lbm_counters")
    return list(arr)


def lbm_profile_step(ctx, n: int):
    """(ms in the fused step kernels, ms for the n steps) via HIP events."""
    out = (ctypes.c_double * 2)()
    _check(library().lbm_profile_step(ctx, int(n), out), "lbm_profile_step")
    return out[0], out[1]


def lbm_profile_backward(ctx, dL_dfT, dL_df0, dL_domega=None):
    """(summed adjoint-kernel ms, whole backward ms)."""
    out = (ctypes.c_double * 2)()
    _check(library().lbm_profile_backward(ctx, _ptr(dL_dfT), _ptr(dL_df0), _ptr(dL_domega),
                                          _dtype_code(dL_dfT), out), "lbm_profile_backward")
    return out[0], out[1]


def lbm_step_noalloc(cfg: lbm_config, f_src, f_dst):
    """One step from f_src into f_dst (device tensors in the storage form of
    cfg.storage, [Q][ny][nx]) without any allocation, on the current stream."""
    _check(library().lbm_step_noalloc(ctypes.byref(cfg), _ptr(f_src), _ptr(f_dst),
                                      _stream_handle()), "lbm_step_noalloc")


def lbm_destroy(ctx):
    library().lbm_destroy(ctx)


# ---------------------------------------------------------------------------
# Convenience layer: configuration from a workload description, and an object
# that owns the workspace tensor and the context.
# ---------------------------------------------------------------------------
_BC = {"periodic": LBM_BC_PERIODIC, "bounceback": LBM_BC_BOUNCEBACK, "cavity": LBM_BC_CAVITY,
       "couette": LBM_BC_COUETTE, "diffusive": LBM_BC_DIFFUSIVE}
_COLL = {"lbgk": LBM_LBGK, "mrt": LBM_MRT, "elbm": LBM_ELBM}
_STORE = {"f64": LBM_F64, "f32": LBM_F32, "f16s": LBM_F16S, "bf16s": LBM_BF16S}
_PRESET = {"given": LBM_RATES_GIVEN, "trt": LBM_RATES_TRT, "mrt_trtq": LBM_RATES_MRT_TRTQ,
           "mrt1": LBM_RATES_MRT1, "shear": LBM_RATES_SHEAR}
_SEL = {"equilibrium": LBM_SEL_EQUILIBRIUM, "mrt": LBM_SEL_MRT}
_ENS = {"none": LBM_ENS_NONE, "threshold": LBM_ENS_THRESHOLD, "smooth": LBM_ENS_SMOOTH,
        "double_monotone": LBM_ENS_DOUBLE_MONOTONE, "pointwise": LBM_ENS_POINTWISE}


def make_config(*, lattice="D2Q9", nx=64, ny=64, bc="periodic", u_lid=0.0, rho_wall=1.0,
                collision="lbgk", equilibrium="poly", nu=None, omega=None, mrt_basis="M1",
                s_e=1.64, s_eps=1.54, s_q=1.9, ehrenfest=False, ehr_k=0, ehr_delta=0.0,
                median=False, med_delta=1e-3, positivity=False, elbm_norm="entropic",
                elbm_fallback="positivity", elbm_eps=1e-14, elbm_max_iter=32,
                elbm_dS_cut=1e-15, elbm_f64_below=3.0, storage="f32", rho0=1.0,
                omega_field=False, checkpoint_every=0, max_steps=0, check_interval=0,
                mrt_preset="given", sel_action="equilibrium", ens_limiter="none",
                ens_delta0=0.1, ens_delta=0.0, ens_alpha=1.0, ens_k=1.0, nz=1, nl_coef=None,
                **_ignored) -> lbm_config:
    c = lbm_config_default()
    c.lattice = {"D1Q3": LBM_D1Q3, "D2Q9": LBM_D2Q9, "D3Q27": LBM_D3Q27}[lattice]
    c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
    if nl_coef is not None:
        c.nl_filter = 1
        for k, v in enumerate(nl_coef):
            c.nl_coef[k] = float(v)
    c.bc = _BC[bc]
    c.u_lid, c.rho_wall = float(u_lid), float(rho_wall)
    c.collision = _COLL[collision]
    c.equilibrium = LBM_EQ_ENTROPIC if equilibrium == "entropic" else LBM_EQ_POLY
    if nu is not None:
        c.nu = float(nu)
    else:
        c.nu, c.omega = -1.0, float(omega if omega is not None else 1.0)
    c.mrt_basis = LBM_MRT_M2 if mrt_basis == "M2" else LBM_MRT_M1
    c.s_e, c.s_eps, c.s_q = float(s_e), float(s_eps), float(s_q)
    c.limiters = ((LBM_LIM_EHRENFEST if ehrenfest else 0) | (LBM_LIM_POSITIVITY if positivity else 0)
                  | (LBM_LIM_MEDIAN if median else 0))
    c.ehr_k, c.ehr_delta, c.med_delta = int(ehr_k), float(ehr_delta), float(med_delta)
    c.elbm_norm = LBM_NORM_L1 if elbm_norm == "l1" else LBM_NORM_ENTROPIC
    c.elbm_fallback = LBM_FB_EHRENFEST if elbm_fallback == "ehrenfest" else LBM_FB_POSITIVITY
    c.elbm_eps, c.elbm_max_iter = float(elbm_eps), int(elbm_max_iter)
    c.elbm_dS_cut, c.elbm_f64_below = float(elbm_dS_cut), float(elbm_f64_below)
    c.storage = _STORE[storage]
    c.rho0 = float(rho0)
    c.omega_field = 1 if omega_field else 0
    c.checkpoint_every, c.max_steps = int(checkpoint_every), int(max_steps)
    c.check_interval = int(check_interval)
    c.mrt_preset = _PRESET[mrt_preset]
    c.sel_action = _SEL[sel_action]
    c.ens_limiter = _ENS[ens_limiter]
    c.ens_delta0, c.ens_delta = float(ens_delta0), float(ens_delta)
    c.ens_alpha, c.ens_k = float(ens_alpha), float(ens_k)
    return c


class Simulation:
    """Owns a workspace tensor and a context on the current device/stream."""

    def __init__(self, cfg: lbm_config, device="cuda"):
        self.cfg = cfg
        self.Q = {LBM_D1Q3: 3, LBM_D2Q9: 9, LBM_D3Q27: 27}[cfg.lattice]
        self.shape = ((27, cfg.nz, cfg.ny, cfg.nx) if cfg.lattice == LBM_D3Q27
                      else (self.Q, cfg.ny, cfg.nx))
        nbytes = lbm_workspace_bytes(cfg)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.ctx = lbm_init(cfg, self._ws)
        # Identity of the rollout the context records: the generation changes
        # with every call that resets the lattice or the relaxation field,
        # and the step count grows with every step.  LBMRollout checks both
        # before it runs the adjoint.
        self.generation = 0
        self.steps_taken = 0

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and _lib is not None:
            lbm_destroy(ctx)
            self.ctx = None

    def set_equilibrium(self, rho, ux, uy=None):
        lbm_set_equilibrium(self.ctx, rho, ux, uy)
        self.generation += 1
        self.steps_taken = 0

    def set_equilibrium3d(self, rho, ux, uy, uz):
        lbm_set_equilibrium3d(self.ctx, rho, ux, uy, uz)
        self.generation += 1
        self.steps_taken = 0

    def set_populations(self, f):
        lbm_set_populations(self.ctx, f)
        self.generation += 1
        self.steps_taken = 0

    def populations(self, dtype=torch.float64):
        f = torch.empty(self.shape, dtype=dtype, device=self.workspace.device)
        lbm_get_populations(self.ctx, f)
        return f

    def set_omega(self, omega):
        lbm_set_omega(self.ctx, omega)
        self.generation += 1

    def step(self, n: int = 1):
        lbm_step(self.ctx, n)
        self.steps_taken += int(n)

    def moments(self, dtype=torch.float64):
        dev = self.workspace.device
        shp = (self.cfg.ny, self.cfg.nx)
        rho = torch.empty(shp, dtype=dtype, device=dev)
        ux = torch.empty(shp, dtype=dtype, device=dev)
        uy = torch.empty(shp, dtype=dtype, device=dev)
        lbm_moments(self.ctx, rho, ux, uy)
        return rho, ux, uy

    def stats(self, allow_status=(LBM_OK,)) -> lbm_stats:
        return lbm_stats_get(self.ctx, allow_status)

    def selected(self):
        idx, n = lbm_selected(self.ctx, int(max(1, self.cfg.ehr_k)))
        return idx

    def counters(self):
        return lbm_counters(self.ctx)

    def profile_step(self, n: int):
        out = lbm_profile_step(self.ctx, n)
        self.steps_taken += int(n)
        return out

    def backward(self, dL_dfT, dL_df0, dL_domega=None):
        lbm_backward(self.ctx, dL_dfT, dL_df0, dL_domega)

    def profile_backward(self, dL_dfT, dL_df0, dL_domega=None):
        return lbm_profile_backward(self.ctx, dL_dfT, dL_df0, dL_domega)


class LBMRollout(torch.autograd.Function):
    """f_T = n steps of the library from f0 (and a per-site omega field);
    backward runs the library's adjoint (lbm_backward)."""

    @staticmethod
    def forward(ctx, f0, omega, sim: Simulation, n: int):
        sim.set_populations(f0.contiguous())
        if omega is not None:
            sim.set_omega(omega.contiguous())
        sim.step(n)
        ctx.sim = sim
        ctx.rollout = (sim.generation, sim.steps_taken)
        ctx.has_omega = omega is not None
        ctx.dtype = f0.dtype
        return sim.populations(f0.dtype)

    @staticmethod
    def backward(ctx, grad_fT):
        sim = ctx.sim
        if (sim.generation, sim.steps_taken) != ctx.rollout:
            raise RuntimeError("LBMRollout.backward: the Simulation was reset, given a new "
                               "relaxation field or stepped after this rollout's forward "
                               "pass, so the rollout it recorded is gone")
        g0 = torch.empty(sim.shape, dtype=ctx.dtype, device=grad_fT.device)
        gw = (torch.zeros((sim.cfg.ny, sim.cfg.nx), dtype=ctx.dtype, device=grad_fT.device)
              if ctx.has_omega else None)
        sim.backward(grad_fT.contiguous().to(ctx.dtype), g0, gw)
        return g0, gw, None, None
