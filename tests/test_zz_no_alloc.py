"""lbm_step_noalloc (one step, no allocation, scratch in a static device
array) against lbm_step through a context with its own workspace: the same
kernels, so the same bits.  Two calls in a row on one device, the second on
a smaller lattice (the array keeps the first call's contents, which the
second must not see), in FP64 and in shifted FP32 storage, with the
Ehrenfest and positivity limiters; and ELBM in FP32 (its FP64-solve list
lives in the array too)."""
import numpy as np
import pytest
import torch

from tests.parity_util import make_sim, random_state

pytestmark = pytest.mark.gpu

W1 = (1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0)


def _weights(Q):
    if Q == 3:
        return torch.tensor(W1, dtype=torch.float64)
    return torch.tensor([W1[i % 3] * W1[i // 3] for i in range(9)], dtype=torch.float64)


def _storage_form(f, storage):
    """The lattice as the library stores it: f (FP64) or f - w rho0 rounded
    to FP32 (rho0 = 1)."""
    if storage == "f64":
        return f.clone()
    w = _weights(f.shape[0]).view(-1, 1, 1)
    return (f - w * 1.0).float()


def _unshift(g, storage):
    if storage == "f64":
        return g
    w = _weights(g.shape[0]).view(-1, 1, 1)
    return g.double() + w * 1.0


def _one_case(p, storage, seed, amp):
    from paper_1110_0270_amd import lbm as B
    kind = "entropic" if p.get("collision") == "elbm" else "poly"
    f0 = random_state(p, seed, amp=amp, kind=kind)
    # the existing entry point: a context with its own workspace
    sim = make_sim(p, storage)
    sim.set_populations(f0.to("cuda"))
    sim.step(1)
    ref = sim.populations().cpu()
    del sim
    # the allocation-free one
    cfg = B.make_config(**{**p, "storage": storage})
    src = _storage_form(f0, storage).to("cuda").contiguous()
    dst = torch.full_like(src, float("nan"))
    B.lbm_step_noalloc(cfg, src, dst)
    torch.cuda.synchronize()
    out = _unshift(dst.cpu(), storage)
    assert torch.equal(out, ref), f"max |diff| {float((out - ref).abs().max()):.3e}"


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_matches_lbm_step_two_calls(storage):
    big = dict(lattice="D2Q9", nx=300, ny=41, bc="cavity", u_lid=0.1, nu=1e-3,
               ehrenfest=True, ehr_k=60, ehr_delta=0.0, positivity=True)
    small = dict(lattice="D2Q9", nx=70, ny=37, bc="periodic", nu=1e-3,
                 ehrenfest=True, ehr_k=9, ehr_delta=0.0, positivity=True)
    _one_case(big, storage, 5, 0.4)
    _one_case(small, storage, 6, 0.4)


def test_noalloc_elbm_fp32_two_calls():
    big = dict(lattice="D2Q9", nx=300, ny=13, bc="periodic", nu=1e-4, collision="elbm",
               positivity=True)
    small = dict(lattice="D2Q9", nx=70, ny=37, bc="periodic", nu=1e-4, collision="elbm",
                 positivity=True)
    _one_case(big, "f32", 7, 0.6)
    _one_case(small, "f32", 8, 0.6)


def test_noalloc_rejects_oversized_config():
    from paper_1110_0270_amd import lbm as B
    cfg = B.make_config(nx=4096, ny=4096, storage="f32", nu=1e-5, ehrenfest=True, ehr_k=16778)
    x = torch.zeros(8, device="cuda")
    y = torch.zeros(8, device="cuda")
    with pytest.raises(B.LBMError) as e:
        B.lbm_step_noalloc(cfg, x, y)
    assert e.value.status == B.LBM_EWORKSPACE
