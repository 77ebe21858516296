"""Replays of the captured step graph against eager stepping.

A run of at least 16 steps without periodic checks replays a HIP graph of
16 captured steps (while a rollout is recorded, only groups that do not
span a checkpoint); single steps run eagerly.
Two simulations start from the same state: one takes step(1) calls, the
other step(n) calls that replay the graph.  After every call, with eager
work (population and counter reads, torch arithmetic, synchronisation)
between the replays, the populations, the Ehrenfest set and the limiter
counters must agree bit for bit."""
import numpy as np
import pytest
import torch

from tests.parity_util import make_sim, random_state

pytestmark = pytest.mark.gpu

CASES = {
    "cavity_f32_lbgk_ehr_pos": dict(nx=96, ny=80, bc="cavity", u_lid=0.1, collision="lbgk",
                                    nu=0.002, ehrenfest=True, ehr_k=40, ehr_delta=1e-6,
                                    positivity=True),
    "periodic_f16s_elbm_ehr": dict(nx=256, ny=40, bc="periodic", collision="elbm", nu=1e-4,
                                   ehrenfest=True, ehr_k=30, ehr_delta=1e-7, positivity=True),
    "periodic_f64_mrt_median": dict(nx=70, ny=33, bc="periodic", collision="mrt", nu=0.001,
                                    median=True, med_delta=1e-4, positivity=True),
    "d1q3_bf16s_lbgk_ehr": dict(lattice="D1Q3", nx=1000, ny=1, bc="periodic", collision="lbgk",
                                nu=0.01, ehrenfest=True, ehr_k=8, ehr_delta=1e-6),
}
STORAGE = {"cavity_f32_lbgk_ehr_pos": "f32", "periodic_f16s_elbm_ehr": "f16s",
           "periodic_f64_mrt_median": "f64", "d1q3_bf16s_lbgk_ehr": "bf16s"}
# step(n) calls of the replaying simulation: graphs of 16 plus eager remainders
CALLS = [16, 32, 5, 16, 47, 16]


@pytest.mark.parametrize("name", sorted(CASES))
def test_graph_replays_match_eager(name):
    p = CASES[name]
    storage = STORAGE[name]
    f0 = random_state(p, seed=97, amp=0.04, umax=0.06)
    eager = make_sim(p, storage)
    graph = make_sim(p, storage)
    for s in (eager, graph):
        s.set_populations(f0.to("cuda"))
    scratch = torch.zeros(1 << 16, device="cuda")
    for i, n in enumerate(CALLS):
        for _ in range(n):
            eager.step(1)
        graph.step(n)
        # eager work between replays
        scratch.add_(float(i + 1)).mul_(0.5)
        torch.cuda.synchronize()
        fe, fg = eager.populations(), graph.populations()
        assert torch.equal(fe, fg), f"call {i} (step({n})): populations differ"
        if p.get("ehrenfest"):
            assert sorted(eager.selected()) == sorted(graph.selected()), f"call {i}: selection"
        assert eager.counters() == graph.counters(), f"call {i}: counters"
    assert torch.isfinite(graph.populations()).all()
    # a fresh state set between replays restarts from the new lattice contents
    f1 = random_state(p, seed=98, amp=0.04, umax=0.06)
    for s in (eager, graph):
        s.set_populations(f1.to("cuda"))
    for _ in range(32):
        eager.step(1)
    graph.step(32)
    torch.cuda.synchronize()
    assert torch.equal(eager.populations(), graph.populations())


REC_CASES = {
    "cavity_f32_mrt_ehr_pos": (dict(nx=96, ny=80, bc="cavity", u_lid=0.1, collision="mrt", nu=0.002,
                                    s_e=1.64, s_eps=1.64, s_q=1.9, ehrenfest=True, ehr_k=9,
                                    ehr_delta=1e-6, positivity=True), "f32"),
    "periodic_f64_lbgk_ehr": (dict(nx=300, ny=13, bc="periodic", collision="lbgk", nu=1e-4,
                                   ehrenfest=True, ehr_k=20, ehr_delta=0.0), "f64"),
}


@pytest.mark.parametrize("name", sorted(REC_CASES))
def test_recorded_rollout_graphs_match_eager(name):
    """A recorded rollout (checkpoints every 32 steps, 87 steps: graph groups
    between checkpoints, eager steps across them and at the end) against the
    same rollout taken one step at a time: final state, last selection and
    the backward pass's gradients bit for bit."""
    p0, storage = REC_CASES[name]
    p = {**p0, "checkpoint_every": 32, "max_steps": 96}
    f0 = random_state(p, 71, amp=0.04, umax=0.06)
    w = torch.tensor(np.random.default_rng(72).normal(size=f0.shape), dtype=torch.float64)
    out = []
    for mode in ("graph", "eager"):
        sim = make_sim(p, storage)
        sim.set_populations(f0.to("cuda"))
        if mode == "graph":
            sim.step(40)
            torch.cuda.synchronize()
            sim.step(47)
        else:
            for _ in range(87):
                sim.step(1)
        fT = sim.populations().cpu()
        sel = sorted(sim.selected())
        g0 = torch.empty(sim.shape, dtype=torch.float64, device="cuda")
        sim.backward(w.to("cuda"), g0, None)
        torch.cuda.synchronize()
        out.append((fT, sel, g0.cpu()))
        del sim
    assert torch.equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][2], out[1][2])


@pytest.mark.parametrize("ci", [48, 40])
def test_periodic_checks_with_graphs(ci):
    """Periodic divergence checks every ci steps between graph groups (40 is
    not a multiple of 16: the steps around each check run eagerly): state
    and the checks' statistics equal to eager stepping."""
    p = dict(nx=96, ny=80, bc="cavity", u_lid=0.1, collision="lbgk", nu=0.002,
             positivity=True, check_interval=ci)
    f0 = random_state(p, 81, amp=0.04, umax=0.06)
    res = []
    for mode in ("graph", "eager"):
        sim = make_sim(p, "f32")
        sim.set_populations(f0.to("cuda"))
        if mode == "graph":
            sim.step(150)
            sim.step(53)
        else:
            for _ in range(203):
                sim.step(1)
        st = sim.stats()
        res.append((sim.populations().cpu(), st.mass, st.entropy, int(st.diverged_step)))
        del sim
    assert torch.equal(res[0][0], res[1][0])
    assert res[0][1:] == res[1][1:]
