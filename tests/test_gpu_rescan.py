"""Ehrenfest selection on steps that rescan the lattice (section 4: the k
sites of largest Delta S, every step).

The candidate floor of a step comes from the previous step of the same
parity.  With omega = 1 one collision takes a random state to equilibrium,
so Delta S collapses between the first steps; fewer than k sites then reach
the floor carried over, and the step falls back to a rescan of the whole
lattice.  Every step's selected set and populations must equal the oracle's
step from the same input, and the run must have rescanned."""
import pytest
import torch

import oracle as O
from tests.parity_util import lattice, make_sim, near_tie_ok, oracle_config, random_state, rel_err

pytestmark = pytest.mark.gpu

P = dict(lattice="D2Q9", nx=96, ny=80, bc="periodic", collision="lbgk", nu=1.0 / 6.0,
         ehrenfest=True, ehr_k=40, ehr_delta=0.0)


@pytest.mark.parametrize("storage,rtol,ftol", [("f64", 1e-9, 1e-12), ("f32", 1e-5, 1e-5)])
def test_rescan_steps_match_oracle(storage, rtol, ftol):
    f0 = random_state(P, 131, amp=0.05)
    sim = make_sim(P, storage)
    sim.set_populations(f0.to("cuda"))
    fb0 = int(sim.stats().select_fallbacks)
    for t in range(8):
        f_in = sim.populations().cpu()
        sim.step(1)
        f_gpu = sim.populations().cpu()
        sel = sorted(sim.selected())
        with torch.no_grad():
            f_ora, info = O.step(lattice(P), oracle_config(P), f_in)
        sel_ora = sorted(info["selected"].tolist())
        assert len(sel) == P["ehr_k"], f"step {t}: {len(sel)} sites selected"
        assert near_tie_ok(sel, sel_ora, info["dS"], P["ehr_k"], rtol), f"step {t}: selection"
        if sel == sel_ora:
            err = rel_err(f_gpu, f_ora)
            assert err <= ftol, f"step {t}: populations differ by {err:.3e}"
    rescans = int(sim.stats().select_fallbacks) - fb0
    print(f"{storage}: {rescans} rescans in 8 steps")
    assert rescans > 0, "the case must exercise the rescan"
