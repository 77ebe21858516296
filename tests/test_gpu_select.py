"""Ehrenfest selection with exact ties in Delta S (section 4: the k sites of
largest Delta S; ties go to the lower site index).

The lattice holds two horizontal bands of identical states, the upper one
further from equilibrium.  Away from the band edges every site of a band
pulls the same populations, so whole rows share one Delta S bit for bit, in
the oracle and in the kernels alike.  k falls inside the upper band's tie
group, so the boundary bucket of the selection holds the whole group and
the site indices decide the set: groups larger than the selection's LDS
staging (2048 entries; with and without room for the 16-byte records of
the exact resolution's global scratch), within it, and short enough (at
most 256) to be ranked directly.  The selected set must equal the oracle's exactly."""
import numpy as np
import pytest
import torch

import oracle as O
from tests.parity_util import lattice, make_sim, oracle_config

pytestmark = pytest.mark.gpu

AMP = [0.03, -0.02, 0.01, 0.02, -0.01, 0.015, -0.03, 0.02, 0.01]


def _band_state(nx, ny, hi_rows=None):
    lat = O.Lattice("D2Q9")
    rho = np.ones((ny, nx))
    ux = np.full((ny, nx), 0.02)
    uy = np.full((ny, nx), -0.01)
    f = O.init_equilibrium(lat, rho, ux, uy)
    amp = torch.tensor(AMP, dtype=torch.float64).view(9, 1, 1)
    scale = torch.ones(1, ny, 1, dtype=torch.float64)
    scale[:, (ny // 2 if hi_rows is None else hi_rows):, :] = 0.5
    return f * (1.0 + amp * scale)


@pytest.mark.parametrize("nx,ny,k,hi", [(256, 64, 4000, None), (256, 128, 3000, 16),
                                        (32, 64, 500, None), (32, 64, 960, None),
                                        (16, 64, 200, None), (8, 64, 100, None),
                                        (8, 64, 240, None)],
                         ids=["group_7680_k4000", "group_3584_k3000_records", "group_960_k500",
                              "group_960_k960", "group_480_k200", "group_240_k100",
                              "group_240_k240"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_selection_exact_ties(nx, ny, k, hi, storage):
    p = dict(lattice="D2Q9", nx=nx, ny=ny, bc="periodic", collision="lbgk", nu=1e-4,
             ehrenfest=True, ehr_k=k, ehr_delta=0.0)
    f0 = _band_state(nx, ny, hi)
    sim = make_sim(p, storage)
    sim.set_populations(f0.to("cuda"))
    f_in = sim.populations().cpu()
    sim.step(1)
    sel_gpu = sim.selected()
    torch.cuda.synchronize()
    with torch.no_grad():
        _, info = O.step(lattice(p), oracle_config(p), f_in)
    dS = info["dS"].flatten()
    sel_ora = info["selected"].tolist()
    # the tie group really is one value and k falls inside it
    kth = float(torch.sort(dS, descending=True).values[k - 1])
    group = int((dS == kth).sum())
    assert group >= 240
    assert sorted(sel_gpu) == sorted(sel_ora)
