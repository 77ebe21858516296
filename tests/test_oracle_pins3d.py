"""Pins of the D3Q27 oracle (27-site median entropy filter) and of the
general nonlocal f_neq filter (section 4, "Median entropy filter" and
"General nonlocal filters") against what the paper and the mathematics fix:

- the D3Q27 lattice: normalisation, isotropy up to fourth order;
- the product equilibria: density, momentum and the second moments in
  closed form (sum_a a^2 phi_a = 1/3 + u^2, resp. (2 sqrt(1 + 3u^2) - 1)/3);
- free flight moves each population by its velocity;
- the median of 27 is the 14th smallest (brute force over Python lists);
- the nonlocal filter: brute force, moments kept, identity and uniform
  fields in closed form;
- a D3Q27 state that is a product w_c g_ab along one axis steps exactly as
  the (already pinned) D2Q9 step of g in the other two, for all three axes
  (this fixes the handling of every axis and every population index);
- conservation of mass and momentum, the uniform equilibrium as a fixed
  point, and invariance of the step under permutations of the axes."""
import itertools
import math

import numpy as np
import pytest
import torch

import oracle as O
from lbm_inputs import generators as G

W1 = (1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0)


def test_d3q27_lattice_isotropy():
    lat = O.Lattice3()
    w, v = lat.w, torch.stack([lat.vx, lat.vy, lat.vz])
    assert abs(float(w.sum()) - 1.0) < 1e-15
    assert len(set(lat.vel)) == 27
    for i, (a, b, c) in enumerate(lat.vel):
        assert lat.vel[lat.opp[i]] == (-a, -b, -c) and lat.opp[i] == 26 - i
    for al in range(3):
        assert abs(float((w * v[al]).sum())) < 1e-16
        for be in range(3):
            assert abs(float((w * v[al] * v[be]).sum()) - (1 / 3 if al == be else 0)) < 1e-15
        # fourth order: sum w v_a^4 = 3 c_s^4 = 1/3, sum w v_a^2 v_b^2 = c_s^4 = 1/9
        assert abs(float((w * v[al] ** 4).sum()) - 1 / 3) < 1e-15
    assert abs(float((w * v[0] ** 2 * v[1] ** 2).sum()) - 1 / 9) < 1e-15


@pytest.mark.parametrize("kind", ["poly", "entropic"])
def test_equilibrium3_moments_closed_form(kind):
    rng = np.random.default_rng(3)
    shape = (3, 4, 5)
    rho = torch.tensor(1 + 0.2 * rng.uniform(-1, 1, shape))
    u = [torch.tensor(0.15 * rng.uniform(-1, 1, shape)) for _ in range(3)]
    f = O.equilibrium3(rho, *u, kind)
    lat = O.Lattice3()
    r, jx, jy, jz = O.moments3(f)
    assert float((r - rho).abs().max()) < 1e-14
    for j, uu in zip((jx, jy, jz), u):
        assert float((j - rho * uu).abs().max()) < 1e-14
    for vel, uu in zip((lat.vx, lat.vy, lat.vz), u):
        p = (lat.col(vel) ** 2 * f).sum(0)
        if kind == "poly":
            want = rho * (1 / 3 + uu * uu)
        else:
            want = rho * (2 * torch.sqrt(1 + 3 * uu * uu) - 1) / 3
        assert float((p - want).abs().max()) < 1e-14


def test_stream3_moves_each_population_by_its_velocity():
    nz, ny, nx = 4, 5, 6
    g = torch.zeros(27, nz, ny, nx, dtype=torch.float64)
    src = (1, 2, 3)
    g[:, src[0], src[1], src[2]] = torch.arange(1, 28, dtype=torch.float64)
    out = O.stream3(g)
    for i, (a, b, c) in enumerate(O.Lattice3().vel):
        dst = ((src[0] + c) % nz, (src[1] + b) % ny, (src[2] + a) % nx)
        assert float(out[i][dst]) == i + 1
        assert float(out[i].abs().sum()) == i + 1


def _median_brute(dS):
    nz, ny, nx = dS.shape
    med = torch.empty_like(dS)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        vals = sorted(float(dS[(z + dz) % nz, (y + dy) % ny, (x + dx) % nx])
                      for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))
        med[z, y, x] = vals[13]
    return med


def test_median3_brute_force():
    rng = np.random.default_rng(7)
    nz, ny, nx = 3, 4, 5
    # values drawn from a small set, so that ties occur
    dS = torch.tensor(rng.choice([0.0, 1e-4, 2e-4, 5e-4, 1e-3, 3e-3], size=(nz, ny, nx)))
    f = torch.tensor(rng.uniform(0.01, 0.1, (27, nz, ny, nx)))
    feq = torch.tensor(rng.uniform(0.01, 0.1, (27, nz, ny, nx)))
    delta = 1.5e-4
    out, mask = O.median_filter3(f, feq, dS, delta)
    med = _median_brute(dS)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        s, m = float(dS[z, y, x]), float(med[z, y, x])
        acc = s > delta and m < s
        assert bool(mask[z, y, x]) == acc
        c = math.sqrt(m / s) if acc else 1.0
        want = feq[:, z, y, x] + c * (f[:, z, y, x] - feq[:, z, y, x])
        assert float((out[:, z, y, x] - want).abs().max()) < 1e-16


def test_median3_of_27_picks_14th():
    # a single site whose neighbourhood holds 0..26 (a permutation)
    rng = np.random.default_rng(1)
    vals = torch.tensor(rng.permutation(27).astype(float)).view(3, 3, 3)
    med = O.median_filter3(torch.ones(27, 3, 3, 3, dtype=torch.float64) * 2,
                           torch.ones(27, 3, 3, 3, dtype=torch.float64), vals, -1.0)
    # every site of a 3^3 periodic lattice sees all 27 values
    centre = float(vals[1, 1, 1])
    acc = bool(med[1][1, 1, 1])
    assert acc == (13.0 < centre)
    if acc:
        assert abs(float(med[0][0, 1, 1, 1]) - (1 + math.sqrt(13.0 / centre))) < 1e-15


def _nl_brute_2d(lat, f, feq, coef):
    Q, ny, nx = f.shape
    out = feq.clone()
    offs = O.stencil_offsets(lat)
    for i, y, x in itertools.product(range(Q), range(ny), range(nx)):
        s = 0.0
        for c, (dy, dx) in zip(coef, offs):
            s += c * float(f[i, (y + dy) % ny, (x + dx) % nx] - feq[i, (y + dy) % ny, (x + dx) % nx])
        out[i, y, x] = feq[i, y, x] + s
    return out


def _nl_brute_3d(f, feq, coef):
    Q, nz, ny, nx = f.shape
    out = feq.clone()
    neq = f - feq
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        s = torch.zeros(Q, dtype=torch.float64)
        for c, (dz, dy, dx) in zip(coef, O.stencil_offsets3()):
            s += c * neq[:, (z + dz) % nz, (y + dy) % ny, (x + dx) % nx]
        out[:, z, y, x] = feq[:, z, y, x] + s
    return out


@pytest.mark.parametrize("name", ["D1Q3", "D2Q9"])
def test_nonlocal_filter_brute_force_and_moments(name):
    lat = O.Lattice(name)
    rng = np.random.default_rng(11)
    ny, nx = (1, 7) if name == "D1Q3" else (4, 5)
    rho = torch.tensor(1 + 0.1 * rng.uniform(-1, 1, (ny, nx)))
    ux = torch.tensor(0.1 * rng.uniform(-1, 1, (ny, nx)))
    uy = torch.tensor(0.1 * rng.uniform(-1, 1, (ny, nx))) if name == "D2Q9" else torch.zeros(ny, nx,
                                                                                             dtype=torch.float64)
    feq = O.equilibrium(lat, rho, ux, uy)
    f = feq * (1 + torch.tensor(rng.uniform(-0.2, 0.2, feq.shape)))
    r, jx, jy = O.moments(lat, f)
    feq = O.equilibrium(lat, r, jx / r, jy / r)          # f* of f itself
    coef = tuple(rng.uniform(-0.5, 1.0, 3 if name == "D1Q3" else 9))
    out = O.nonlocal_filter(lat, f, feq, coef)
    assert float((out - _nl_brute_2d(lat, f, feq, coef)).abs().max()) < 1e-15
    r2, jx2, jy2 = O.moments(lat, out)
    assert float((r2 - r).abs().max()) < 1e-14
    assert float((jx2 - jx).abs().max()) < 1e-14 and float((jy2 - jy).abs().max()) < 1e-14
    # the identity stencil keeps f; a uniform field scales f_neq by sum d
    ident = tuple(1.0 if o == (0, 0) else 0.0 for o in O.stencil_offsets(lat))
    assert float((O.nonlocal_filter(lat, f, feq, ident) - f).abs().max()) < 1e-16
    fu, fequ = f[:, :1, :1].expand_as(f), feq[:, :1, :1].expand_as(f)
    want = fequ + sum(coef) * (fu - fequ)
    assert float((O.nonlocal_filter(lat, fu, fequ, coef) - want).abs().max()) < 1e-15


def test_nonlocal_filter3_brute_force_and_moments():
    rng = np.random.default_rng(12)
    shape = (3, 4, 5)
    rho = torch.tensor(1 + 0.1 * rng.uniform(-1, 1, shape))
    u = [torch.tensor(0.1 * rng.uniform(-1, 1, shape)) for _ in range(3)]
    f = O.equilibrium3(rho, *u) * (1 + torch.tensor(rng.uniform(-0.2, 0.2, (27,) + shape)))
    r, jx, jy, jz = O.moments3(f)
    feq = O.equilibrium3(r, jx / r, jy / r, jz / r)
    coef = tuple(rng.uniform(-0.3, 0.6, 27))
    out = O.nonlocal_filter3(f, feq, coef)
    assert float((out - _nl_brute_3d(f, feq, coef)).abs().max()) < 1e-15
    for a, b in zip(O.moments3(out), (r, jx, jy, jz)):
        assert float((a - b).abs().max()) < 1e-14


# --- the D3Q27 step against the D2Q9 step on product states ---------------
def _i2(a, b):
    return 3 * (b + 1) + (a + 1)


def _lift(g2, axis, n):
    """The D3Q27 state w_(missing velocity) g2 that does not vary along
    `axis`; g2 is a D2Q9 state on the other two axes (its x the lower one)."""
    lat = O.Lattice3()
    _, p, q = g2.shape
    if axis == "z":
        out = torch.empty(27, n, p, q, dtype=torch.float64)
    elif axis == "y":
        out = torch.empty(27, p, n, q, dtype=torch.float64)
    else:
        out = torch.empty(27, p, q, n, dtype=torch.float64)
    for i, (a, b, c) in enumerate(lat.vel):
        if axis == "z":
            out[i] = (g2[_i2(a, b)] * W1[c + 1]).unsqueeze(0)
        elif axis == "y":
            out[i] = (g2[_i2(a, c)] * W1[b + 1]).unsqueeze(1)
        else:
            out[i] = (g2[_i2(b, c)] * W1[a + 1]).unsqueeze(2)
    return out


def _coef2(coef3, axis):
    d = torch.tensor(coef3).view(3, 3, 3)          # (dz, dy, dx)
    red = {"z": d.sum(0), "y": d.sum(1), "x": d.sum(2)}[axis]
    return tuple(float(v) for v in red.flatten())


OPTS = {
    "lbgk": dict(),
    "median": dict(median=True, med_delta=1e-5),
    "positivity": dict(positivity=True),
    "nonlocal": dict(nl=True),
    "all": dict(median=True, med_delta=0.0, positivity=True, nl=True),
}


@pytest.mark.parametrize("axis", ["z", "y", "x"])
@pytest.mark.parametrize("kind", ["poly", "entropic"])
@pytest.mark.parametrize("opt", list(OPTS))
def test_step3_reduces_to_d2q9_on_product_states(axis, kind, opt):
    rng = np.random.default_rng(21)
    p2, q2, n = 6, 5, 3
    lat2 = O.Lattice("D2Q9")
    rho = torch.tensor(1 + 0.1 * rng.uniform(-1, 1, (p2, q2)))
    ux = torch.tensor(0.1 * rng.uniform(-1, 1, (p2, q2)))
    uy = torch.tensor(0.1 * rng.uniform(-1, 1, (p2, q2)))
    amp = 0.6 if "positivity" in OPTS[opt] else 0.2
    g2 = O.equilibrium(lat2, rho, ux, uy, kind) * (1 + torch.tensor(rng.uniform(-amp, amp, (9, p2, q2))))
    o = dict(OPTS[opt])
    nl = o.pop("nl", False)
    coef3 = tuple(rng.uniform(-0.2, 0.4, 27)) if nl else None
    cfg3 = O.Config3(equilibrium=kind, nu=1e-4, nl_coef=coef3, **o)
    cfg2 = O.Config(lattice="D2Q9", nx=q2, ny=p2, bc="periodic", equilibrium=kind, nu=1e-4,
                    nl_coef=_coef2(coef3, axis) if nl else None, **o)
    g3 = _lift(g2, axis, n)
    out3, info3 = O.step3(cfg3, g3)
    out2, info2 = O.step(lat2, cfg2, g2)
    want = _lift(out2, axis, n)
    assert float((out3 - want).abs().max()) < 1e-13
    if o.get("median"):
        m2 = info2["median_mask"]
        m3 = m2.unsqueeze({"z": 0, "y": 1, "x": 2}[axis]).expand_as(info3["median_mask"])
        # a decision may differ only where the site's own Delta S is the
        # median (a tie, decided by the rounding of the copies along the
        # axis; the populations agree either way, the factor is 1)
        diff = (info3["median_mask"] != m3).any({"z": 0, "y": 1, "x": 2}[axis])
        dS2 = info2["dS"]
        for yy, xx in diff.nonzero().tolist():
            nb = sorted(float(dS2[(yy + dy) % p2, (xx + dx) % q2])
                        for dy in (-1, 0, 1) for dx in (-1, 0, 1))
            assert abs(nb[4] - float(dS2[yy, xx])) <= 1e-14 * float(dS2[yy, xx])
        assert bool(info2["median_mask"].any())
    if o.get("positivity"):
        assert bool(info2["positivity_mask"].any())


def _permute(g, perm):
    """The state with its axes permuted: new axis k is old axis perm[k]
    (axes in (x, y, z) order); each population moves to the index of its
    permuted velocity."""
    lat = O.Lattice3()
    gx = g.permute(0, 3, 2, 1)                              # (27, nx, ny, nz)
    res = [None] * 27
    for i, v in enumerate(lat.vel):
        j = lat.vel.index(tuple(v[perm[k]] for k in range(3)))
        res[j] = gx[i].permute(*perm)
    return torch.stack(res).permute(0, 3, 2, 1).contiguous()


def test_step3_commutes_with_axis_permutations():
    rng = np.random.default_rng(31)
    nz, ny, nx = 3, 4, 5
    shape = (nz, ny, nx)
    rho = torch.tensor(1 + 0.1 * rng.uniform(-1, 1, shape))
    u = [torch.tensor(0.1 * rng.uniform(-1, 1, shape)) for _ in range(3)]
    g = O.equilibrium3(rho, *u) * (1 + torch.tensor(rng.uniform(-0.5, 0.5, (27,) + shape)))
    cfg = O.Config3(nu=1e-4, median=True, med_delta=0.0, positivity=True)
    out, _ = O.step3(cfg, g)
    for perm in [(1, 2, 0), (2, 0, 1), (1, 0, 2)]:
        gp = _permute(g, perm)
        outp, _ = O.step3(cfg, gp)
        assert float((outp - _permute(out, perm)).abs().max()) < 1e-14


def test_step3_conserves_and_keeps_equilibrium():
    rng = np.random.default_rng(41)
    shape = (4, 5, 6)
    rho0 = torch.tensor(1 + 0.1 * rng.uniform(-1, 1, shape))
    u = [torch.tensor(0.1 * rng.uniform(-1, 1, shape)) for _ in range(3)]
    g = O.equilibrium3(rho0, *u, "entropic") * (1 + torch.tensor(rng.uniform(-0.3, 0.3, (27,) + shape)))
    coef = tuple(rng.uniform(-0.2, 0.4, 27))
    cfg = O.Config3(equilibrium="entropic", nu=1e-3, median=True, med_delta=0.0,
                    positivity=True, nl_coef=coef)
    s0 = O.stats3(g)
    out = O.run3(cfg, g, 4)
    s1 = O.stats3(out)
    for k in ("mass", "mom_x", "mom_y", "mom_z"):
        assert abs(s1[k] - s0[k]) < 1e-12 * max(1.0, abs(s0[k])), k
    # a uniform equilibrium is a fixed point
    ones = torch.ones(shape, dtype=torch.float64)
    eq = O.equilibrium3(ones, 0.03 * ones, -0.02 * ones, 0.01 * ones, "entropic")
    assert float((O.run3(cfg, eq, 2) - eq).abs().max()) < 1e-15


def test_taylor_green_3d_generator_is_divergence_free():
    rho, ux, uy, uz = G.taylor_green_3d(16, 16, 8)
    assert rho.shape == (8, 16, 16)
    # spectral derivative along each axis: div u = 0 for the Taylor-Green field
    def d(a, axis):
        k = np.fft.fftfreq(a.shape[axis]) * 2 * np.pi
        sh = [1, 1, 1]
        sh[axis] = -1
        return np.real(np.fft.ifft(1j * k.reshape(sh) * np.fft.fft(a, axis=axis), axis=axis))
    div = d(ux, 2) + d(uy, 1) + d(uz, 0)
    assert np.abs(div).max() < 1e-12
