"""Pins of the FP64 oracle against what the paper and the mathematics fix:
printed matrices, invariants, closed forms, special cases and brute force.
None of these tests touches the GPU library."""
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest
import torch

import oracle as O
from lbm_inputs import generators as G

DT = torch.float64
GOLD = os.path.join(os.path.dirname(__file__), "golden")
L2 = O.Lattice("D2Q9")
L1 = O.Lattice("D1Q3")


def rand_state(lat, ny, nx, seed, amp=0.05, umax=0.08, kind="poly"):
    """Equilibrium of random moments plus a zero-moment-free random
    perturbation (the perturbation changes the moments; that is fine)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.uniform(-1, 1, (ny, nx))
    ux = umax * rng.uniform(-1, 1, (ny, nx))
    uy = umax * rng.uniform(-1, 1, (ny, nx)) if lat.name == "D2Q9" else np.zeros((ny, nx))
    f = O.init_equilibrium(lat, rho, ux, uy, kind)
    noise = torch.tensor(rng.uniform(-amp, amp, f.shape), dtype=DT)
    return f * (1.0 + noise)


# ---------------------------------------------------------------- lattices
@pytest.mark.parametrize("lat", [L1, L2], ids=["D1Q3", "D2Q9"])
def test_lattice_isotropy(lat):
    w, vx, vy = lat.w, lat.vx, lat.vy
    assert abs(float(w.sum()) - 1.0) < 1e-15
    assert abs(float((w * vx).sum())) < 1e-16
    assert abs(float((w * vx * vx).sum()) - 1.0 / 3.0) < 1e-15   # c_s^2 = 1/3
    if lat.name == "D2Q9":
        assert abs(float((w * vx * vy).sum())) < 1e-16
        assert abs(float((w * vx ** 4).sum()) - 1.0 / 3.0) < 1e-15
        assert abs(float((w * vx ** 2 * vy ** 2).sum()) - 1.0 / 9.0) < 1e-15
    for i, j in enumerate(lat.opp):
        assert lat.vel[j] == (-lat.vel[i][0], -lat.vel[i][1])


# ---------------------------------------------------------------- equilibria
@pytest.mark.parametrize("kind", ["poly", "entropic"])
@pytest.mark.parametrize("lat", [L1, L2], ids=["D1Q3", "D2Q9"])
def test_equilibrium_moments(lat, kind):
    rng = np.random.default_rng(7)
    rho = torch.tensor(1 + 0.3 * rng.uniform(-1, 1, (5, 6)))
    ux = torch.tensor(0.2 * rng.uniform(-1, 1, (5, 6)))
    uy = torch.tensor(0.2 * rng.uniform(-1, 1, (5, 6))) if lat.name == "D2Q9" else torch.zeros(5, 6, dtype=DT)
    f = O.equilibrium(lat, rho, ux, uy, kind)
    r, jx, jy = O.moments(lat, f)
    assert torch.allclose(r, rho, rtol=0, atol=1e-15)
    assert torch.allclose(jx, rho * ux, rtol=0, atol=1e-15)
    assert torch.allclose(jy, rho * uy, rtol=0, atol=1e-15)
    zero = torch.zeros_like(ux)
    assert torch.allclose(O.equilibrium(lat, rho, zero, zero, kind),
                          lat.col(lat.w) * rho, rtol=0, atol=1e-15)


def test_poly_equilibrium_pressure_tensor():
    """The product polynomial equilibrium carries the isothermal pressure
    tensor rho (delta/3 + u u) exactly (second-order quasi-equilibrium)."""
    rng = np.random.default_rng(8)
    rho = torch.tensor(1 + 0.3 * rng.uniform(-1, 1, (4, 4)))
    ux = torch.tensor(0.2 * rng.uniform(-1, 1, (4, 4)))
    uy = torch.tensor(0.2 * rng.uniform(-1, 1, (4, 4)))
    f = O.equilibrium(L2, rho, ux, uy, "poly")
    c = L2.col
    pxx = (c(L2.vx * L2.vx) * f).sum(0)
    pxy = (c(L2.vx * L2.vy) * f).sum(0)
    pyy = (c(L2.vy * L2.vy) * f).sum(0)
    assert torch.allclose(pxx, rho * (1 / 3 + ux * ux), atol=1e-15, rtol=0)
    assert torch.allclose(pyy, rho * (1 / 3 + uy * uy), atol=1e-15, rtol=0)
    assert torch.allclose(pxy, rho * ux * uy, atol=1e-15, rtol=0)


def test_entropic_equilibrium_is_entropy_maximum():
    """ln(f*/W) is affine in the velocity (Lagrange multipliers of section 4),
    f*_0^2 = 16 f*_- f*_+ in 1D (stationarity of eq. ELBMEntropy), and any
    zero-moment perturbation lowers S."""
    rng = np.random.default_rng(9)
    rho = torch.tensor(1 + 0.3 * rng.uniform(-1, 1, (3, 3)))
    ux = torch.tensor(0.25 * rng.uniform(-1, 1, (3, 3)))
    uy = torch.tensor(0.25 * rng.uniform(-1, 1, (3, 3)))
    f = O.equilibrium(L2, rho, ux, uy, "entropic")
    lnr = torch.log(f / L2.col(L2.w)).reshape(9, -1)
    A = torch.stack([torch.ones(9, dtype=DT), L2.vx, L2.vy], 1)
    coef = torch.linalg.lstsq(A, lnr).solution
    assert float((A @ coef - lnr).abs().max()) < 1e-14
    f1 = O.equilibrium(L1, rho, ux, torch.zeros_like(ux), "entropic")
    assert torch.allclose(f1[1] ** 2, 16 * f1[0] * f1[2], rtol=1e-14, atol=0)
    # polynomial equilibrium is NOT affine in log space
    fp = O.equilibrium(L2, rho, ux, uy, "poly")
    lp = torch.log(fp / L2.col(L2.w)).reshape(9, -1)
    cp = torch.linalg.lstsq(A, lp).solution
    assert float((A @ cp - lp).abs().max()) > 1e-6
    # maximum: zero-moment perturbations (null space of the moment map)
    Mom = torch.stack([torch.ones(9, dtype=DT), L2.vx, L2.vy])
    null = torch.linalg.svd(Mom).Vh[3:]
    g0 = f.reshape(9, -1)[:, 0]
    S0 = O.entropy(L2, g0.view(9, 1, 1))
    for k in range(20):
        d = null.T @ torch.tensor(rng.normal(size=6)) * 1e-3
        assert float(O.entropy(L2, (g0 + d).view(9, 1, 1)) - S0) < 0


# ---------------------------------------------------------------- streaming
def test_periodic_streaming_is_a_permutation():
    """omega = 0 leaves pure free flight; on an n x n periodic lattice every
    population returns to its start after n steps, bit for bit."""
    cfg = O.Config(nx=6, ny=6, bc="periodic", omega=0.0)
    g0 = rand_state(L2, 6, 6, 1)
    g = O.run(L2, cfg, g0, 6)
    assert torch.equal(g, g0)
    g1, _ = O.step(L2, cfg, g0)
    # one step moves population i by its velocity
    for i, (a, b) in enumerate(L2.vel):
        assert float(g1[i, (2 + b) % 6, (3 + a) % 6]) == float(g0[i, 2, 3])


def test_d1q3_bounceback_period():
    """Free flight in a 1D tube with bounce-back ends: each moving population
    crosses the tube, reflects and returns: period 2N."""
    n = 7
    cfg = O.Config(lattice="D1Q3", nx=n, ny=1, bc="bounceback", omega=0.0)
    g0 = rand_state(L1, 1, n, 2)
    g = O.run(L1, cfg, g0, 2 * n)
    assert torch.equal(g, g0)
    assert not torch.equal(O.run(L1, cfg, g0, n), g0)


def test_cavity_walls_conserve_mass():
    cfg = O.Config(nx=8, ny=8, bc="cavity", u_lid=0.1, nu=0.02)
    g = O.init_equilibrium(L2, *G.uniform_rest(8, 8))
    m0 = O.stats(L2, g)["mass"]
    for _ in range(20):
        g, _ = O.step(L2, cfg, g)
    assert abs(O.stats(L2, g)["mass"] - m0) < 1e-12
    rho, ux, uy = O.velocity(L2, g)
    assert float(ux[-1].mean()) > 0.03           # the lid drags the top row along +x


def test_couette_flow_is_linear():
    """Plane Couette flow between a resting bounce-back floor and the moving
    lid: the steady LBGK solution is u_x = u_lid (y + 1/2) / ny, the walls
    sitting half a spacing outside the first and last rows.  Halfway
    bounce-back with the moving-wall term 6 w_i rho (v_i . u_wall) reproduces
    it to rounding, so this pins the sign, size and precision of that term."""
    ny, u = 8, 0.05
    cfg = O.Config(nx=2, ny=ny, bc="couette", u_lid=u, omega=1.2)
    g = O.init_equilibrium(L2, *G.uniform_rest(2, ny))
    g = O.run(L2, cfg, g, 3000)
    pre = O.stream(L2, g, "couette", u)
    _, ux, uy = O.velocity(L2, pre)
    exact = u * (torch.arange(ny, dtype=DT) + 0.5) / ny
    assert torch.allclose(ux[:, 0], exact, atol=1e-13, rtol=0)
    assert float(uy.abs().max()) < 1e-12


def test_bounceback_reflects_into_opposite():
    cfg = O.Config(nx=3, ny=3, bc="bounceback", omega=0.0)
    g0 = rand_state(L2, 3, 3, 3)
    g1, _ = O.step(L2, cfg, g0)
    # population moving +x (a=1,b=0) at x=0 came from the wall: it is the
    # -x population of the same node.
    i = L2.vel.index((1, 0))
    assert torch.equal(g1[i, :, 0], g0[L2.opp[i], :, 0])


# ---------------------------------------------------------------- LBGK
def test_lbgk_conserves_and_fixes_equilibrium():
    f = rand_state(L2, 5, 5, 4)
    rho, ux, uy = O.velocity(L2, f)
    feq = O.equilibrium(L2, rho, ux, uy)
    post = O.lbgk(f, feq, 1.7)
    r2, jx2, jy2 = O.moments(L2, post)
    assert torch.allclose(r2, rho, atol=1e-15, rtol=0)
    assert torch.allclose(jx2, rho * ux, atol=1e-15, rtol=0)
    assert torch.allclose(O.lbgk(feq, feq, 1.7), feq, atol=1e-16, rtol=0)


def test_lbgk_entropy_production_quadratic():
    """Near equilibrium one LBGK collision scales Delta S by (1 - omega)^2,
    i.e. the production [1 - (2 beta - 1)^2] Delta S of the dissipation
    monitor (section 4, 'Monitoring total dissipation'), beta = omega/2."""
    f0 = rand_state(L2, 3, 3, 5, amp=0.0)
    rho, ux, uy = O.velocity(L2, f0)
    feq = O.equilibrium(L2, rho, ux, uy)
    rng = np.random.default_rng(5)
    Mom = torch.stack([torch.ones(9, dtype=DT), L2.vx, L2.vy])
    null = torch.linalg.svd(Mom).Vh[3:]
    d = (null.T @ torch.tensor(rng.normal(size=(6, 9)))).reshape(9, 3, 3) * 1e-8
    f = feq + d
    for omega in (0.7, 1.3, 1.9):
        post = O.lbgk(f, feq, omega)
        ratio = O.kullback_dS(post, feq) / O.kullback_dS(f, feq)
        assert torch.allclose(ratio, torch.full_like(ratio, (1 - omega) ** 2), rtol=1e-5, atol=0)
        beta = omega / 2
        prod = O.kullback_dS(f, feq) - O.kullback_dS(post, feq)
        assert torch.allclose(prod, (1 - (2 * beta - 1) ** 2) * O.kullback_dS(f, feq), rtol=1e-5)


def shear_decay_rate(cfg, n=64):
    """Exponential decay rate of the shear-wave amplitude, measured after the
    start-up transient of an equilibrium initialisation (from T/4 to T,
    T = n / (4 u0) steps)."""
    rho, ux, uy = G.shear_wave(n, 0.05)
    g = O.init_equilibrium(L2, rho, ux, uy)
    T = int(n / 0.05) // 4
    s = torch.sin(2 * math.pi * torch.arange(n, dtype=DT) / n)

    def amp(g):
        _, _, vy = O.velocity(L2, g)
        return float((vy.mean(0) * s).sum() / (s * s).sum())
    g = O.run(L2, cfg, g, T // 4)
    a1 = amp(g)
    g = O.run(L2, cfg, g, T - T // 4)
    return -math.log(amp(g) / a1) / (T - T // 4)


@pytest.mark.parametrize("collision,basis,preset", [("lbgk", "M1", "given"), ("mrt", "M1", "given"),
                                                    ("mrt", "M2", "given"), ("mrt", "M1", "trt"),
                                                    ("mrt", "M1", "shear")])
def test_shear_wave_viscosity(collision, basis, preset):
    """Section 7: the shear wave decays as exp(-nu k^2 t) with
    nu = c_s^2 (1/omega - 1/2), k = 2 pi / n; MRT produces the same shear
    viscosity as BGK, whatever its other rates (the TRT and shear-wave
    presets included).  The lattice error is O(k^2): 0.3 % at n = 32,
    0.08 % at n = 64."""
    n, nu = 64, 0.02
    cfg = O.Config(nx=n, ny=n, bc="periodic", nu=nu, collision=collision,
                   mrt_basis=basis, s_e=1.64, s_eps=1.54, s_q=1.9, mrt_preset=preset)
    rate = shear_decay_rate(cfg, n)
    k = 2 * math.pi / n
    assert abs(rate / (nu * k * k) - 1) < 2e-3


def test_mrt_presets():
    """The M1 rate presets.  TRT (section 5) sets s_e = s_eps = s_nu and its
    third-order rate so that the product of the two relaxation parameters
    Lambda = (1/s_nu - 1/2)(1/s_q - 1/2) is the constant 3/16 for every
    s_nu; the shear-wave MRT of section 7 has Lambda = 1/12; the cavity
    study's MRT takes the TRT third-order rate with s_e = 1.64,
    s_eps = 1.54; MRT1 (section 8) is s_q = 1.9, s_e = 1.64, s_eps = 1.54.
    Per-site shear rates give per-site presets."""
    s_nu = torch.tensor([0.5, 1.0, 1.5, 1.9, 1.99], dtype=DT)
    lam = lambda sq: (1 / s_nu - 0.5) * (1 / sq - 0.5)  # noqa: E731
    se, seps, sq = O.mrt_preset_rates("trt", s_nu)
    assert torch.equal(se, s_nu) and torch.equal(seps, s_nu)
    assert torch.allclose(lam(sq), torch.full_like(s_nu, 3 / 16), rtol=1e-12, atol=0)
    se, seps, sq = O.mrt_preset_rates("shear", s_nu)
    assert (se, seps) == (1.64, 1.54)
    assert torch.allclose(lam(sq), torch.full_like(s_nu, 1 / 12), rtol=1e-12, atol=0)
    se, seps, sq2 = O.mrt_preset_rates("mrt_trtq", s_nu)
    assert (se, seps) == (1.64, 1.54) and torch.equal(sq2, O.mrt_preset_rates("trt", s_nu)[2])
    assert O.mrt_preset_rates("mrt1", s_nu) == (1.64, 1.54, 1.9)
    assert O.mrt_preset_rates("given", s_nu, 1.1, 1.2, 1.3) == (1.1, 1.2, 1.3)
    # a TRT step relaxes e and epsilon at the shear rate: the energy-like
    # nonequilibrium moments decay exactly like the shear ones
    f = rand_state(L2, 2, 3, 95, amp=0.1)
    r, vx, vy = O.velocity(L2, f)
    q = O.equilibrium(L2, r, vx, vy)
    M = O.mrt_basis("M1")
    cfg = O.Config(nx=3, ny=2, bc="periodic", omega=1.3, collision="mrt", mrt_preset="trt")
    post = O.mrt(f, q, M, O.mrt_rates("M1", *O.mrt_preset_rates("trt", 1.3), 1.3))
    dm_in = (M @ (f - q).reshape(9, -1))
    dm_out = (M @ (post - q).reshape(9, -1))
    for row in (1, 2, 7, 8):
        assert torch.allclose(dm_out[row], (1 - 1.3) * dm_in[row], atol=1e-15, rtol=0)
    a, _ = O.step(L2, cfg, f)
    assert a.shape == f.shape


def test_mrt_limiter():
    """The MRT limiter of section 5 on an LBGK lattice: the k sites of
    largest Delta S > delta receive the MRT collision (M2/C2: every mode but
    shear sent to equilibrium) instead of LBGK's; all other sites are LBGK.
    With k >= N and delta = 0 the step is the MRT step at every site; with a
    small k exactly the brute-force top-k sites differ from LBGK; moments
    are conserved."""
    g = rand_state(L2, 5, 6, 96, amp=0.1)
    base = dict(nx=6, ny=5, bc="periodic", nu=1e-3, ehrenfest=True, ehr_delta=0.0,
                sel_action="mrt", mrt_basis="M2")
    a, _ = O.step(L2, O.Config(**base, ehr_k=30), g)
    b, _ = O.step(L2, O.Config(**{**base, "ehrenfest": False}, collision="mrt"), g)
    assert torch.allclose(a, b, atol=1e-16, rtol=0)
    c, info = O.step(L2, O.Config(**base, ehr_k=4), g)
    d, _ = O.step(L2, O.Config(**{**base, "ehrenfest": False}), g)
    diff = ((c - d).abs().amax(0) > 0).flatten().nonzero().flatten().tolist()
    dS = info["dS"].flatten()
    top = sorted(range(30), key=lambda i: (-float(dS[i]), i))[:4]
    assert diff == sorted(top) == info["selected"].tolist()
    for m_c, m_g in zip(O.moments(L2, c), O.moments(L2, O.stream(L2, g, "periodic"))):
        assert torch.allclose(m_c, m_g, atol=1e-15, rtol=0)


# ---------------------------------------------------------------- MRT
def _printed(name):
    lines = [l for l in open(os.path.join(GOLD, name)) if l.strip() and not l.startswith("#")]
    vel = [tuple(int(t) for t in p.split(",")) for p in lines[0].split()[1:]]
    M = torch.tensor([[float(t) for t in l.split()] for l in lines[1:]], dtype=DT)
    return vel, M


def test_m1_matches_printed_matrix():
    vel, Mp = _printed("m1_printed.txt")
    perm = [vel.index(v) for v in L2.vel]     # printed column for each of our columns
    assert torch.equal(O.mrt_basis("M1"), Mp[:, perm])
    M = O.mrt_basis("M1")
    assert torch.equal(M @ M.T, torch.diag(torch.tensor([9., 36, 36, 6, 12, 6, 12, 4, 4], dtype=DT)))


def test_m2_matches_printed_matrix():
    vel, Mp = _printed("m2_printed.txt")
    perm = [vel.index(v) for v in L2.vel]
    M = O.mrt_basis("M2")
    Pm = Mp[:, perm]
    assert torch.equal(M[:6], Pm[:6]) and torch.equal(M[8], Pm[8])
    assert torch.equal(M[6], Pm[7]) and torch.equal(M[7], Pm[6])   # printed rows 7/8 swapped


def test_a2_sparsity_and_symmetry():
    """A2 = M2^-1 C2 M2 is symmetric with twelve off-diagonal pairs
    (24 nonzero off-diagonal entries)."""
    M = O.mrt_basis("M2")
    for s_nu in (0.6, 1.3, 1.9):
        A = torch.linalg.inv(M) @ torch.diag(O.mrt_rates("M2", 0, 0, 0, s_nu)) @ M
        assert torch.allclose(A, A.T, atol=1e-14)
        off = A - torch.diag(torch.diag(A))
        assert int((off.abs() > 1e-12).sum()) == 24


def test_mrt_special_cases():
    f = rand_state(L2, 4, 4, 6)
    rho, ux, uy = O.velocity(L2, f)
    feq = O.equilibrium(L2, rho, ux, uy)
    om = 1.37
    M1 = O.mrt_basis("M1")
    allsame = O.mrt(f, feq, M1, torch.full((9,), om, dtype=DT))
    assert torch.allclose(allsame, O.lbgk(f, feq, om), atol=1e-15, rtol=0)
    M2 = O.mrt_basis("M2")
    ehr = O.mrt(f, feq, M2, O.mrt_rates("M2", 0, 0, 0, 1.0))
    assert torch.allclose(ehr, feq, atol=1e-15, rtol=0)
    post = O.mrt(f, feq, M1, O.mrt_rates("M1", 1.64, 1.54, 1.9, om))
    r2, jx2, jy2 = O.moments(L2, post)
    assert torch.allclose(r2, rho, atol=1e-15, rtol=0)
    assert torch.allclose(jx2, rho * ux, atol=1e-15, rtol=0)
    assert torch.allclose(jy2, rho * uy, atol=1e-15, rtol=0)
    # per-site shear rate equals the scalar one where they agree
    field = torch.full((4, 4), om, dtype=DT)
    a = O.mrt(f, feq, M1, O.mrt_rates("M1", 1.64, 1.54, 1.9, field))
    assert torch.allclose(a, post, atol=1e-16, rtol=0)


# ---------------------------------------------------------------- Delta S
getcontext().prec = 50


def _dec_S(g, W):
    return -sum((gi * (gi / wi).ln()) if gi > 0 else Decimal(0) for gi, wi in zip(g, W))


def test_kullback_matches_high_precision():
    """Delta S equals the Kullback sum sum f ln(f/f*) evaluated in 50-digit
    decimal arithmetic, to full double precision, from large deviations down
    to ones far below the rounding of rho; for entropic f* it equals
    S(f*) - S(f) (eq. DelS)."""
    rng = np.random.default_rng(11)
    for amp in (0.3, 1e-2, 1e-5, 1e-8):
        f = rand_state(L2, 1, 6, int(amp * 1e9) % 1000, amp=0.0, kind="entropic")
        rho, ux, uy = O.velocity(L2, f)
        Mom = torch.stack([torch.ones(9, dtype=DT), L2.vx, L2.vy])
        null = torch.linalg.svd(Mom).Vh[3:]
        d = (null.T @ torch.tensor(rng.normal(size=(6, 6)))).reshape(9, 1, 6) * amp * 0.1
        g = (f + d).clamp(min=1e-6)
        r, vx, vy = O.velocity(L2, g)
        for kind in ("poly", "entropic"):
            q = O.equilibrium(L2, r, vx, vy, kind)
            dS = O.kullback_dS(g, q)
            for s in range(6):
                gd = [Decimal(float(x)) for x in g[:, 0, s]]
                qd = [Decimal(float(x)) for x in q[:, 0, s]]
                lit = sum(a * (a / b).ln() for a, b in zip(gd, qd)) - (sum(gd) - sum(qd))
                assert abs(float(lit) - float(dS[0, s])) <= 4e-16 * abs(float(lit)) + 1e-300
                if kind == "entropic":
                    W = [Decimal(float(w)) for w in L2.w]
                    diff = _dec_S(qd, W) - _dec_S(gd, W)
                    # exact for the exact f*; the rounding of f* to double
                    # leaves an absolute residue of order 1e-16
                    assert abs(float(diff) - float(dS[0, s])) <= 1e-13 * float(dS[0, s]) + 2e-15


def test_kullback_quadratic_approximation():
    """In quadratic approximation Delta S ~ (1/2) sum (f - f*)^2 / f*; eq.
    KulSq prints the sum without the 1/2, which this test shows is off by 2."""
    f0 = rand_state(L2, 2, 2, 12, amp=0.0)
    rho, ux, uy = O.velocity(L2, f0)
    q = O.equilibrium(L2, rho, ux, uy)
    Mom = torch.stack([torch.ones(9, dtype=DT), L2.vx, L2.vy])
    null = torch.linalg.svd(Mom).Vh[3:]
    d = (null.T @ torch.tensor(np.random.default_rng(1).normal(size=(6, 4)))).reshape(9, 2, 2) * 1e-8
    dS = O.kullback_dS(q + d, q)
    quad = 0.5 * (d * d / q).sum(0)
    assert torch.allclose(dS, quad, rtol=1e-5, atol=0)


def test_kullback_negative_population_ranks_first():
    f = rand_state(L2, 1, 2, 13)
    f[3, 0, 1] = -1e-3
    rho, ux, uy = O.velocity(L2, f)
    dS = O.kullback_dS(f, O.equilibrium(L2, rho, ux, uy))
    assert math.isinf(float(dS[0, 1])) and math.isfinite(float(dS[0, 0]))


# ---------------------------------------------------------------- ELBM
def _dec_entropic_eq(fd):
    """Entropic D2Q9 equilibrium of the moments of fd, in decimal."""
    rho = sum(fd)
    ux = sum(Decimal(a) * x for (a, _), x in zip(L2.vel, fd)) / rho
    uy = sum(Decimal(b) * x for (_, b), x in zip(L2.vel, fd)) / rho

    def phi(u):
        s = (1 + 3 * u * u).sqrt()
        return [(-3 * u - 1 + 2 * s) / 6, Decimal(2) / 3 * (2 - s), (3 * u - 1 + 2 * s) / 6]
    px, py = phi(ux), phi(uy)
    return [rho * px[a + 1] * py[b + 1] for (a, b) in L2.vel]


def _dec_root(f, lo, hi, iters=200):
    """Bisection, in 50-digit decimal, of S(f + a (f* - f)) - S(f) on
    (lo, hi), with f* the exact entropic equilibrium of f."""
    W = [Decimal(1) / 36, Decimal(1) / 9, Decimal(1) / 36, Decimal(1) / 9, Decimal(4) / 9,
         Decimal(1) / 9, Decimal(1) / 36, Decimal(1) / 9, Decimal(1) / 36]
    fd = [Decimal(float(x)) for x in f]
    qd = _dec_entropic_eq(fd)
    Dd = [b - a for a, b in zip(fd, qd)]
    S0 = _dec_S(fd, W)

    def Sf(a):
        return _dec_S([x + a * d for x, d in zip(fd, Dd)], W) - S0
    lo, hi = Decimal(lo), Decimal(hi)
    for _ in range(iters):
        mid = (lo + hi) / 2
        if Sf(mid) > 0:
            lo = mid
        else:
            hi = mid
    return float(lo), Sf


def test_elbm_root_matches_bisection_and_is_a_lower_estimate():
    """The ELBM alpha is the nontrivial root of S(f + alpha Delta) = S(f)
    (eq. ELBMCondition) to within eps / ||Delta||, and never above it
    (the sign check of section 3)."""
    rng = np.random.default_rng(21)
    checked = 0
    for amp in (0.02, 0.1, 0.3):
        f0 = rand_state(L2, 1, 5, 30 + int(amp * 100), amp=0.0, kind="entropic")
        Mom = torch.stack([torch.ones(9, dtype=DT), L2.vx, L2.vy])
        null = torch.linalg.svd(Mom).Vh[3:]
        d = (null.T @ torch.tensor(rng.normal(size=(6, 5)))).reshape(9, 1, 5) * amp * 0.05
        f = (f0 + d).reshape(9, -1)
        assert bool((f > 0).all())
        r, vx, vy = O.velocity(L2, f.view(9, 1, 5))
        q = O.equilibrium(L2, r, vx, vy, "entropic").reshape(9, -1)
        alpha, branch = O.elbm_alpha(f, q)
        D = q - f
        nrm = torch.sqrt((D * D / q).sum(0))
        for s in range(5):
            if int(branch[s]) != O.ELBM_ROOT:
                continue
            ratios = [float(f[i, s] / -D[i, s]) for i in range(9) if D[i, s] < 0]
            hi = min(ratios) if ratios else 10.0
            root, Sf = _dec_root(f[:, s], 1.0 + 1e-12, hi)
            a = float(alpha[s])
            # lower estimate, up to a few ulp of alpha and the rounding of f*
            assert a <= root + 2e-15
            assert root - a <= 2 * 1e-14 / float(nrm[s]) + 1e-13
            checked += 1
    assert checked >= 10


def _dec_sf_d1(f, a):
    """S_f(a) = S(f + a D) - S(f) and its derivative in a, evaluated from the
    definition in 50-digit decimal with the exact entropic equilibrium of f
    (D = f* - f).  Returns (S_f, S_f', D, f*)."""
    W = [Decimal(1) / 36, Decimal(1) / 9, Decimal(1) / 36, Decimal(1) / 9, Decimal(4) / 9,
         Decimal(1) / 9, Decimal(1) / 36, Decimal(1) / 9, Decimal(1) / 36]
    fd = [Decimal(float(x)) for x in f]
    qd = _dec_entropic_eq(fd)
    Dd = [b - x for x, b in zip(fd, qd)]
    a = Decimal(a)
    g = [x + a * d for x, d in zip(fd, Dd)]
    sf = _dec_S(g, W) - _dec_S(fd, W)
    # dS(f + a D)/da = -sum D_i (ln(g_i / W_i) + 1), and sum D_i = 0
    d1 = -sum(d * (gi / wi).ln() for d, gi, wi in zip(Dd, g, W))
    return sf, d1, Dd, qd


def test_elbm_l1_norm_stopping_rule():
    """The stopping test of the root iteration, |S_f / S_f'| ||Delta|| < eps
    (section 3, "Numerical method"), with either norm of Delta: the L1 norm
    sum |Delta_i| or the entropic norm sqrt(sum Delta_i^2 / f*_i).

    (i) eps = 1e-14, L1 norm: alpha is a lower estimate of the root within
    2 eps / ||Delta||_1 (50-digit bisection), as for the entropic norm.
    (ii) The test at the start alpha_0 = 2: with eps set to the geometric mean
    of |S_f/S_f'|(2) ||Delta||_1 and |S_f/S_f'|(2) ||Delta||_ent (both from the
    definition, in decimal), exactly one of the two norms stops at alpha_0,
    and its result is alpha_0 followed by the sign check (alpha_0 when
    S_f(2) >= 0, else the double-length Newton step 2 - 2 S_f / S_f'); the
    other norm iterates on to the root.  A wrong norm (a missing absolute
    value, a missing square root, a swapped option) changes which one stops."""
    rng = np.random.default_rng(23)
    checked = both = 0
    for amp in (0.02, 0.1, 0.3):
        f0 = rand_state(L2, 1, 6, 40 + int(amp * 100), amp=0.0, kind="entropic")
        Mom = torch.stack([torch.ones(9, dtype=DT), L2.vx, L2.vy])
        null = torch.linalg.svd(Mom).Vh[3:]
        d = (null.T @ torch.tensor(rng.normal(size=(6, 6)))).reshape(9, 1, 6) * amp * 0.05
        f = (f0 + d).reshape(9, -1)
        assert bool((f > 0).all())
        r, vx, vy = O.velocity(L2, f.view(9, 1, 6))
        q = O.equilibrium(L2, r, vx, vy, "entropic").reshape(9, -1)
        alpha, branch = O.elbm_alpha(f, q, norm="l1")
        for s in range(6):
            if int(branch[s]) != O.ELBM_ROOT:
                continue
            sf, d1, Dd, qd = _dec_sf_d1(f[:, s], 2)
            n1 = sum(abs(x) for x in Dd)
            ne = sum(x * x / y for x, y in zip(Dd, qd)).sqrt()
            hi = min([float(f[i, s] / (q[i, s] - f[i, s])) * -1 for i in range(9)
                      if q[i, s] < f[i, s]] or [10.0])
            root, _ = _dec_root(f[:, s], 1.0 + 1e-12, hi)
            a = float(alpha[s])
            assert a <= root + 2e-15
            assert root - a <= 2 * 1e-14 / float(n1) + 1e-13
            checked += 1
            # (ii): eps between the two norms' values of the test at alpha = 2
            r0 = abs(sf / d1)
            lo_n, hi_n = min(n1, ne), max(n1, ne)
            if hi_n / lo_n < Decimal("1.02"):
                continue
            eps = float(r0 * (n1 * ne).sqrt())
            stop_val = 2.0 if sf >= 0 else float(2 - 2 * sf / d1)
            a1, _ = O.elbm_alpha(f[:, s:s + 1], q[:, s:s + 1], norm="l1", eps=eps)
            ae, _ = O.elbm_alpha(f[:, s:s + 1], q[:, s:s + 1], norm="entropic", eps=eps)
            stopped, iterated = (a1, ae) if n1 < ne else (ae, a1)
            assert abs(float(stopped[0]) - stop_val) <= 1e-14
            assert abs(float(iterated[0]) - root) < abs(stop_val - root)
            both += 1
    assert checked >= 10 and both >= 5


def test_elbm_nonpositive_population_reading():
    """Reading: a site with a population <= 0 has no entropy (ln of a
    non-positive number), so no entropic root exists; it takes alpha = 1, the
    Ehrenfest-rule value (section 3, rule 1), and the ELBM collision is then
    f + beta (f* - f).  The branch is reported as non-positive."""
    f = rand_state(L2, 1, 3, 90, amp=0.05, kind="entropic").reshape(9, -1).clone()
    f[2, 0] = 0.0
    f[5, 1] = -1e-3
    r, vx, vy = O.velocity(L2, f.view(9, 1, 3))
    q = O.equilibrium(L2, r, vx, vy, "entropic").reshape(9, -1)
    a, b = O.elbm_alpha(f, q)
    assert b.tolist()[:2] == [O.ELBM_NONPOS, O.ELBM_NONPOS] and int(b[2]) != O.ELBM_NONPOS
    assert float(a[0]) == 1.0 and float(a[1]) == 1.0
    om = 1.7
    post, alpha, branch = O.elbm(f.view(9, 1, 3), q.view(9, 1, 3), om)
    exp = f[:, :2] + (om / 2) * (q[:, :2] - f[:, :2])
    assert torch.equal(post.reshape(9, -1)[:, :2], exp)


def test_elbm_alpha_tends_to_two_and_cutoff():
    f0 = rand_state(L2, 1, 3, 40, amp=0.0, kind="entropic").reshape(9, -1)
    r, vx, vy = O.velocity(L2, f0.view(9, 1, 3))
    q = O.equilibrium(L2, r, vx, vy, "entropic").reshape(9, -1)
    Mom = torch.stack([torch.ones(9, dtype=DT), L2.vx, L2.vy])
    null = torch.linalg.svd(Mom).Vh[3:]
    d = null.T @ torch.tensor(np.random.default_rng(3).normal(size=(6, 3)))
    prev = None
    for amp in (1e-2, 1e-3, 1e-4, 1e-5):
        a, b = O.elbm_alpha(q + amp * d, q)
        err = float((a - 2).abs().max())
        if prev is not None:
            assert err < prev * 0.2          # |alpha - 2| = O(|Delta|)
        prev = err
    a, b = O.elbm_alpha(q + 1e-9 * d, q)      # Delta S ~ 1e-17 < 1e-15
    assert torch.equal(a, torch.full_like(a, 2.0))
    assert bool((b == O.ELBM_CUTOFF).all())


def test_elbm_no_root_positivity_rule():
    """A state far from equilibrium whose mirror state would need negative
    populations: S_f(alpha_max) >= 0, so the positivity rule takes the
    largest alpha keeping f + alpha (f* - f) >= 0 (section 3, rule 2)."""
    f = torch.tensor([0.3, 0.001, 0.001, 0.001, 0.3, 0.001, 0.001, 0.001, 0.3], dtype=DT).view(9, 1)
    r, vx, vy = O.velocity(L2, f.view(9, 1, 1))
    q = O.equilibrium(L2, r, vx, vy, "entropic").reshape(9, 1)
    a, b = O.elbm_alpha(f, q)
    assert int(b[0]) == O.ELBM_NOROOT
    g = f + a * (q - f)
    assert float(g.min()) >= -1e-16 and float(g.min()) < 1e-15
    a2, b2 = O.elbm_alpha(f, q, fallback="ehrenfest")
    assert float(a2[0]) == 1.0


def test_elbm_total_entropy_non_decreasing():
    """H theorem (section 3): on a periodic lattice streaming permutes
    populations of equal weight, and the ELBM collision with beta <= 1 does
    not lower the local entropy, so the total entropy never falls."""
    cfg = O.Config(nx=12, ny=12, bc="periodic", nu=1e-4, collision="elbm")
    rho, ux, uy = G.spectral_velocity(12, k_peak=3, u_rms=0.08, seed=5)
    g = O.init_equilibrium(L2, rho, ux, uy, "entropic")
    g = g * (1 + 0.02 * torch.tensor(G.uniform_noise(g.shape, 6)))
    S = O.stats(L2, g)["entropy"]
    for _ in range(15):
        g, info = O.step(L2, cfg, g)
        S2 = O.stats(L2, g)["entropy"]
        assert S2 >= S - 1e-13
        S = S2


# ---------------------------------------------------------------- positivity
def test_positivity_rule():
    """Section 4: a state with negative components moves along the line to
    f* until the first component reaches 0; moments are unchanged because the
    state and f* share them."""
    f = rand_state(L2, 3, 4, 50, amp=0.0)
    rho, ux, uy = O.velocity(L2, f)
    q = O.equilibrium(L2, rho, ux, uy)
    Mom = torch.stack([torch.ones(9, dtype=DT), L2.vx, L2.vy])
    null = torch.linalg.svd(Mom).Vh[3:]
    d = (null.T @ torch.tensor(np.random.default_rng(51).normal(size=(6, 12)))).reshape(9, 3, 4)
    post = q + 0.12 * d
    out, act = O.positivity(post, q)
    assert bool(act.any()) and bool((~act).any())
    assert float(out.min()) >= 0.0
    mins = out.reshape(9, -1).min(0).values
    assert bool((mins[act.flatten()] == 0).all())
    assert torch.equal(out[:, ~act], post[:, ~act])
    for m_out, m_in in zip(O.moments(L2, out), O.moments(L2, post)):
        assert torch.allclose(m_out, m_in, atol=1e-15, rtol=0)
    # on the straight line through post and f*, between them
    d_out, d_in = (out - q).reshape(9, -1), (post - q).reshape(9, -1)
    lam = (d_out * d_in).sum(0) / (d_in * d_in).sum(0)
    assert torch.allclose(d_out, lam * d_in, atol=1e-15)
    assert bool(((lam > 0) & (lam <= 1)).all())


# ---------------------------------------------------------------- Ehrenfest
def test_ehrenfest_selection_brute_force():
    rng = np.random.default_rng(60)
    vals = rng.choice([0.0, 1e-4, 2e-4, 3e-4, 5e-3], size=40).astype(float)
    vals[[3, 9, 17]] = 7e-3                                   # ties
    dS = torch.tensor(vals)
    for k, delta in ((0, 0.0), (2, 0.0), (4, 1e-4), (7, 0.0), (100, 0.0), (5, 1.0)):
        got = O.ehrenfest_select(dS, k, delta).tolist()
        cand = [i for i in range(40) if vals[i] > delta]
        cand.sort(key=lambda i: (-vals[i], i))
        assert got == sorted(cand[:k])


def test_ehrenfest_all_sites_is_omega_one():
    """With k >= N and delta = 0 every non-equilibrium site is sent to f*,
    which is the LBGK step with omega = 1."""
    g = rand_state(L2, 5, 5, 61)
    cfg = O.Config(nx=5, ny=5, bc="periodic", nu=1e-3, ehrenfest=True, ehr_k=25, ehr_delta=0.0)
    a, _ = O.step(L2, cfg, g)
    b, _ = O.step(L2, cfg.with_(ehrenfest=False, nu=None, omega=1.0), g)
    assert torch.allclose(a, b, atol=1e-16, rtol=0)


# ---------------------------------------------------------------- ensemble limiters
def test_ens_threshold_solves_entthresh_by_brute_force():
    """Eq. EntThresh over an empirical distribution: the returned Delta S_0
    satisfies sum_{Delta S > Delta S_0} (Delta S - Delta S_0) = delta_0 P by
    direct summation, for distinct values, ties and zeros, and the left side
    is strictly larger just below it (unique root); delta_0 P at or above
    sum Delta S gives 0; +inf values are ignored."""
    rng = np.random.default_rng(101)
    cases = [rng.exponential(1e-3, 40), np.array([5e-3] * 7 + [1e-3] * 5 + [0.0] * 4),
             rng.lognormal(-8, 2, 300)]
    for vals in cases:
        dS = torch.tensor(vals)
        P = float(dS.sum())
        for d0 in (1e-3, 0.05, 0.3, 0.9):
            s0 = O.ens_threshold(dS, P, d0)
            lhs = float(torch.clamp(dS - s0, min=0).sum())
            assert abs(lhs - d0 * P) <= 1e-12 * P
            assert float(torch.clamp(dS - s0 * (1 - 1e-9), min=0).sum()) > d0 * P
        assert 0.0 <= O.ens_threshold(dS, P, 1.0) <= 1e-14 * float(dS.max())
    dS = torch.tensor([1e-3, 2e-3, math.inf, 4e-3], dtype=DT)
    s0 = O.ens_threshold(dS, 7e-3, 0.1)
    assert abs(float(torch.clamp(dS[torch.isfinite(dS)] - s0, min=0).sum()) - 7e-4) < 1e-15


def test_ensemble_phi_closed_forms():
    """The phi of section 4.  phiExamp: 1 at Delta S = alpha E, -> 1 for
    small Delta S, -> sqrt(alpha E / Delta S) for large.  DoublMonSpec: the
    solution exp(-1/2 int_0^x eta(chi)/chi dchi) of eq. DoublMonGen with
    eta = x^k / (Delta S_t^k + x^k) (numerical quadrature), double monotone
    (phi + 2 x phi' >= 0, phi' <= 0), 1 - x^k / (2k Delta S_t^k) for small
    x and sqrt(Delta S_t / x) for large.  Pointwise 1/(1 + alpha x^k) is
    dissipative.  Threshold: entrHom above Delta S_t, 1 below.  phi = 0 at
    Delta S = +inf."""
    cfg = O.Config(ens_alpha=2.0, ens_k=1.5)
    x = torch.tensor([1e-9, 1e-6, 1e-4, 1e-3, 2e-3, 1e-1, 10.0, math.inf], dtype=DT)
    E, t = 1e-3, 2e-3
    sm = O.ens_phi(cfg.with_(ens_limiter="smooth"), x, E, t)
    assert abs(float(sm[4]) - 1.0) < 1e-15 and abs(float(sm[0]) - 1) < 1e-5
    assert abs(float(sm[6]) / math.sqrt(2 * E / 10.0) - 1) < 2e-2 and float(sm[7]) == 0.0
    for k in (0.5, 1.0, 2.0):
        c = cfg.with_(ens_limiter="double_monotone", ens_k=k)
        xs = torch.tensor(np.geomspace(1e-7, 1e2, 400))
        ph = O.ens_phi(c, xs, E, t)
        # eq. DoublMonGen by quadrature in log chi
        lx = np.log(xs.numpy())
        eta = xs.numpy() ** k / (t ** k + xs.numpy() ** k)
        integ = np.concatenate([[eta[0] / k], eta[0] / k + np.cumsum(0.5 * (eta[1:] + eta[:-1]) * np.diff(lx))])
        ref = np.exp(-0.5 * integ)
        assert np.allclose(ph.numpy(), ref, rtol=2e-4)
        d = np.gradient(ph.numpy(), xs.numpy())
        # finite differences on the geometric grid: error about 2e-4 where
        # phi + 2 x phi' tends to 0
        assert (d <= 1e-12).all() and (ph.numpy() + 2 * xs.numpy() * d >= -1e-3).all()
        u = (float(xs[0]) / t) ** k            # second-order remainder O(u^2)
        assert abs(float(ph[0]) - (1 - u / (2 * k))) < u * u + 4e-16
        assert abs(float(ph[-1]) / math.sqrt(t / float(xs[-1])) - 1) < 1e-2
    pw = O.ens_phi(cfg.with_(ens_limiter="pointwise"), x, E, t)
    assert bool(((pw >= 0) & (pw <= 1)).all())
    th = O.ens_phi(cfg.with_(ens_limiter="threshold"), x, E, t)
    assert torch.equal(th[:4], torch.ones(4, dtype=DT)) and float(th[4]) == 1.0
    assert abs(float(th[5]) - math.sqrt(t / 0.1)) < 1e-15 and float(th[7]) == 0.0


def test_threshold_limiter_dissipation_budget():
    """Section 4, "Monitoring total dissipation": with Delta S_t = Delta S_0 of
    eq. EntThresh (above delta), the threshold limiter's entropy production in
    quadratic approximation, sum (1 - phi^2) Delta S, is exactly delta_0
    times the LBGK production [1 - (2 beta - 1)^2] sum Delta S; the limited
    sites' Delta S becomes Delta S_t in that approximation and the moments
    are kept.  A whole step with the limiter on agrees with the limiter
    applied by hand before the LBGK collision."""
    g = rand_state(L2, 12, 12, 102, amp=0.2)
    cfg = O.Config(nx=12, ny=12, bc="periodic", nu=1e-3, ens_limiter="threshold",
                   ens_delta0=0.05, ens_delta=0.0)
    pre = O.stream(L2, g, "periodic")
    r, vx, vy = O.velocity(L2, pre)
    q = O.equilibrium(L2, r, vx, vy)
    dS = O.kullback_dS(pre, q)
    om = O.relaxation_rate(cfg)
    out, info = O.ensemble_limiter(cfg, pre, q, dS, om)
    P = (1 - (om - 1) ** 2) * float(dS.sum())
    assert abs(info["lbgk_production"] - P) <= 1e-12 * P
    assert abs(info["limiter_production"] - 0.05 * P) <= 1e-11 * P
    acc = dS >= info["threshold"]
    assert 0 < int(acc.sum()) < 144
    approx = (info["phi"] ** 2 * dS)[acc]
    assert torch.allclose(approx, torch.full_like(approx, info["threshold"]), rtol=1e-12)
    for a, b in zip(O.moments(L2, out), O.moments(L2, pre)):
        assert torch.allclose(a, b, atol=1e-15, rtol=0)
    full, inf2 = O.step(L2, cfg, g)
    by_hand = O.lbgk(out, q, om)
    assert torch.allclose(full, by_hand, atol=1e-16, rtol=0)
    assert inf2["ensemble"]["threshold"] == info["threshold"]


# ---------------------------------------------------------------- median
def _median_brute(dS, periodic, wrap_x=None):
    wrap_x = periodic if wrap_x is None else wrap_x
    ny, nx = dS.shape
    med = np.zeros_like(dS)
    for y in range(ny):
        for x in range(nx):
            vals = []
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if ny == 1 and dy != 0:
                        continue
                    yy, xx = y + dy, x + dx
                    if periodic:
                        yy = yy % ny
                    if wrap_x:
                        xx = xx % nx
                    if not (0 <= yy < ny and 0 <= xx < nx):
                        continue
                    vals.append(dS[yy, xx])
            vals.sort()
            med[y, x] = vals[(len(vals) + 1) // 2 - 1]
    return med


@pytest.mark.parametrize("lat,ny,nx,bc", [(L2, 5, 6, "cavity"), (L2, 4, 5, "periodic"),
                                          (L2, 5, 6, "couette"),
                                          (L1, 1, 9, "bounceback"), (L1, 1, 9, "periodic")])
def test_median_filter_brute_force(lat, ny, nx, bc):
    f = rand_state(lat, ny, nx, 70, amp=0.1)
    rho, ux, uy = O.velocity(lat, f)
    q = O.equilibrium(lat, rho, ux, uy)
    dS = O.kullback_dS(f, q)
    cfg = O.Config(lattice=lat.name, nx=nx, ny=ny, bc=bc, med_delta=1e-4)
    out, acc = O.median_filter(lat, cfg, f, q, dS)
    med = _median_brute(dS.numpy(), bc == "periodic", bc in ("periodic", "couette"))
    exp_acc = (dS.numpy() > 1e-4) & (med < dS.numpy())
    assert np.array_equal(acc.numpy(), exp_acc) and exp_acc.any()
    coef = np.where(exp_acc, np.sqrt(med / dS.numpy()), 1.0)
    exp = q + torch.tensor(coef) * (f - q)
    assert torch.allclose(out, exp, atol=1e-16, rtol=0)
    dS2 = O.kullback_dS(out, q)
    assert bool((dS2 <= dS + 1e-18).all())                # dissipative only
    for a, b in zip(O.moments(lat, out), O.moments(lat, f)):
        assert torch.allclose(a, b, atol=1e-15, rtol=0)


def test_median_filter_zero_median_gradient():
    """A lone non-equilibrium site among sites at exact equilibrium has a zero
    median: the filter maps it onto f* (section 4, median entropy filter).
    Reading for gradients: none flows through the zero median (its one-sided
    derivative is infinite), so the filtered site's gradient is exactly that
    of f*(p), the transposed Jacobian of the equilibrium."""
    n = 5
    rho, ux, uy = np.ones((n, n)), np.full((n, n), 0.03), np.full((n, n), -0.02)
    f = O.init_equilibrium(L2, rho, ux, uy).clone()
    for _ in range(8):          # a floating-point fixed point of f -> f*(m(f))
        f = O.equilibrium(L2, *O.velocity(L2, f))
    f[:, 2, 2] *= 1 + torch.tensor(np.random.default_rng(71).uniform(-0.2, 0.2, 9))
    cfg = O.Config(nx=n, ny=n, bc="periodic", med_delta=1e-6)
    g = f.clone().requires_grad_(True)
    r, vx, vy = O.velocity(L2, g)
    q = O.equilibrium(L2, r, vx, vy)
    dS = O.kullback_dS(g, q)
    assert int((dS == 0).sum()) == n * n - 1
    out, acc = O.median_filter(L2, cfg, g, q, dS)
    assert bool(acc[2, 2]) and int(acc.sum()) == 1
    assert torch.allclose(out[:, 2, 2], q[:, 2, 2], atol=1e-16, rtol=0)
    w = torch.tensor(np.random.default_rng(72).normal(size=9))
    (out[:, 2, 2] * w).sum().backward()
    p = f[:, 2, 2].clone().requires_grad_(True)
    r1, vx1, vy1 = O.velocity(L2, p.view(9, 1, 1))
    (O.equilibrium(L2, r1, vx1, vy1).view(9) * w).sum().backward()
    assert bool(torch.isfinite(g.grad).all())
    assert torch.allclose(g.grad[:, 2, 2], p.grad, atol=1e-14, rtol=0)
    others = g.grad.clone()
    others[:, 2, 2] = 0
    assert float(others.abs().max()) == 0.0


# ---------------------------------------------------------------- gradient
@pytest.mark.parametrize("name", ["lbgk", "mrt_field", "elbm", "ehrenfest_pos", "median"])
def test_oracle_gradient_matches_central_differences(name):
    """The autograd (sub)gradient of a few oracle steps equals central finite
    differences of the oracle itself along a random direction."""
    n = 6
    base = dict(nx=n, ny=n, bc="periodic", nu=0.01)
    omega_field = None
    if name == "lbgk":
        cfg = O.Config(**base)
    elif name == "mrt_field":
        cfg = O.Config(**{**base, "bc": "cavity", "u_lid": 0.1}, collision="mrt")
        omega_field = torch.tensor(G.smooth_omega_field(n, n, seed=41), dtype=DT)
    elif name == "elbm":
        cfg = O.Config(**base, collision="elbm")
    elif name == "ehrenfest_pos":
        cfg = O.Config(**base, ehrenfest=True, ehr_k=4, ehr_delta=0.0, positivity=True)
    else:
        cfg = O.Config(**{**base, "bc": "cavity", "u_lid": 0.1}, median=True, med_delta=1e-6)
    kind = "entropic" if name == "elbm" else "poly"
    g0 = rand_state(L2, n, n, 80, amp=0.03, kind=kind)
    tx, ty = G.fourier_target(n, n, seed=4)
    tx, ty = torch.tensor(tx), torch.tensor(ty)

    def loss(g, om):
        g = O.run(L2, cfg, g, 3, omega_field=om)
        _, ux, uy = O.velocity(L2, g)
        return ((ux - tx) ** 2 + (uy - ty) ** 2).sum()

    g = g0.clone().requires_grad_(True)
    om = omega_field.clone().requires_grad_(True) if omega_field is not None else None
    L = loss(g, om)
    L.backward()
    rng = np.random.default_rng(81)
    dirg = torch.tensor(rng.normal(size=g0.shape))
    h = 1e-6
    with torch.no_grad():
        fd = (loss(g0 + h * dirg, omega_field) - loss(g0 - h * dirg, omega_field)) / (2 * h)
    ad = float((g.grad * dirg).sum())
    assert abs(ad - float(fd)) <= 1e-6 * abs(ad) + 1e-9
    if om is not None:
        dirw = torch.tensor(rng.normal(size=omega_field.shape))
        with torch.no_grad():
            fdw = (loss(g0, omega_field + h * dirw) - loss(g0, omega_field - h * dirw)) / (2 * h)
        adw = float((om.grad * dirw).sum())
        assert abs(adw - float(fdw)) <= 1e-6 * abs(adw) + 1e-9


# ---------------------------------------------------------------- shock tube
def test_shock_tube_runs_and_conserves_mass():
    """Section 6: 800-node tube, LBGK at nu = 1e-9 with the four sites of
    largest Delta S > 1e-3 sent to equilibrium each step; bounce-back ends
    conserve mass exactly up to rounding."""
    rho, ux, uy = G.shock_tube_1d(800)
    g = O.init_equilibrium(L1, rho, ux, uy)
    cfg = O.Config(lattice="D1Q3", nx=800, ny=1, bc="bounceback", nu=1e-9,
                   ehrenfest=True, ehr_k=4, ehr_delta=1e-3)
    m0 = O.stats(L1, g)["mass"]
    g, infos = O.run(L1, cfg, g, 400, keep_info=True)
    assert abs(O.stats(L1, g)["mass"] - m0) < 1e-10
    assert max(len(i["selected"]) for i in infos) == 4
    r, u, _ = O.velocity(L1, g)
    assert float(r.min()) > 0.4 and float(r.max()) < 1.1


# --------------------------------------------------- diffusive Maxwell wall
# Section 8, "First Hopf bifurcation": the wall re-emits, proportional to its
# equilibrium, what reached it (mass balance), and coincides with bounce-back
# in the corners.
def _edge_sites(ny, nx):
    """(ys, xs, inward normal) of the four edges without their corners."""
    X, Y = nx - 1, ny - 1
    return [(torch.full((nx - 2,), Y), torch.arange(1, X), (0, -1)),
            (torch.full((nx - 2,), 0), torch.arange(1, X), (0, 1)),
            (torch.arange(1, Y), torch.full((ny - 2,), 0), (1, 0)),
            (torch.arange(1, Y), torch.full((ny - 2,), X), (-1, 0))]


@pytest.mark.parametrize("kind", ["poly", "entropic"])
def test_diffusive_wall_no_normal_mass_flux(kind):
    """After the rule, no mass crosses any straight wall: the normal mass
    flux sum_i f_i (v_i . n) vanishes at every edge site, whatever reached
    the wall and whatever the lid speed."""
    ny, nx = 7, 9
    pre = rand_state(L2, ny, nx, 81, amp=0.3)
    out = O.diffusive_wall(L2, pre, 0.1, kind)
    vx, vy = L2.vx.view(9, 1), L2.vy.view(9, 1)
    for ys, xs, (n_x, n_y) in _edge_sites(ny, nx):
        f = out[:, ys, xs]
        flux = (f * (vx * n_x + vy * n_y)).sum(0)
        assert float(flux.abs().max()) < 1e-15
        # and the interior of the lattice is untouched
    assert torch.equal(out[:, 1:-1, 1:-1], pre[:, 1:-1, 1:-1])


@pytest.mark.parametrize("kind", ["poly", "entropic"])
def test_diffusive_wall_reemits_its_maxwellian(kind):
    """If what reaches a wall is the wall's own equilibrium at some density
    rho' (moving with the wall), the wall sends back exactly that
    equilibrium: on the lid the tangential lid velocity is carried by the
    emitted S, SW, SE populations."""
    ny, nx, u_lid = 6, 8, 0.1
    rng = np.random.default_rng(5)
    pre = rand_state(L2, ny, nx, 82, amp=0.3)
    dens = torch.tensor(0.7 + 0.6 * rng.uniform(size=(ny, nx)), dtype=DT)
    for ys, xs, (n_x, n_y) in _edge_sites(ny, nx):
        u = u_lid if (n_x, n_y) == (0, -1) else 0.0
        feq = O.equilibrium(L2, dens[ys, xs], torch.full_like(dens[ys, xs], u),
                            torch.zeros_like(dens[ys, xs]), kind)
        for i, (a, b) in enumerate(L2.vel):
            if a * n_x + b * n_y < 0:          # reaches the wall
                pre[i, ys, xs] = feq[i]
    out = O.diffusive_wall(L2, pre, u_lid, kind)
    for ys, xs, (n_x, n_y) in _edge_sites(ny, nx):
        u = u_lid if (n_x, n_y) == (0, -1) else 0.0
        feq = O.equilibrium(L2, dens[ys, xs], torch.full_like(dens[ys, xs], u),
                            torch.zeros_like(dens[ys, xs]), kind)
        for i, (a, b) in enumerate(L2.vel):
            if a * n_x + b * n_y > 0:          # emitted into the fluid
                assert torch.allclose(out[i, ys, xs], feq[i], rtol=1e-14, atol=0)


def test_diffusive_wall_is_bounce_back_in_the_corners():
    ny, nx = 5, 6
    pre = rand_state(L2, ny, nx, 83, amp=0.4)
    out = O.diffusive_wall(L2, pre, 0.1, "entropic")
    idx = {v: i for i, v in enumerate(L2.vel)}
    for (y, x, n) in [(0, 0, (1, 1)), (0, nx - 1, (-1, 1)), (ny - 1, 0, (1, -1)),
                      (ny - 1, nx - 1, (-1, -1))]:
        i_in, i_out = idx[n], idx[(-n[0], -n[1])]
        assert float(out[i_in, y, x]) == float(pre[i_out, y, x])


@pytest.mark.parametrize("collision,kind", [("lbgk", "poly"), ("lbgk", "entropic"),
                                            ("elbm", "entropic"), ("mrt", "poly")])
def test_diffusive_cavity_at_rest_is_a_fixed_point(collision, kind):
    """A uniform equilibrium at rest inside resting diffusive walls is a
    fixed point of the whole step (streaming, wall rule, collision)."""
    ny, nx = 6, 7
    cfg = O.Config(nx=nx, ny=ny, bc="diffusive", u_lid=0.0, collision=collision,
                   equilibrium=kind, nu=0.01, median=True, med_delta=1e-12)
    rho = torch.full((ny, nx), 1.3, dtype=DT)
    z = torch.zeros((ny, nx), dtype=DT)
    f = O.equilibrium(L2, rho, z, z, "entropic" if collision == "elbm" else kind)
    g, info = O.step(L2, cfg, f)
    assert torch.allclose(g, f, rtol=2e-15, atol=0)
    assert not bool(info["median_mask"].any())


def test_diffusive_wall_sites_do_not_collide():
    """Wall sites keep the streamed state after the rule, and the fluid
    sites take a plain LBGK collision of the same streamed state."""
    ny, nx = 6, 8
    cfg = O.Config(nx=nx, ny=ny, bc="diffusive", u_lid=0.1, collision="lbgk", nu=0.02)
    f = rand_state(L2, ny, nx, 84, amp=0.2)
    g, _ = O.step(L2, cfg, f)
    pre = O.diffusive_wall(L2, O.stream(L2, f, "diffusive"), 0.1, "poly")
    wall = O.wall_nodes(ny, nx)
    assert torch.equal(g[:, wall], pre[:, wall])
    r, jx, jy = O.moments(L2, pre)
    feq = O.equilibrium(L2, r, jx / r, jy / r)
    post = O.lbgk(pre, feq, O.relaxation_rate(cfg))
    assert torch.allclose(g[:, ~wall], post[:, ~wall], rtol=1e-15, atol=1e-17)


def test_median_filter_excludes_diffusive_walls():
    ny, nx = 6, 7
    f = rand_state(L2, ny, nx, 85, amp=0.1)
    rho, ux, uy = O.velocity(L2, f)
    q = O.equilibrium(L2, rho, ux, uy)
    dS = O.kullback_dS(f, q)
    wall = O.wall_nodes(ny, nx)
    cfg = O.Config(nx=nx, ny=ny, bc="diffusive", med_delta=1e-5)
    out, acc = O.median_filter(L2, cfg, f, q, dS, wall)
    d = dS.numpy()
    for y in range(1, ny - 1):
        for x in range(1, nx - 1):
            vals = sorted(d[yy, xx] for yy in (y - 1, y, y + 1) for xx in (x - 1, x, x + 1)
                          if 0 < yy < ny - 1 and 0 < xx < nx - 1)
            med = vals[(len(vals) + 1) // 2 - 1]
            assert bool(acc[y, x]) == bool(d[y, x] > 1e-5 and med < d[y, x])
    assert not bool(acc[wall].any())


def test_hopf_energy_of_a_sine():
    """E_u (eq. energy) of whole periods of A sin: the mean is 0 and the
    squares average A^2/2, so E_u = A sqrt(L / (2 u0))."""
    n, A, L, u0 = 4000, 0.013, 100.0, 0.1
    s = 0.2 + A * np.sin(2 * np.pi * 7 * np.arange(n) / n)
    assert abs(O.hopf_energy(s, L, u0) - A * math.sqrt(L / (2 * u0))) < 1e-13


def test_enstrophy_of_rigid_rotation():
    """Rigid rotation u = Omega (-(y - yc), x - xc) has vorticity 2 Omega,
    which central differences reproduce exactly: enstrophy 4 Omega^2."""
    ny, nx, om = 9, 11, 3e-3
    ys, xs = np.mgrid[0:ny, 0:nx].astype(float)
    ux = -om * (ys - 4.0)
    uy = om * (xs - 5.0)
    f = O.init_equilibrium(L2, np.ones((ny, nx)), ux, uy)
    assert abs(O.enstrophy(L2, f, "diffusive") - 4 * om * om) < 1e-18
