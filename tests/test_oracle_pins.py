"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test names the passage it follows.  None compares the oracle with
itself: closed forms, invariants, special cases reducing to textbook results
and brute force between the two independent oracle tiers.
"""

import dataclasses
import math
import os

import numpy as np
import pytest
import scipy.special

import synth
from oracle import o1_dense as o1

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
rng0 = np.random.default_rng(1234)


def _random_states(n=40, du=0.1, df=1e-2, seed=0):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.9, 1.1, n)
    u = rng.uniform(-du, du, (n, 3))
    f = o1.equilibrium_product(rho, u) + rng.normal(0.0, df, (n, 27))
    return f


# ---- lattice ------------------------------------------------------------------

def test_weights_match_textbook_golden():
    """D3Q27 weights (golden file, textbook values) and the lattice isotropy
    sums sum w = 1, sum w c c = cs^2 I that Eq. (3) relies on."""
    table = {}
    with open(os.path.join(GOLDEN, "d3q27_weights.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, c2, count, w = line.split()
            num, den = w.split("/")
            table[int(c2)] = (int(count), float(num) / float(den))
    c2 = (o1.C ** 2).sum(axis=1)
    for k, (count, w) in table.items():
        assert np.count_nonzero(c2 == k) == count
        assert np.allclose(o1.W[c2 == k], w, rtol=0, atol=1e-16)
    assert abs(o1.W.sum() - 1.0) < 1e-15
    second = np.einsum("a,ai,aj->ij", o1.W, o1.C, o1.C)
    assert np.allclose(second, np.eye(3) / 3.0, atol=1e-16)
    assert all(np.array_equal(o1.C[o1.OPP[a]], -o1.C[a]) for a in range(27))


# ---- P1-P5: closed forms and invariants of Eqs. (3), (6)-(8) -----------------------

def test_P1_series_equilibrium_equals_product_form():
    """Eq. (3) with the full D3Q27 expansion (Sec. 2.1.3) equals the product of
    one-dimensional factors."""
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.8, 1.2, 64)
    u = rng.uniform(-0.2, 0.2, (64, 3))
    a = o1.equilibrium_series(rho, u)
    b = o1.equilibrium_product(rho, u)
    assert np.max(np.abs(a - b)) < 1e-14


def test_P1b_equilibrium_moments():
    """The equilibrium reproduces rho and rho u (Eqs. (4)-(5))."""
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.8, 1.2, 16)
    u = rng.uniform(-0.2, 0.2, (16, 3))
    feq = o1.equilibrium_series(rho, u)
    assert np.allclose(feq.sum(axis=1), rho, atol=1e-14, rtol=0)
    assert np.allclose(feq @ o1.C, rho[:, None] * u, atol=1e-14, rtol=0)


def test_P2_central_moments_of_equilibrium():
    """T f_eq = (rho, 0, ..., 0): Eqs. (7)-(8a,b)."""
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.8, 1.2, 32)
    u = rng.uniform(-0.2, 0.2, (32, 3))
    m = np.einsum("nma,na->nm", o1.central_transform(u), o1.equilibrium_series(rho, u))
    assert np.max(np.abs(m[:, 0] - rho)) < 1e-14
    assert np.max(np.abs(m[:, 1:])) < 1e-14


def test_P2b_second_order_second_rate_only_changes_viscous_moments():
    """Only the six second-order rows carry s2 (Sec. 2.1.3): with every other rate
    equal to 1 and s2 = 1, the post-collision central moments vanish except
    order 0 (rho) and order 1 (rho g / 2, the forcing reading)."""
    f = _random_states(8)
    g = (1e-4, -2e-4, 3e-4)
    fp, rho, _, u = o1.collide(f, 1.0, (1.0, 1.0, 1.0, 1.0), g)
    m = np.einsum("nma,na->nm", o1.central_transform(u), fp)
    assert np.allclose(m[:, 0], rho, atol=1e-14)
    for d, idx in enumerate((1, 3, 9)):
        assert np.allclose(m[:, idx], 0.5 * rho * g[d], atol=1e-15)
    rest = [k for k in range(27) if k not in (0, 1, 3, 9)]
    assert np.max(np.abs(m[:, rest])) < 1e-14


def test_P3_transform_invertible_and_factored_equals_dense(o2lib):
    """T is invertible for any u, and the factored per-axis transforms of tier O2
    give the same collision as the dense linear solve of tier O1."""
    rng = np.random.default_rng(4)
    u = rng.uniform(-0.3, 0.3, (16, 3))
    T = o1.central_transform(u)
    assert np.min(np.abs(np.linalg.det(T))) > 1e-6
    case = synth.periodic_box_case(4, 2, 2, tau=0.7, g=(1e-4, 2e-4, -1e-4),
                                   rates=(1.3, 0.7, 1.6, 1.1))
    sim = o2lib.O2Sim(case, nthreads=1)
    f = _random_states(sim.n, seed=5)
    sim.f[...] = f
    sim.collide()
    fp, _, _, _ = o1.collide(f, case.tau, case.rates, case.g)
    assert np.max(np.abs(sim.fpost - fp)) < 1e-14


def test_P4_equal_rates_reduce_to_bgk(o2lib):
    """All rates equal to 1/tau: CHM-MRT becomes the BGK operator of Eq. (2),
    in both oracle tiers."""
    f = _random_states(32, seed=6)
    tau = 0.73
    fp, rho, _, u = o1.collide(f, tau, (1 / tau,) * 4, (0.0, 0.0, 0.0))
    feq = o1.equilibrium_product(rho, u)
    bgk = f + (feq - f) / tau
    assert np.max(np.abs(fp - bgk)) < 1e-14
    case = synth.periodic_box_case(4, 4, 2, tau=tau, rates=(1 / tau,) * 4)
    sim = o2lib.O2Sim(case, nthreads=1)
    sim.f[...] = f
    sim.collide()
    assert np.max(np.abs(sim.fpost - bgk)) < 1e-14


def test_P5_collision_conserves_mass_and_adds_rho_g():
    """sum f* = sum f and sum c f* = sum c f + rho g (forcing reading)."""
    f = _random_states(32, seed=7)
    g = np.array([3e-4, -1e-4, 2e-4])
    fp, rho, j, _ = o1.collide(f, 0.9, (1.2, 0.8, 1.5, 0.6), g)
    assert np.max(np.abs(fp.sum(1) - f.sum(1))) < 1e-14
    assert np.max(np.abs(fp @ o1.C - (j + rho[:, None] * g[None, :]))) < 1e-14


# ---- P6-P9: whole-step invariants ------------------------------------------------

def _closed_random_case(seed):
    case = synth.random_tiny_case(seed)
    case.mask[case.mask >= 2] = synth.SOLID
    case.inlet = None
    return case


@pytest.mark.parametrize("seed", [0, 1])
def test_P6_rest_state_is_bitwise_fixed_point(o2lib, seed):
    """With g = 0 the rest equilibrium f = w is unchanged by collision,
    bounce-back and periodic streaming (to FP64 rounding of the unshifted
    oracle arithmetic)."""
    case = _closed_random_case(seed)
    case.g = (0.0, 0.0, 0.0)
    sim = o2lib.O2Sim(case, nthreads=1)
    f0 = sim.f.copy()
    sim.run(5)
    assert np.max(np.abs(sim.f - f0)) < 1e-16
    st = o1.run(case, 3)
    fl = st.fluid
    assert np.max(np.abs(st.f[fl[:, 0], fl[:, 1], fl[:, 2]] - o1.W[None, :])) < 1e-15


def test_P6b_uniform_flow_in_periodic_box_is_fixed_point(o2lib):
    case = synth.periodic_box_case(5, 4, 3, tau=0.6, rates=(1.1, 0.9, 1.4, 0.7))
    sim = o2lib.O2Sim(case, nthreads=1)
    u = np.tile([[0.05, -0.03, 0.02]], (sim.n, 1))
    sim.f[...] = o1.equilibrium_product(np.ones(sim.n), u)
    f0 = sim.f.copy()
    sim.run(10)
    assert np.max(np.abs(sim.f - f0)) < 1e-15


@pytest.mark.parametrize("seed", [2, 3])
def test_P7_zero_rates_make_a_step_a_permutation(o2lib, seed):
    """With every rate of order >= 2 set to 0 and g = 0 the collision is the
    identity, so a step only permutes the population values (streaming and
    bounce-back, Eqs. (1) and (9)); sorted values agree to FP64 rounding (rho ~ 13 here) while
    distinct values are ~1e-4 apart."""
    case = _closed_random_case(seed)
    case.g = (0.0, 0.0, 0.0)
    sim = o2lib.O2Sim(case, nthreads=1, rates5=(0.0,) * 5)
    rng = np.random.default_rng(seed)
    sim.f[...] = rng.random((sim.n, 27))
    before = np.sort(sim.f.ravel())
    sim.run(3)
    assert np.max(np.abs(np.sort(sim.f.ravel()) - before)) < 1e-13


def test_P8_pipe_mass_conserved_2000_steps(o2lib):
    """Closed periodic pipe (64x24x24, R = 10, g = 1e-6, tau = 0.8): mass is
    conserved over 2000 steps (collision conserves mass, halfway bounce-back
    returns every population).  The bound is FP64 rounding of the unshifted
    oracle arithmetic, about 1e-16 per node update over 4e7 updates."""
    case = synth.pipe_case()
    sim = o2lib.O2Sim(case, nthreads=8)
    m0 = sim.f.sum()
    mon = sim.run(2000)
    assert sim.n == 20224
    assert abs(mon[0] - m0) / m0 < 1e-12


@pytest.mark.parametrize("seed", [0, 4, 5])
def test_P8b_open_system_mass_balance(o2lib, seed):
    """With inlet and outlet ghosts, M(t+1) - M(t) equals the boundary flux of
    that step exactly (to rounding), in both tiers."""
    case = synth.random_tiny_case(seed)
    sim = o2lib.O2Sim(case, nthreads=1)
    st = o1.O1State(case)
    m_prev = sim.f.sum()
    for _ in range(10):
        mon = sim.run(1)
        assert abs(mon[0] - m_prev - (mon[7] + mon[8])) < 1e-13 * mon[0]
        m_prev = mon[0]
        mprev1 = st.f.sum()
        o1.step(st)
        assert abs(st.monitors[0] - mprev1 - (st.monitors[7] + st.monitors[8])) < 1e-13 * mprev1


def test_P9_periodic_box_momentum_grows_as_M_g_t(o2lib):
    case = synth.periodic_box_case(6, 5, 4, tau=0.9, g=(2e-5, -1e-5, 3e-5),
                                   rates=(1.2, 0.8, 1.5, 1.7))
    sim = o2lib.O2Sim(case, nthreads=2)
    for t in (7, 50):
        mon = sim.run(t - sim.t)
        expect = mon[0] * np.asarray(case.g) * t
        assert np.max(np.abs(mon[1:4] - expect)) < 1e-12 * np.max(np.abs(expect)) + 1e-16


# ---- P10-P13: closed-form flows ---------------------------------------------------

def _shear_rate_error(o2lib, L, tau, rates):
    case = synth.periodic_box_case(4, L, 1, tau=tau, rates=rates)
    sim = o2lib.O2Sim(case, nthreads=4)
    y = sim.coords[:, 1]
    shape = np.sin(2 * np.pi * y / L)
    u0 = np.zeros((sim.n, 3))
    u0[:, 0] = 1e-3 * shape
    sim.f[...] = o1.equilibrium_product(np.ones(sim.n), u0)
    amps = []
    t1, t2 = (L * L) // 10, (3 * L * L) // 10
    for t in (t1, t2):
        sim.run(t - sim.t)
        _, u = sim.macroscopic()
        amps.append((u[:, 0] * shape).sum() / (shape * shape).sum())
    rate = -math.log(amps[1] / amps[0]) / (t2 - t1)
    return rate / (case.nu * (2 * math.pi / L) ** 2) - 1.0


def test_P10_shear_wave_decays_at_viscous_rate(o2lib):
    """A sinusoidal shear wave decays as exp(-nu k^2 t) with nu = (tau - 1/2)/3,
    which ties the second-order rate 1/tau to the viscosity (Sec. 2.1.3).  The
    relative rate error is a truncation error of order k^2: small at L = 32 and
    about four times smaller at L = 64."""
    for tau, rates in ((0.8, (1.0,) * 4), (0.6, (1.4, 0.9, 1.2, 1.0))):
        e32 = _shear_rate_error(o2lib, 32, tau, rates)
        e64 = _shear_rate_error(o2lib, 64, tau, rates)
        assert abs(e32) < 5e-3
        assert abs(e64) < abs(e32) / 3.0


def _poiseuille_startup(r, t, R, nu, g):
    lam = scipy.special.jn_zeros(0, 60)
    u = g * (R * R - r * r) / (4 * nu)
    for l in lam:
        u = u - 2 * g * R * R / nu * scipy.special.j0(l * r / R) / (l ** 3 * scipy.special.j1(l)) \
            * np.exp(-l * l * nu * t / (R * R))
    return u


def _pipe_error(o2lib, R, steps, nx=4):
    n = int(2 * R + 4)
    c = synth.pipe_case(nx=nx, ny=n, nz=n, radius=R, center=((n - 1) / 2, (n - 1) / 2))
    sim = o2lib.O2Sim(c, nthreads=8)
    sim.run(steps)
    _, u = sim.macroscopic()
    y = sim.coords[:, 1] - (n - 1) / 2
    z = sim.coords[:, 2] - (n - 1) / 2
    ua = _poiseuille_startup(np.sqrt(y * y + z * z), steps, R, c.nu, 1e-6)
    return np.sqrt(((u[:, 0] - ua) ** 2).sum() / (ua ** 2).sum()), np.abs(u[:, 1:]).max()


def test_P11_pipe_poiseuille_and_staircase_trend(o2lib):
    """Config-1 pipe against the Poiseuille start-up series: a few per cent L2
    error from the staircase wall at R = 10, shrinking at least as 1/R at R = 20."""
    e10, cross10 = _pipe_error(o2lib, 10, 2000)
    e20, _ = _pipe_error(o2lib, 20, 8000)
    assert e10 < 0.05
    assert e20 < e10 / 2.0
    assert cross10 < 1e-14


def test_P13_womersley_pipe(o2lib):
    """Periodic pipe driven by g(t) = g0 + g1 cos(omega t) at Womersley number 3
    (the paper's pulsatile case has Wo = 2.54, Sec. 2.2.2): after five periods
    the profile follows the Womersley closed form to the staircase error."""
    R, n, tau = 10.0, 24, 0.8
    nu = (tau - 0.5) / 3
    w = 9.0 * nu / R ** 2
    g0 = g1 = 1e-6
    c = synth.pipe_case(nx=4, ny=n, nz=n, radius=R, center=((n - 1) / 2, (n - 1) / 2), g=g0, tau=tau)
    sim = o2lib.O2Sim(c, nthreads=8, g_time=((g0, 0, 0), (g1, 0, 0), w))
    period = 2 * math.pi / w
    sim.run(int(round(5 * period)))
    y = sim.coords[:, 1] - (n - 1) / 2
    z = sim.coords[:, 2] - (n - 1) / 2
    r = np.sqrt(y * y + z * z)
    worst = 0.0
    for _ in range(8):
        sim.run(int(round(period / 8)))
        t = sim.t
        _, u = sim.macroscopic(g=(g0 + g1 * math.cos(w * t), 0, 0))
        ua = o1.womersley_speed(r, t, R, nu, g0, g1, w)
        worst = max(worst, math.sqrt(((u[:, 0] - ua) ** 2).sum() / (ua ** 2).sum()))
    assert worst < 0.06


def test_womersley_profile_solves_its_ode():
    """The inlet profile solves i w U = G1 + nu (U'' + U'/r) for its oscillating
    part, vanishes at the wall and reduces to Poiseuille for w = 0."""
    R, nu, w, G1 = 12.0, 0.025, 2 * math.pi / 4000, 2e-5
    r = np.linspace(0.5, R - 0.5, 200)
    h = 1e-3
    # complex amplitude = value at t=0 minus i * value at a quarter period
    def amp(rr):
        a = o1.womersley_speed(rr, 0.0, R, nu, 0.0, G1, w)
        b = o1.womersley_speed(rr, math.pi / (2 * w), R, nu, 0.0, G1, w)
        return a - 1j * b
    U = amp(r)
    d2 = (amp(r + h) - 2 * U + amp(r - h)) / h ** 2
    d1 = (amp(r + h) - amp(r - h)) / (2 * h)
    res = 1j * w * U - G1 - nu * (d2 + d1 / r)
    assert np.max(np.abs(res)) < 1e-6 * G1 + 1e-12
    assert abs(amp(np.array([R - 1e-9]))[0]) < 1e-9
    steady = o1.womersley_speed(r, 0.0, R, nu, 3e-5, 0.0, 0.0)
    assert np.allclose(steady, 3e-5 * (R * R - r * r) / (4 * nu), rtol=1e-14)


def test_oracle_bessel_series_matches_scipy(o2lib):
    """Tier O2 evaluates J0 by its power series; tier O1 uses scipy.  Their inlet
    velocities agree (checked through one streaming step with only inlet links)."""
    case = synth.random_tiny_case(11)
    sim = o2lib.O2Sim(case, nthreads=1)
    st = o1.O1State(case)
    for _ in range(3):
        sim.run(1)
        o1.step(st)
    fl = st.fluid
    assert np.max(np.abs(st.f[fl[:, 0], fl[:, 1], fl[:, 2]] - sim.f)) < 1e-14


# ---- P14: acoustic scaling --------------------------------------------------------

def test_P14_acoustic_scaling_matches_paper_pair():
    """Sec. 2.2.3 prints tau = 0.506 (dx 1e-4, dt 5e-6) and 0.503 (dx 2e-4,
    dt 1e-5): tau - 1/2 halves when dx and dt double.  The aneurysm cases follow
    the same rule between 128^3, 256^3 and 512^3."""
    vals = {}
    with open(os.path.join(GOLDEN, "acoustic_scaling.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    assert vals["coarse_dt"] / vals["fine_dt"] == vals["coarse_dx"] / vals["fine_dx"] == 2.0
    assert abs((vals["coarse_tau"] - 0.5) - (vals["fine_tau"] - 0.5) / 2) < 1e-12
    taus = {}
    for n in (128, 256):
        c = synth.aneurysm_case(n, seed=0)
        taus[n] = c.tau
    taus[512] = 0.5 + 2 * (taus[256] - 0.5)
    assert abs((taus[128] - 0.5) - (taus[256] - 0.5) / 2) < 1e-15
    assert abs(taus[256] - 0.575398) < 1e-6


# ---- P15: brute force between the tiers -------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_P15_dense_and_factored_oracles_agree(o2lib, seed):
    """Tiny random masks with walls, periodic axes, inlet and outlet ghosts,
    random rates, force and inlet: O1 (dense definition) == O2 (factored)."""
    case = synth.random_tiny_case(seed)
    st = o1.run(case, 20)
    sim = o2lib.O2Sim(case, nthreads=2)
    sim.run(20)
    fl = st.fluid
    assert np.max(np.abs(st.f[fl[:, 0], fl[:, 1], fl[:, 2]] - sim.f)) < 1e-13
    assert np.max(np.abs(st.monitors - sim.monitors)) < 1e-12


def test_oracle_catches_planted_mistakes(o2lib, monkeypatch):
    """A dropped forcing term or a wrong order-to-rate assignment changes the
    result far above rounding, so the brute-force pin P15 would catch it
    (planted in tier O1, on the CPU)."""
    case = synth.random_tiny_case(0)
    ref = o1.run(case, 5).f.copy()
    # 1) drop the (I - S/2) F forcing term
    orig = o1.collide

    def no_force(f, tau, rates, g):
        return orig(f, tau, rates, (0.0, 0.0, 0.0))
    monkeypatch.setattr(o1, "collide", no_force)
    bad = o1.run(case, 5).f
    monkeypatch.setattr(o1, "collide", orig)
    assert np.max(np.abs(bad - ref)) > 1e-8
    # 2) wrong order -> rate assignment (swap orders 3 and 4)
    orig_rates = o1.relaxation_rates

    def swapped(tau, rates):
        r = list(rates)
        r[0], r[1] = r[1], r[0]
        return orig_rates(tau, r)
    monkeypatch.setattr(o1, "relaxation_rates", swapped)
    bad = o1.run(case, 5).f
    monkeypatch.setattr(o1, "relaxation_rates", orig_rates)
    assert np.max(np.abs(bad - ref)) > 1e-8


# ---------------------------------------------------------------------------
# Curved walls (Sec. 2.1.4, Eq. (9)-(10)): linear interpolated bounce-back
# ---------------------------------------------------------------------------

def _wall_q_map(links, q):
    return {tuple(int(v) for v in lk): float(qq) for lk, qq in zip(links, q)}


@pytest.mark.parametrize("seed", [0, 1, 3])
def test_P16_curved_walls_at_half_equal_halfway_bounce_back(o2lib, seed):
    """q = 1/2 on every wall link is halfway bounce-back (both branches of
    Eq. (9) reduce to it): identical populations and monitors, bit for bit."""
    case = synth.random_tiny_case(seed)
    links = synth.wall_links(case.mask, case.periodic)
    assert len(links) > 0
    a = o2lib.O2Sim(case, nthreads=2)
    b = o2lib.O2Sim(case, nthreads=2, wall_q=_wall_q_map(links, np.full(len(links), 0.5)))
    ma, mb = a.run(15).copy(), b.run(15).copy()
    assert np.array_equal(a.f, b.f)
    assert np.array_equal(ma, mb)


def _pipe_error_curved(o2lib, R, curved):
    """L2 error of the axial velocity against the Poiseuille start-up series
    after 20 R^2 steps (diffusive scaling), pipe axis off the lattice."""
    n = int(2 * R + 4)
    c = synth.pipe_case(nx=4, ny=n, nz=n, radius=R, center=((n - 1) / 2 + 0.3, (n - 1) / 2 - 0.2))
    wq = None
    if curved:
        links = synth.wall_links(c.mask, c.periodic)
        wq = _wall_q_map(links, synth.wall_distances(c, links))
    steps = int(20 * R * R)
    sim = o2lib.O2Sim(c, nthreads=8, wall_q=wq)
    sim.run(steps)
    _, u = sim.macroscopic()
    cy, cz = c.meta["center"]
    y, z = sim.coords[:, 1] - cy, sim.coords[:, 2] - cz
    ua = _poiseuille_startup(np.sqrt(y * y + z * z), steps, R, c.nu, 1e-6)
    return math.sqrt(((u[:, 0] - ua) ** 2).sum() / (ua ** 2).sum())


def test_P17_curved_walls_converge_at_second_order(o2lib):
    """Pipe Poiseuille with the exact wall distance of the circular wall: the
    error falls by about 4 per halving of the grid spacing (second order),
    against about 2 for halfway bounce-back on the staircase (first order)."""
    e = {R: _pipe_error_curved(o2lib, R, True) for R in (5, 10, 20)}
    h = {R: _pipe_error_curved(o2lib, R, False) for R in (5, 10, 20)}
    assert e[5] / e[10] > 3.5 and e[10] / e[20] > 3.5
    assert h[5] / h[10] < 2.8 and h[10] / h[20] < 2.8
    assert e[20] < 1e-3 < h[20]


# ---------------------------------------------------------------------------
# SRT comparator (Sec. 2.1.1-2.1.2): BGK with the second-order EDF
# ---------------------------------------------------------------------------

def test_P18_second_order_edf_and_force_moments():
    """The truncated EDF keeps exactly the moments it is built to match --
    rho, rho u and rho (u u + cs^2 I) -- and Guo's force populations carry no
    mass, momentum rho g and second moment rho (u g + g u)."""
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.9, 1.1, 50)
    u = rng.uniform(-0.08, 0.08, (50, 3))
    g = np.array([2e-4, -1e-4, 3e-4])
    feq = o1.equilibrium_second_order(rho, u)
    Cf = o1.C.astype(np.float64)
    assert np.allclose(feq.sum(1), rho, rtol=0, atol=1e-15)
    assert np.allclose(feq @ Cf, rho[:, None] * u, rtol=0, atol=1e-15)
    P = np.einsum("na,ai,aj->nij", feq, Cf, Cf)
    assert np.allclose(P, rho[:, None, None] * (u[:, :, None] * u[:, None, :] + np.eye(3) / 3.0), rtol=0, atol=1e-15)
    # it differs from the full expansion only at third order in u
    full = o1.equilibrium_product(rho, u)
    d1 = np.abs(full - feq).max()
    d2 = np.abs(o1.equilibrium_product(rho, u / 2) - o1.equilibrium_second_order(rho, u / 2)).max()
    assert 6.0 < d1 / d2 < 10.0
    F = o1.guo_force(rho, u, g)
    assert np.allclose(F.sum(1), 0.0, atol=1e-18)
    assert np.allclose(F @ Cf, rho[:, None] * g[None, :], rtol=0, atol=1e-18)
    S = np.einsum("na,ai,aj->nij", F, Cf, Cf)
    ug = u[:, :, None] * g[None, None, :]
    assert np.allclose(S, rho[:, None, None] * (ug + ug.transpose(0, 2, 1)), rtol=0, atol=1e-18)


def _srt(case):
    return dataclasses.replace(case, collision="srt2")


def test_P19_srt_shear_wave_and_momentum(o2lib):
    """SRT with the second-order EDF: a shear wave decays at nu = (tau - 1/2)/3
    (truncation error of order k^2), and a periodic box gains M g per step."""
    def rate_error(L, tau):
        case = _srt(synth.periodic_box_case(4, L, 1, tau=tau))
        sim = o2lib.O2Sim(case, nthreads=4)
        y = sim.coords[:, 1]
        shape = np.sin(2 * np.pi * y / L)
        u0 = np.zeros((sim.n, 3))
        u0[:, 0] = 1e-3 * shape
        sim.f[...] = o1.equilibrium_second_order(np.ones(sim.n), u0)
        amps = []
        t1, t2 = (L * L) // 10, (3 * L * L) // 10
        for t in (t1, t2):
            sim.run(t - sim.t)
            _, u = sim.macroscopic()
            amps.append((u[:, 0] * shape).sum() / (shape * shape).sum())
        rate = -math.log(amps[1] / amps[0]) / (t2 - t1)
        return rate / (case.nu * (2 * math.pi / L) ** 2) - 1.0
    for tau in (0.8, 0.6):
        e32, e64 = rate_error(32, tau), rate_error(64, tau)
        assert abs(e32) < 5e-3 and abs(e64) < abs(e32) / 3.0
    case = _srt(synth.periodic_box_case(6, 5, 4, tau=0.9, g=(2e-5, -1e-5, 3e-5)))
    sim = o2lib.O2Sim(case, nthreads=2)
    for t in (7, 50):
        mon = sim.run(t - sim.t)
        expect = mon[0] * np.asarray(case.g) * t
        assert np.max(np.abs(mon[1:4] - expect)) < 1e-12 * np.max(np.abs(expect)) + 1e-16
        assert abs(mon[0] - sim.n) < 1e-11


@pytest.mark.parametrize("seed", range(4))
def test_P20_srt_dense_and_fast_oracles_agree(o2lib, seed):
    """Tiny random masks (walls, periodic axes, inlet and outlet ghosts, force):
    the dense SRT collision of O1 equals the one of O2."""
    case = _srt(synth.random_tiny_case(seed))
    st = o1.run(case, 20)
    sim = o2lib.O2Sim(case, nthreads=2)
    sim.run(20)
    fl = st.fluid
    assert np.max(np.abs(st.f[fl[:, 0], fl[:, 1], fl[:, 2]] - sim.f)) < 1e-13
    assert np.max(np.abs(st.monitors - sim.monitors)) < 1e-12


# ---------------------------------------------------------------------------
# P12: wall position of halfway bounce-back (Sec. 2.1.2-2.1.3)
# ---------------------------------------------------------------------------

def _channel_error(o2lib, tau, s3, H=8, g=1e-6):
    c = dataclasses.replace(synth.channel_case(4, H + 2, 2, tau, g), rates=(s3, 1.0, 1.0, 1.0))
    nu = c.nu
    sim = o2lib.O2Sim(c, nthreads=4)
    sim.run(int(40 * H * H / nu))
    _, u = sim.macroscopic()
    y = sim.coords[:, 1].astype(float)
    ua = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y)      # walls halfway between nodes
    return float(np.abs(u[:, 0] - ua).max() / ua.max())


def test_P12_free_third_order_rate_fixes_the_wall_position(o2lib):
    """With SRT-like rates the halfway wall sits at a tau-dependent place, the
    shortcoming Sec. 2.1.2 recalls; CHM-MRT's free rates give the degree of
    freedom to fix it (Sec. 2.1.3).  With (1/s2 - 1/2)(1/s3 - 1/2) = 3/16
    steady channel Poiseuille flow is exact to rounding for every tau, while
    s3 = 1 leaves a tau-dependent slip error."""
    for tau in (0.6, 0.9, 1.5):
        s3 = 1.0 / (0.5 + 0.1875 / (tau - 0.5))
        assert _channel_error(o2lib, tau, s3) < 1e-9
        assert _channel_error(o2lib, tau, 1.0) > 5e-4


# ---------------------------------------------------------------------------
# Open boundaries (Sec. 2.1.2: the bounce-back family enforces velocity and
# pressure conditions; Sec. 2.2.1: constant inflow, open outflow) and the wall
# force.  Readings C8 (moving-wall bounce-back), C9 (anti-bounce-back) and the
# momentum-exchange wall force, pinned against their textbook forms and against
# a steady open pipe.
# ---------------------------------------------------------------------------

def _one_node_case(kind, rho_out=1.0, u_max=0.05):
    """One fluid node at (1, 1, 1) of a 3^3 box whose x = 0 face is made of
    ghost cells of the given kind (inlet: steady Poiseuille profile along +x
    with its axis through (y, z) = (1, 1), radius 10)."""
    mask = np.zeros((3, 3, 3), np.uint8)
    mask[1, 1, 1] = synth.FLUID
    mask[:, :, 0] = kind
    R, tau = 10.0, 0.8
    nu = (tau - 0.5) / 3.0
    inlet = synth.geometry.Inlet(axis=(1.0, 0.0, 0.0), center=(0.0, 1.0, 1.0), radius=R,
                                 G0=4.0 * nu * u_max / (R * R), G1=0.0, omega=0.0)
    return synth.Case(name=f"onenode{kind}", mask=mask, tau=tau, rho_out=rho_out, inlet=inlet), R, nu


def _boundary_step(tier, case, fpost, u, o2lib=None):
    """Populations arriving at the single node after streaming fpost [27]."""
    if tier == "o1":
        st = o1.O1State(case)
        new, _, _, _ = o1.stream(st, fpost[None, :], u[None, :])
        return new[1, 1, 1]
    sim = o2lib.O2Sim(case, nthreads=1)
    sim.stream_from_post(fpost[None, :], u[None, :], 0)
    return sim.f[0]


def _inlet_rule_error(tier, o2lib=None):
    """Largest deviation of the inlet rule from Ladd's moving-wall bounce-back,
    f_abar(x, t+1) = f*_a(x, t) - 2 w_a rho0 (c_a . u_w) / cs^2 for the link in
    direction a into the wall, u_w the Poiseuille velocity at the link midpoint.
    For u_w along a lattice axis the full-expansion equilibria give exactly
    this (their difference has no higher-order terms), so the pin is sharp."""
    case, R, nu = _one_node_case(synth.INLET)
    rng = np.random.default_rng(3)
    fpost = o1.W * (1.0 + rng.uniform(-0.1, 0.1, 27))
    new = _boundary_step(tier, case, fpost, np.zeros(3), o2lib)
    err = 0.0
    for a in range(27):
        c = o1.C[a]
        if c[0] != -1:
            continue
        r = 0.5 * math.hypot(c[1], c[2])              # midpoint (0.5, 1 + cy/2, 1 + cz/2) from the axis
        U = case.inlet.G0 * (R * R - r * r) / (4.0 * nu)
        ladd = fpost[a] - 2.0 * o1.W[a] * 1.0 * (c[0] * U) / o1.CS2
        err = max(err, abs(new[o1.OPP[a]] - ladd))
    return err


def _outlet_rule_error(tier, o2lib=None):
    """Largest deviation of the outlet rule from the anti-bounce-back pressure
    condition with the second-order equilibrium's even part,
    f_abar(x, t+1) = -f*_a(x, t) + 2 w_a rho_out [1 + (c.u)^2 / (2 cs^4) - u.u / (2 cs^2)],
    u the node's own velocity.  The full expansion adds terms of order u^4;
    at |u| ~ 3e-4 they are below 1e-14."""
    rho_out = 0.993
    case, _, _ = _one_node_case(synth.OUTLET, rho_out=rho_out)
    rng = np.random.default_rng(4)
    fpost = o1.W * (1.0 + rng.uniform(-0.1, 0.1, 27))
    u = rng.uniform(-3e-4, 3e-4, 3)
    new = _boundary_step(tier, case, fpost, u, o2lib)
    err = 0.0
    for a in range(27):
        c = o1.C[a]
        if c[0] != -1:
            continue
        cu = float(c @ u)
        abb = -fpost[a] + 2.0 * o1.W[a] * rho_out * (1.0 + cu * cu / (2 * o1.CS2 ** 2) - (u @ u) / (2 * o1.CS2))
        err = max(err, abs(new[o1.OPP[a]] - abb))
    return err


INLET_RULE_TOL = 1e-14
OUTLET_RULE_TOL = 1e-13


@pytest.mark.parametrize("tier", ["o1", "o2"])
def test_P21_inlet_rule_is_moving_wall_bounce_back(o2lib, tier):
    assert _inlet_rule_error(tier, o2lib) < INLET_RULE_TOL


@pytest.mark.parametrize("tier", ["o1", "o2"])
def test_P22_outlet_rule_is_anti_bounce_back(o2lib, tier):
    assert _outlet_rule_error(tier, o2lib) < OUTLET_RULE_TOL


def test_P23_open_pipe_velocity_inlet_pressure_outlet(o2lib):
    """Straight pipe (R = 5, 30 fluid layers, tau = 1) with the steady
    Poiseuille profile (centreline 0.01) imposed by the inlet and rho_out = 1
    at the outlet, run to steady state (6000 steps; the velocity then changes
    by under 1e-6 of the centreline speed per 500 steps).  Closed forms it must meet:
    * mass conservation: the exact flux through every plane between two
      layers (fluid-to-fluid links only) equals the inlet inflow and the
      outlet outflow, and is positive (flow along +x);
    * that flux is the lattice integral of the imposed profile, sum over a
      cross-section of u(r), within 3 % (the diagonal links sample u at
      half-cell offsets);
    * the developed profile is Poiseuille's, u(r) = G0 (R^2 - r^2) / (4 nu),
      within 8 % in L2 (staircase wall of radius 5);
    * the pressure p = rho / 3 falls linearly with Poiseuille's gradient,
      d rho / dx = -3 G0, within 5 %;
    * extrapolated to the outlet plane (x = nx - 3/2, midway to the ghost
      layer) the density is rho_out within 5 % of the total drop.
    A sign error in either boundary rule reverses the flow or lets the mass
    run away; a dropped inlet term stops the flow."""
    nx = 32
    case = synth.open_pipe_case(nx=nx, tau=1.0)
    sim = o2lib.O2Sim(case, nthreads=8)
    sim.run(5500)
    _, u_prev = sim.macroscopic()
    mon = sim.run(500)
    rho, u = sim.macroscopic()
    assert np.max(np.abs(u - u_prev)) < 1e-6 * case.meta["u_max"]
    x, y, z = sim.coords[:, 0], sim.coords[:, 1], sim.coords[:, 2]
    C = o1.C
    fp = sim.fpost
    Q = []
    for xx in range(1, nx - 2):
        tot = 0.0
        for a in range(27):
            cx, cy, cz = C[a]
            if cx == 0:
                continue
            src = x == (xx if cx == 1 else xx + 1)
            fl = case.mask[z[src] + cz, y[src] + cy, x[src] + cx] == synth.FLUID
            tot += cx * fp[src][fl, a].sum()
        Q.append(tot)
    Q = np.array(Q)
    q_in, q_out = mon[7], mon[8]
    assert q_in > 0
    assert np.max(np.abs(Q - q_in)) < 1e-7 * q_in
    assert abs(q_out + q_in) < 1e-7 * q_in
    R = case.meta["radius"]
    cy0, cz0 = case.meta["center"]
    nu = case.nu
    G0 = case.inlet.G0
    r = np.sqrt((y - cy0) ** 2 + (z - cz0) ** 2)
    U = G0 * (R * R - r * r) / (4.0 * nu)
    mid = x == nx // 2
    assert abs(q_in / U[mid].sum() - 1.0) < 0.03
    assert np.sqrt(((u[mid, 0] - U[mid]) ** 2).sum() / (U[mid] ** 2).sum()) < 0.08
    assert np.max(np.abs(u[mid, 1:])) < 1e-3 * case.meta["u_max"]
    xs = np.arange(1, nx - 1)
    rm = np.array([rho[x == xx].mean() for xx in xs])
    sel = (xs > 5) & (xs < nx - 6)
    slope, icept = np.polyfit(xs[sel], rm[sel], 1)
    assert abs(slope / (-3.0 * G0) - 1.0) < 0.05
    drop = -slope * (nx - 2)
    assert abs(slope * (nx - 1.5) + icept - case.rho_out) < 0.05 * drop


def _momentum_balance(case, steps, step_fn):
    """Largest |P(t+1) - P(t) - M(t) g + F_wall(t)| over the steps, relative
    to |M g|: each collision adds rho g per node (Sec. 2.1.1 forcing,
    reading C6) and each halfway bounce-back link hands 2 f* c to the wall, so
    with the momentum-exchange wall force this balance is exact to rounding."""
    g = np.asarray(case.g, np.float64)
    worst = 0.0
    mass, mom = step_fn(0)
    for k in range(steps):
        mon = step_fn(1)
        resid = mon[1:4] - mom - mass * g + mon[4:7]
        worst = max(worst, float(np.max(np.abs(resid)) / np.max(np.abs(mass * g))))
        mass, mom = mon[0], mon[1:4]
    return worst


def _o2_stepper(sim):
    def fn(n):
        if n == 0:
            return sim.f.sum(), (sim.f @ o1.C.astype(np.float64)).sum(axis=0)
        return sim.run(n).copy()
    return fn


def _o1_stepper(st):
    def fn(n):
        if n == 0:
            fl = st.fluid
            f = st.f[fl[:, 0], fl[:, 1], fl[:, 2]]
            return f.sum(), (f @ o1.C.astype(np.float64)).sum(axis=0)
        o1.step(st)
        return st.monitors.copy()
    return fn


MOMENTUM_TOL = 1e-9


def test_P24_wall_force_balances_momentum(o2lib):
    """Periodic pipe under a body force (config 1 at a smaller radius): the
    per-step momentum balance P(t+1) = P(t) + M g - F_wall holds to rounding in
    both tiers, and at steady state the walls carry the whole driving force,
    F_wall = M g (the transient decays as exp(-5.78 nu t / R^2), below 1e-10 of
    it after 1200 steps at R = 5, nu = 0.1)."""
    case = synth.pipe_case(nx=4, ny=14, nz=14, radius=5.0, center=(6.3, 6.6), g=1e-5)
    sim = o2lib.O2Sim(case, nthreads=2)
    assert _momentum_balance(case, 30, _o2_stepper(sim)) < MOMENTUM_TOL
    mon = sim.run(1200)
    Mg = mon[0] * case.g[0]
    assert abs(mon[4] - Mg) < 1e-8 * Mg
    assert max(abs(mon[5]), abs(mon[6])) < 1e-8 * Mg
    small = synth.pipe_case(nx=3, ny=8, nz=8, radius=3.0, center=(3.4, 3.7), g=1e-5)
    assert _momentum_balance(small, 4, _o1_stepper(o1.O1State(small))) < MOMENTUM_TOL


def test_oracle_catches_planted_boundary_mistakes(o2lib, monkeypatch):
    """A sign flip planted in the inlet rule or the outlet rule, or a wall
    force without its factor 2 (each planted in tier O1, on the CPU), fails
    the pin of that rule by far more than its tolerance."""
    assert _inlet_rule_error("o1") < INLET_RULE_TOL
    monkeypatch.setattr(o1, "moving_wall_value", lambda src, fa, fb: src - (fb - fa))
    assert _inlet_rule_error("o1") > 1e3 * INLET_RULE_TOL
    monkeypatch.undo()
    assert _outlet_rule_error("o1") < OUTLET_RULE_TOL
    monkeypatch.setattr(o1, "anti_bounce_back_value", lambda src, fa, fb: src + fb + fa)
    assert _outlet_rule_error("o1") > 1e3 * OUTLET_RULE_TOL
    monkeypatch.setattr(o1, "anti_bounce_back_value", lambda src, fa, fb: -src - (fb + fa))
    assert _outlet_rule_error("o1") > 1e3 * OUTLET_RULE_TOL
    monkeypatch.undo()
    small = synth.pipe_case(nx=3, ny=8, nz=8, radius=3.0, center=(3.4, 3.7), g=1e-5)
    monkeypatch.setattr(o1, "wall_force_of_links", lambda src, c: 1.0 * src.sum() * c)
    assert _momentum_balance(small, 3, _o1_stepper(o1.O1State(small))) > 1e3 * MOMENTUM_TOL
    monkeypatch.setattr(o1, "wall_force_of_links", lambda src, c: -2.0 * src.sum() * c)
    assert _momentum_balance(small, 3, _o1_stepper(o1.O1State(small))) > 1e3 * MOMENTUM_TOL
