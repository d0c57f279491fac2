"""Pins of the oracle's time stepping, eq. (3), L1 and donor growth.

Kepler's two-body solution pins G, the inverse-square law and the kick-drift-kick integrator;
the energy error's dt^2 scaling pins the integrator's order; eq. (3)'s limits, the L1 root's
symmetry and Hill limit, and the closed-form growth stop step pin the support functions.
"""

import math

import numpy as np
import pytest

import synth

TINY_D = 1e-4  # element diameter far below any separation used: pure Newtonian gravity


def _two_body(orc, sep, v_rel, dt, m=0.5):
    # two elements of mass m (total 1) on the x axis, relative velocity along +y for element 1
    pos = np.array([[-sep / 2, 0.0, 0.0], [sep / 2, 0.0, 0.0]])
    vel = np.array([[0.0, -v_rel / 2, 0.0], [0.0, v_rel / 2, 0.0]])
    return orc.Run(pos, vel, n1=1, G=1.0, m=m, dt=dt, D1=TINY_D, D2=TINY_D, q=1.0,
                   growth_on=False)


@pytest.mark.parametrize("a", [1.0, 2.0])
def test_circular_kepler_period_and_radius(orc, a):
    GM = 1.0  # G (m1 + m2)
    T = 2 * math.pi * math.sqrt(a**3 / GM)
    dt = T / 8000
    run = _two_body(orc, a, math.sqrt(GM / a), dt)
    seps = []
    for _ in range(8):
        run.advance(1000)
        p = run.pos
        seps.append(np.linalg.norm(p[1] - p[0]))
    assert max(abs(s - a) for s in seps) < 1e-6 * a
    # after exactly one period the pair is back where it started
    p = run.pos
    assert np.allclose(p, [[-a / 2, 0, 0], [a / 2, 0, 0]], atol=5e-6 * a)


def _kepler_relative(a, e, GM, t):
    n = math.sqrt(GM / a**3)
    Mean = n * t
    E = Mean
    for _ in range(60):  # Newton on Kepler's equation E - e sin E = M
        E -= (E - e * math.sin(E) - Mean) / (1 - e * math.cos(E))
    return np.array([a * (math.cos(E) - e), a * math.sqrt(1 - e * e) * math.sin(E), 0.0])


def test_eccentric_kepler_against_keplers_equation(orc):
    a, e, GM = 1.0, 0.5, 1.0
    rp = a * (1 - e)
    vp = math.sqrt(GM * (1 + e) / rp)
    T = 2 * math.pi
    dt = 2e-4
    run = _two_body(orc, rp, vp, dt)
    nsteps = int(round(T / 3 / dt))
    run.advance(nsteps)
    p = run.pos
    rel = p[1] - p[0]
    expect = _kepler_relative(a, e, GM, nsteps * dt)
    assert np.linalg.norm(rel - expect) < 2e-6


def test_energy_error_is_second_order(orc):
    a, e, GM = 1.0, 0.5, 1.0
    rp = a * (1 - e)
    vp = math.sqrt(GM * (1 + e) / rp)

    def max_rel_energy_error(dt):
        run = _two_body(orc, rp, vp, dt)
        E0 = orc.diag(run.pos, run.vel, 1, 1.0, 0.5, TINY_D, TINY_D)["E"]
        worst = 0.0
        nchunks = 40
        per = int(round(2 * math.pi / dt / nchunks))
        for _ in range(nchunks):
            run.advance(per)
            E = orc.diag(run.pos, run.vel, 1, 1.0, 0.5, TINY_D, TINY_D)["E"]
            worst = max(worst, abs(E - E0) / abs(E0))
        return worst

    e1 = max_rel_energy_error(2e-3)
    e2 = max_rel_energy_error(1e-3)
    assert 3.5 < e1 / e2 < 4.5


def test_momentum_conserved_with_contacts(orc):
    ic = synth.make_binary(1024, 0.5, seed=11)
    p, v = ic.f32_as_f64()
    run = orc.Run(p, v, ic.n1, 1.0, ic.m, 1e-4, ic.D1, ic.D2, ic.q)
    d0 = orc.diag(run.pos, run.vel, ic.n1, 1.0, ic.m, ic.D1, run.D2)
    run.advance(50)
    d1 = orc.diag(run.pos, run.vel, ic.n1, 1.0, ic.m, ic.D1, run.D2)
    scale = ic.m * np.abs(run.vel).sum()
    assert np.abs(d1["P"] - d0["P"]).max() < 1e-13 * scale


def test_energy_conserved_with_contacts_without_growth(orc):
    ic = synth.make_binary(1024, 0.5, seed=11)
    p, v = ic.f32_as_f64()
    run = orc.Run(p, v, ic.n1, 1.0, ic.m, 1e-4, ic.D1, ic.D2, ic.q, growth_on=False)
    E0 = orc.diag(run.pos, run.vel, ic.n1, 1.0, ic.m, ic.D1, ic.D2)["E"]
    run.advance(100)
    E1 = orc.diag(run.pos, run.vel, ic.n1, 1.0, ic.m, ic.D1, ic.D2)["E"]
    assert abs(E1 - E0) < 1e-7 * abs(E0)


# ---------------------------------------------------------------- eq. (3)


def test_eggleton_unit_mass_ratio(orc):
    # eq. (3) at q = 1: 0.49 / (0.69 + ln 2)
    assert orc.roche_lobe(1.0) == pytest.approx(0.3542645402, rel=1e-9)


def test_eggleton_limits_and_monotonicity(orc):
    # q -> 0: r_L -> 0.49 q^(1/3); q -> inf: r_L -> 0.49 / 0.69
    q = 1e-12
    assert orc.roche_lobe(q) / q ** (1 / 3) == pytest.approx(0.49, rel=1e-3)
    assert orc.roche_lobe(1e15) == pytest.approx(0.49 / 0.69, rel=1e-4)
    qs = np.linspace(0.01, 5, 200)
    r = np.array([orc.roche_lobe(x) for x in qs])
    assert np.all(np.diff(r) > 0)


# ---------------------------------------------------------------- L1


def test_l1_equal_masses_is_midpoint(orc):
    assert orc.l1_point(1.0) == pytest.approx(0.5, abs=1e-15)


def test_l1_hill_limit(orc):
    # small donor: L1 sits at the Hill distance (mu/3)^(1/3)(1 - (mu/3)^(1/3)/3) from the donor
    for q in (1e-6, 1e-5):
        mu = q / (1 + q)
        h = (mu / 3) ** (1 / 3)
        assert 1 - orc.l1_point(q) == pytest.approx(h * (1 - h / 3), rel=2e-4)


def test_l1_moves_toward_accretor_as_donor_grows(orc):
    qs = np.linspace(0.05, 1.0, 40)
    xi = np.array([orc.l1_point(q) for q in qs])
    assert np.all(np.diff(xi) < 0)
    assert np.all((xi > 0.5 - 1e-15) & (xi < 1))


def _l1_config():
    # star 1: two elements with centre at the origin; star 2: centre at x = 1
    s1 = [[-0.1, 0.0, 0.0], [0.1, 0.0, 0.0]]
    s2 = [[0.55, 0.2, 0.0], [1.2, -0.2, 0.0], [1.25, 0.0, 0.1], [1.0, 0.0, -0.1]]
    return np.array(s1 + s2), 2


def test_l1_counts_hand_placed(orc):
    pos, n1 = _l1_config()  # donor centre (1, 0, 0): L1 at x = 0.5708 for q = 0.5
    side = np.zeros(len(pos), dtype=np.int8)
    assert orc.l1_count(pos, n1, 0.5, side, init=True) == (1, 0, 0)
    # moves that keep the donor centre at x = 1 (shifts sum to zero)
    moved = pos.copy()
    moved[2, 0] = 0.65  # the element past L1 moves back (+0.10)
    moved[5, 0] = 0.50  # one from the donor moves through (-0.50)
    moved[3, 0] = 1.60  # (+0.40)
    assert moved[n1:, 0].mean() == pytest.approx(1.0, abs=1e-15)
    assert orc.l1_count(moved, n1, 0.5, side) == (1, 1, 1)
    moved[2, 0] = 0.40  # (-0.25)
    moved[4, 0] = 1.50  # (+0.25)
    assert orc.l1_count(moved, n1, 0.5, side) == (2, 1, 0)
    assert orc.l1_count(moved, n1, 0.5, side) == (2, 0, 0)
    # for q = 0.3 L1 sits farther out (0.6209): the element at 0.60 counts as past
    moved[2, 0] = 0.60
    moved[4, 0] = 1.30
    assert orc.l1_count(moved, n1, 0.3) == (2, 0, 0)
    assert orc.l1_count(moved, n1, 0.8) == (1, 0, 0)


def test_l1_counts_rotation_invariant(orc):
    pos, n1 = _l1_config()
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    assert orc.l1_count(pos @ R.T + [0.3, -2.0, 0.5], n1, 0.5) == orc.l1_count(pos, n1, 0.5)


# ---------------------------------------------------------------- donor growth


@pytest.mark.parametrize("q", [0.5, 0.8])
def test_growth_stops_at_closed_form_step(orc, q):
    R2_0 = 0.2
    rl = orc.roche_lobe(q)
    nstar = math.ceil(math.log(rl / R2_0) / math.log(1 + 1e-4))
    pos = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    run = orc.Run(pos, np.zeros((2, 3)), 1, 1.0, 1e-3, 1e-4, 0.01, 0.02, q, R2_0=R2_0)
    _, d2 = run.advance(nstar + 5)
    # grows on steps 1..n*, constant afterwards
    assert d2[nstar - 1] > d2[nstar - 2]
    assert np.all(d2[nstar - 1:] == d2[nstar - 1])
    assert d2[nstar - 1] == pytest.approx(0.02 * (1 + 1e-4) ** nstar, rel=1e-12)
    assert run.growth_stopped
    assert R2_0 * d2[nstar - 1] / 0.02 > rl >= R2_0 * d2[nstar - 2] / 0.02


def test_growth_off_keeps_diameter(orc):
    pos = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    run = orc.Run(pos, np.zeros((2, 3)), 1, 1.0, 1e-3, 1e-4, 0.01, 0.02, 0.5, growth_on=False)
    _, d2 = run.advance(10)
    assert np.all(d2 == 0.02)


def test_diagnostics_hand_values(orc):
    """COM, P, L and KE of a hand-placed configuration: a rotating pair plus a drifting third
    element, values worked out by hand."""
    m = 0.25
    pos = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 2.0]])
    vel = np.array([[0.0, 1.0, 0.0], [0.0, -1.0, 0.0], [3.0, 0.0, 0.0]])
    d = orc.diag(pos, vel, 2, 1.0, m, 0.01, 0.01, with_pe=False)
    assert np.allclose(d["com"], [0.0, 0.0, 2.0 / 3.0], atol=1e-15)
    assert np.allclose(d["P"], [3.0 * m, 0.0, 0.0], atol=1e-15)
    # L = sum m r x v: the pair gives m (0, 0, 1) twice; the third element has r = (0, 0, 2),
    # v = (3, 0, 0), r x v = (0, 6, 0)
    assert np.allclose(d["L"], [0.0, 6.0 * m, 2.0 * m], atol=1e-15)
    assert abs(d["KE"] - 0.5 * m * (1.0 + 1.0 + 9.0)) < 1e-15
    assert d["PE"] == 0.0


def test_growth_applies_after_the_step(orc):
    """The donor grows after a step's second kick (the paper does not fix the order within a
    step; this is the order taken on both sides). The first step's forces use the
    initial diameter, so growing and non-growing runs agree exactly after one step, holding D2_0
    (1 + g) and D2_0. The grown diameter first enters the force at the end of the second step:
    after it the positions still agree (they moved with the first step's forces) and the donor
    velocities differ (the donor pair below is in contact, where the force depends on D2)."""
    pos = np.array([[-0.6, 0.0, 0.0], [0.5, 0.0, 0.0], [0.515, 0.0, 0.0]])
    vel = np.array([[0.0, 0.1, 0.0], [0.0, 0.0, 0.01], [0.0, 0.0, -0.01]])
    args = (pos, vel, 1, 1.0, 1e-3, 1e-3, 0.01, 0.02, 0.5)
    grow, keep = orc.Run(*args, R2_0=0.2), orc.Run(*args, R2_0=0.2, growth_on=False)
    _, d_grow = grow.advance(1)
    _, d_keep = keep.advance(1)
    assert np.array_equal(grow.pos, keep.pos) and np.array_equal(grow.vel, keep.vel)
    assert d_grow[0] == 0.02 * (1 + 1e-4) and d_keep[0] == 0.02
    grow.advance(1)
    keep.advance(1)
    assert np.array_equal(grow.pos, keep.pos)
    dv = np.abs(grow.vel - keep.vel).max(axis=1)
    assert dv[1] > 0 and dv[2] > 0
    grow.advance(1)
    keep.advance(1)
    assert not np.array_equal(grow.pos[1:], keep.pos[1:])


def test_l1_count_inside_a_run_ballistic(orc):
    """The count of a run uses each step's final positions. With G = 0 the elements move on
    straight lines. Here the donor centre stays at x = 1 (two elements move apart symmetrically)
    and star 1 sits at the origin, so L1 (q = 0.5) is the plane x = 0.570752. The element from
    x = 0.60 at speed 0.05 (dt = 0.01) is at 0.60 - 0.0005 k after step k, first below the plane
    at k = 59: one forward crossing there, one element past L1 from then on."""
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.60, 0.0, 0.0], [1.40, 0.0, 0.0]])
    vel = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [-0.05, 0.0, 0.0], [0.05, 0.0, 0.0]])
    run = orc.Run(pos, vel, 1, 0.0, 1e-3, 0.01, 0.01, 0.01, 0.5, growth_on=False)
    counts, _ = run.advance(80)
    past, fwd, bwd = counts[:, 0], counts[:, 1], counts[:, 2]
    assert np.all(past[:58] == 0) and np.all(past[58:] == 1)
    assert fwd[58] == 1 and fwd.sum() == 1 and bwd.sum() == 0
    assert run.pos[2, 0] == pytest.approx(0.60 - 0.05 * 0.8, abs=1e-12)


def _contact_oscillator(D=0.1, m=1e-3, dt=1e-3, u0=0.002, v0=0.01):
    """Two elements of one star in contact, moving apart at relative speed v0. Inside D the
    contact law is affine in r, f = (11 G m^2 / D^3) (r - 10 D / 11), so the separation obeys
    u'' = -w^2 u with u = r - r_eq, r_eq = 10 D / 11 and w^2 = 22 G m / D^3 (G = 1). The
    leap-frog map of a linear force is exactly
    u_k = u_0 cos(k theta) + (v_0 dt / sin theta) sin(k theta), cos theta = 1 - (w dt)^2 / 2."""
    r0 = 10.0 * D / 11.0 + u0
    pos = np.array([[-0.5 * r0, 0.0, 0.0], [0.5 * r0, 0.0, 0.0]])
    vel = np.array([[-0.5 * v0, 0.0, 0.0], [0.5 * v0, 0.0, 0.0]])
    w2 = 22.0 * m / D ** 3
    theta = math.acos(1.0 - w2 * dt * dt / 2.0)
    amp = math.hypot(u0, v0 * dt / math.sin(theta))

    def u_exact(k):
        return u0 * math.cos(k * theta) + v0 * dt / math.sin(theta) * math.sin(k * theta)

    return pos, vel, u_exact, 10.0 * D / 11.0, amp


@pytest.mark.parametrize("n1,D1,D2", [(2, 0.1, 0.1), (1, 0.08, 0.12)])
def test_contact_oscillation_matches_the_leapfrog_closed_form(orc, n1, D1, D2):
    """Both elements in star 1 (D = D1), or one in each star (D = (D1 + D2) / 2 = 0.1). Bar:
    FP64 rounding of positions of size 0.05, accumulated over 2000 steps (measured 1.6e-14). A
    wrong stiffness, sign, pair diameter or integrator variant (drift-kick-drift, Euler) misses
    it by orders of magnitude."""
    D, m, dt = 0.1, 1e-3, 1e-3
    pos, vel, u_exact, r_eq, amp = _contact_oscillator(D, m, dt)
    assert r_eq + amp < D and r_eq - amp > 0  # the separation stays where the law is affine
    run = orc.Run(pos, vel, n1, 1.0, m, dt, D1, D2, 0.5, growth_on=False)
    done = 0
    for k in (1, 250, 1000, 2000):
        run.advance(k - done)
        done = k
        p = run.pos
        assert abs((p[1, 0] - p[0, 0]) - r_eq - u_exact(k)) < 2e-13
        assert abs(p[0, 0] + p[1, 0]) < 1e-15  # the centre of mass stays at the origin


def test_no_growth_when_the_donor_starts_beyond_its_lobe(orc):
    """At q = 0.1 the lobe radius r_L = 0.1992 is below the initial donor radius 0.2, so the first
    growth check stops growth for good and the diameter never changes."""
    assert orc.roche_lobe(0.1) < 0.2 < orc.roche_lobe(0.102)
    pos = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    run = orc.Run(pos, np.zeros((2, 3)), 1, 1.0, 1e-3, 1e-4, 0.01, 0.02, 0.1, R2_0=0.2)
    _, d2 = run.advance(5)
    assert np.all(d2 == 0.02) and run.growth_stopped
