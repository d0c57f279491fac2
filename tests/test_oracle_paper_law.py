"""Pins of the oracle's second law, eqs. (4)-(6) (softened attraction, overlap-volume repulsion,
weaker while the pair is not converging)."""

import math

import numpy as np
import pytest

import synth

R = 0.05
G, M = 1.0, 0.01


def test_overlap_volume_matches_lens_formula_and_limits(orc):
    # two spheres of radius R: V = pi (4R + r)(2R - r)^2 / 12 (a different closed form)
    for r in np.linspace(0.0, 2 * R, 11):
        lens = math.pi * (4 * R + r) * (2 * R - r) ** 2 / 12
        assert orc.overlap_volume(r, R) == pytest.approx(lens, rel=1e-12, abs=1e-18)
    assert orc.overlap_volume(0.0, R) == pytest.approx(4 / 3 * math.pi * R**3, rel=1e-15)
    assert orc.overlap_volume(2 * R, R) == 0.0
    assert orc.overlap_volume(3 * R, R) == 0.0


def test_overlap_volume_monte_carlo():
    import oracle

    rng = np.random.default_rng(0)
    r = 0.7 * R
    pts = rng.uniform(-R, R, size=(400000, 3))  # box around sphere 1 (centre 0)
    in1 = (pts**2).sum(axis=1) <= R * R
    in2 = ((pts - [r, 0, 0]) ** 2).sum(axis=1) <= R * R
    mc = (in1 & in2).mean() * (2 * R) ** 3
    assert oracle.overlap_volume(r, R) == pytest.approx(mc, rel=0.01)


def test_softened_far_field(orc):
    eps = 0.003
    f1 = orc.paper_force(3 * R, 0.0, R, G, M, M, eps, 50.0, 0.5)
    f2 = orc.paper_force(5 * R, 0.0, R, G, M, M, eps, 50.0, 0.5)
    assert f1 / f2 == pytest.approx(((5 * R + eps) / (3 * R + eps)) ** 2, rel=1e-14)
    assert f1 == pytest.approx(G * M * M / (3 * R + eps) ** 2, rel=1e-15)


def test_converging_repulsion_is_full_and_diverging_reduced(orc):
    eps, gamma, beta = 0.001, 50.0, 0.3
    for r in (0.3 * R, R, 1.7 * R):
        grav = orc.paper_force(r, 0.0, R, G, M, M, eps, 0.0, 1.0)  # gamma = 0: gravity alone
        conv = orc.paper_force(r, -1.0, R, G, M, M, eps, gamma, beta)
        div = orc.paper_force(r, +1.0, R, G, M, M, eps, gamma, beta)
        assert (grav - conv) / (grav - div) == pytest.approx(1 / beta, rel=1e-12)
        assert grav - conv == pytest.approx(gamma * orc.overlap_volume(r, R), rel=1e-12)


def test_potential_derivative_on_converging_branch(orc):
    eps, gamma = 0.002, 80.0
    for r in np.concatenate([np.linspace(0.1 * R, 1.95 * R, 8), np.linspace(2.05 * R, 6 * R, 5)]):
        h = 1e-7 * R
        dU = (orc.paper_potential(r + h, R, G, M, M, eps, gamma)
              - orc.paper_potential(r - h, R, G, M, M, eps, gamma)) / (2 * h)
        f = orc.paper_force(r, -1.0, R, G, M, M, eps, gamma, 0.5)
        assert dU == pytest.approx(f, rel=2e-6, abs=1e-9)
    # continuous at contact
    assert orc.paper_potential(2 * R * (1 - 1e-13), R, G, M, M, eps, gamma) == pytest.approx(
        -G * M * M / (2 * R + eps), rel=1e-9)


def _head_on(orc, beta, steps=4000, dt=2e-4):
    # two elements approaching along x at speed 1 each, starting 4R apart; weak gravity
    pos = np.array([[-2 * R, 0.0, 0.0], [2 * R, 0.0, 0.0]])
    vel = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    gamma = 2000.0
    run = orc.Run(pos, vel, 1, 1e-6, M, dt, 2 * R, 2 * R, 1.0, growth_on=False, law=1,
                  eps=1e-4, gamma=gamma, beta=beta)

    def energy():
        p, v = run.pos, run.vel
        r = np.linalg.norm(p[1] - p[0])
        ke = 0.5 * M * (v * v).sum()
        return ke + orc.paper_potential(r, R, 1e-6, M, M, 1e-4, gamma)

    E0 = energy()
    Es, P = [E0], []
    for _ in range(40):
        run.advance(steps // 40)
        Es.append(energy())
        P.append((M * run.vel).sum(axis=0))
    return run, np.array(Es), np.array(P)


def test_head_on_collision_elastic_when_beta_is_one(orc):
    run, E, P = _head_on(orc, 1.0)
    v = run.vel
    assert v[0][0] < 0 < v[1][0]  # they bounced
    assert abs(v[1][0]) == pytest.approx(1.0, rel=2e-3)  # elastic: speed restored
    assert np.abs(E - E[0]).max() < 2e-3 * abs(E[0])
    assert np.abs(P).max() < 1e-15


def test_head_on_collision_loses_energy_when_beta_below_one(orc):
    run, E, P = _head_on(orc, 0.25)
    v = run.vel
    assert v[0][0] < 0 < v[1][0]
    out = abs(v[1][0])
    assert 0.2 < out < 0.8  # inelastic rebound
    assert E[-1] < E[0] * (1 - 0.3)  # energy lost in the contact
    assert np.all(np.diff(E) <= 1e-4 * abs(E[0]))  # never gained beyond integrator noise
    assert np.abs(P).max() < 1e-15


def test_c_oracle_matches_numpy_transcription(orc):
    from oracle import np_ref

    ic = synth.make_binary(300, 0.5, seed=3)
    p, v = ic.f32_as_f64()
    rng = np.random.default_rng(1)
    v = v + rng.normal(0.0, 0.5, size=v.shape)
    kw = dict(eps=0.1 * ic.D1, gamma=30.0 * ic.m**2 / ic.D1**5, beta=0.4)
    a = orc.accel_paper(p, v, ic.n1, 1.0, ic.m, ic.D1, ic.D2, **kw)
    b = np_ref.accel_dense_paper(p, v, ic.n1, 1.0, ic.m, ic.D1, ic.D2, **kw)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_reduces_to_newton_without_softening_or_contact(orc):
    ic = synth.make_binary(200, 0.5, seed=2)
    p, v = ic.f32_as_f64()
    tiny = 1e-9  # diameters far below every separation: no contacts
    a = orc.accel_paper(p, v, ic.n1, 1.0, ic.m, tiny, tiny, 0.0, 5.0, 0.5)
    b = orc.accel(p, ic.n1, 1.0, ic.m, tiny, tiny)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_total_force_vanishes_with_random_velocities(orc):
    ic = synth.make_binary(1000, 0.5, seed=6)
    p, v = ic.f32_as_f64()
    v = v + np.random.default_rng(2).normal(0.0, 1.0, size=v.shape)
    a = orc.accel_paper(p, v, ic.n1, 1.0, ic.m, ic.D1, ic.D2, 0.05 * ic.D1,
                        20.0 * ic.m**2 / ic.D1**5, 0.5)
    assert np.abs(a.sum(axis=0)).max() < 1e-12 * np.abs(a).sum()


def test_split_run_equals_one_run(orc):
    """Under law 1 the first kick of a step uses the acceleration evaluated at the end of the
    previous step (with half-step velocities), so advancing 1 + 2 + 3 steps equals advancing 6."""
    rng = np.random.default_rng(12)
    n, n1 = 300, 200
    pos = rng.uniform(-0.1, 0.1, size=(n, 3))
    pos[n1:] += np.array([0.3, 0.0, 0.0])
    vel = rng.normal(0.0, 0.3, size=(n, 3))
    kw = dict(G=1.0, m=1.0 / n, dt=1e-4, D1=0.03, D2=0.025, q=0.5, a=0.3, R2_0=0.1,
              law=1, eps=0.003, gamma=2e3, beta=0.3)
    one = orc.Run(pos, vel, n1, **kw)
    c_one, _ = one.advance(6)
    split = orc.Run(pos, vel, n1, **kw)
    parts = [split.advance(k)[0] for k in (1, 2, 3)]
    assert np.array_equal(one.pos, split.pos)
    assert np.array_equal(one.vel, split.vel)
    assert np.array_equal(c_one, np.concatenate(parts))


def test_force_in_a_step_sees_the_half_step_velocity(orc):
    """Two overlapping elements closing slowly: the first half kick (strong repulsion) reverses
    their relative velocity, so the force at the new positions must take the separating branch
    (gamma beta), which only the half-step velocities show; with the start velocities it would
    take the converging one. One step is written out here from the pinned pair scalar."""
    R, G, m, eps, gamma, beta, dt = 0.05, 1.0, 0.01, 0.001, 2000.0, 0.2, 1e-3
    x0 = np.array([[0.0, 0.0, 0.0], [0.06, 0.0, 0.0]])
    v0 = np.array([[0.001, 0.0, 0.0], [-0.001, 0.0, 0.0]])  # converging, slowly

    def accel(x, v):
        d = x[1] - x[0]
        r = np.linalg.norm(d)
        vr = np.dot(v[1] - v[0], d) / r
        f = orc.paper_force(r, vr, R, G, m, m, eps, gamma, beta)
        a0 = (f / m) * d / r
        return np.array([a0, -a0])

    a = accel(x0, v0)
    vh = v0 + 0.5 * dt * a
    assert np.dot(vh[1] - vh[0], x0[1] - x0[0]) > 0  # the half kick made them separate
    x1 = x0 + dt * vh
    a1_half = accel(x1, vh)
    a1_start = accel(x1, v0)
    assert not np.allclose(a1_half, a1_start)  # the two readings differ here
    v1 = vh + 0.5 * dt * a1_half
    run = orc.Run(x0, v0, 1, G, m, dt, 2 * R, 2 * R, 1.0, growth_on=False, law=1, eps=eps,
                  gamma=gamma, beta=beta)
    run.advance(1)
    assert np.allclose(run.pos, x1, rtol=0, atol=1e-15)
    assert np.allclose(run.vel, v1, rtol=0, atol=1e-12)


# ------------------------------------------------------------------ potential energy sum, eqs. (5)-(6)
#
# The contact energy of a pair is the work done against the overlap repulsion from first touch
# (r = 2R) down to r: gamma * integral_r^2R V(s) ds. The hand values below come from integrating
# the lens volume V(s) = pi (4/3 R^3 - R^2 s + s^3/12) by hand:
#   r = 0: R^4,  r = R/2: 117/256 R^4,  r = R: 7/48 R^4,  r = 3R/2: 5/256 R^4,  r >= 2R: 0
# (each times gamma pi), plus the softened gravity -G m^2 / (r + eps).

PE_EPS, PE_GAMMA = 0.004, 3.0e3


def _pe_two(orc, r, D1=2 * R, D2=2 * R, n1=2):
    pos = np.array([[0.1, -0.2, 0.05], [0.1 + r, -0.2, 0.05]])
    return orc.paper_pe(pos, n1, G, M, D1, D2, PE_EPS, PE_GAMMA)


@pytest.mark.parametrize("frac,contact", [(0.5, 117 / 256), (1.0, 7 / 48), (1.5, 5 / 256),
                                          (2.5, 0.0), (4.0, 0.0)])
def test_paper_pe_two_elements_hand_values(orc, frac, contact):
    r = frac * R
    want = -G * M * M / (r + PE_EPS) + contact * PE_GAMMA * math.pi * R**4
    assert _pe_two(orc, r) == pytest.approx(want, rel=1e-12)


def test_paper_pe_continuous_at_contact_and_full_overlap_limit(orc):
    # just inside contact the overlap energy vanishes like (2R - r)^3
    for r in (2 * R * (1 - 1e-6), 2 * R * (1 + 1e-6)):
        assert _pe_two(orc, r) == pytest.approx(-G * M * M / (r + PE_EPS), rel=1e-12)
    # nearly full overlap: gamma pi R^4 of contact energy
    tiny = 1e-9 * R
    assert _pe_two(orc, tiny) == pytest.approx(
        -G * M * M / (tiny + PE_EPS) + PE_GAMMA * math.pi * R**4, rel=1e-7)


def test_paper_pe_uses_half_the_pair_diameter_per_star_class(orc):
    # D1 != D2: inside star 1 R = D1/2, inside star 2 R = D2/2, across R = (D1 + D2)/4
    D1, D2 = 0.1, 0.06
    for n1, Rp in ((2, D1 / 2), (0, D2 / 2), (1, (D1 + D2) / 4)):
        got = _pe_two(orc, Rp, D1=D1, D2=D2, n1=n1)
        want = -G * M * M / (Rp + PE_EPS) + 7 / 48 * PE_GAMMA * math.pi * Rp**4
        assert got == pytest.approx(want, rel=1e-12), n1


def test_paper_pe_collinear_triple_counts_each_pair_once(orc):
    # elements at 0, R and 5R/2 on a line: pair distances R, 3R/2 and 5R/2
    pos = np.array([[0.0, 0.0, 0.0], [R, 0.0, 0.0], [2.5 * R, 0.0, 0.0]])
    got = orc.paper_pe(pos, 3, G, M, 2 * R, 2 * R, PE_EPS, PE_GAMMA)
    want = (-G * M * M * (1 / (R + PE_EPS) + 1 / (1.5 * R + PE_EPS) + 1 / (2.5 * R + PE_EPS))
            + (7 / 48 + 5 / 256) * PE_GAMMA * math.pi * R**4)
    assert got == pytest.approx(want, rel=1e-12)


def _contact_energy_quadrature(r, Rp):
    """gamma * integral_r^2R V(s) ds with V from the lens formula pi (4R + s)(2R - s)^2 / 12
    (a cubic, so two-point Gauss-Legendre is exact)."""
    lo, hi = r, np.maximum(2 * Rp, r)
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    out = 0.0
    for t in (-1 / math.sqrt(3), 1 / math.sqrt(3)):
        s = mid + half * t
        out = out + half * math.pi * (4 * Rp + s) * (2 * Rp - s) ** 2 / 12
    return PE_GAMMA * out


def test_paper_pe_random_cluster_against_quadrature(orc):
    """Every pair of a dense two-star cluster (many contacts), written out pair by pair with the
    contact energy from quadrature of the lens volume."""
    rng = np.random.default_rng(21)
    n, n1, D1, D2 = 60, 35, 0.08, 0.05
    pos = rng.uniform(-0.12, 0.12, size=(n, 3))
    want = 0.0
    contacts = 0
    for i in range(n):
        for j in range(i + 1, n):
            r = float(np.linalg.norm(pos[j] - pos[i]))
            si, sj = i >= n1, j >= n1
            D = (D1 + D2) / 2 if si != sj else (D2 if si else D1)
            want += -G * M * M / (r + PE_EPS)
            if r < D:
                want += _contact_energy_quadrature(r, D / 2)
                contacts += 1
    assert contacts > 50
    got = orc.paper_pe(pos, n1, G, M, D1, D2, PE_EPS, PE_GAMMA)
    assert got == pytest.approx(want, rel=1e-12)


def test_paper_pe_conserved_in_elastic_head_on_collision(orc):
    """With beta = 1 the law is conservative: KE + paper_pe stays constant through the bounce up
    to the leap-frog's O(dt^2) error, and it is the same energy the pair potential gives."""
    gamma, eps, Gs = 2000.0, 1e-4, 1e-6
    pos = np.array([[-2 * R, 0.0, 0.0], [2 * R, 0.0, 0.0]])
    vel = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    run = orc.Run(pos, vel, 2, Gs, M, 2e-4, 2 * R, 2 * R, 1.0, growth_on=False, law=1, eps=eps,
                  gamma=gamma, beta=1.0)
    energies, min_r = [], 4 * R
    for _ in range(40):
        run.advance(100)
        p, v = run.pos, run.vel
        min_r = min(min_r, float(np.linalg.norm(p[1] - p[0])))
        energies.append(0.5 * M * (v * v).sum() + orc.paper_pe(p, 2, Gs, M, 2 * R, 2 * R, eps,
                                                                 gamma))
    E0 = 0.5 * M * (vel * vel).sum() + orc.paper_pe(pos, 2, Gs, M, 2 * R, 2 * R, eps, gamma)
    assert min_r < 1.5 * R  # the pair went deep into contact
    assert np.abs(np.array(energies) - E0).max() < 2e-3 * abs(E0)
