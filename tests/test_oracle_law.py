"""Pins of the oracle's pair law and all-pairs sum against closed forms and invariants.

The law (Methodology: elements always attract; elements in contact repel):
f(r) = G m^2 / r^2 for r >= D, f(r) = G m^2 r / D^3 - K (1 - r/D) inside, K = 10 G m^2 / D^2.
Each check below pins a different piece, so that a dropped term, a wrong sign or a wrong
diameter fails at least one of them.
"""

import math

import numpy as np
import pytest

import synth

G, M, D = 1.0, 0.01, 0.05


def test_continuous_at_contact(orc):
    # the interior branch must meet Newton exactly at r = D
    inside = orc.pair_force(D * (1 - 1e-13), D, G, M, M)
    at = orc.pair_force(D, D, G, M, M)
    assert at == pytest.approx(G * M * M / D**2, rel=1e-15)
    assert inside == pytest.approx(at, rel=1e-11)


def test_equilibrium_distance(orc):
    # interior attraction G m^2 r/D^3 balances K(1 - r/D) with K = 10 G m^2/D^2 only at r = 10D/11
    scale = G * M * M / D**2
    assert abs(orc.pair_force(10 * D / 11, D, G, M, M)) < 1e-13 * scale
    assert orc.pair_force(0.9 * D, D, G, M, M) < 0  # closer: net repulsion
    assert orc.pair_force(0.92 * D, D, G, M, M) > 0  # farther: net attraction


def test_contact_limit_is_pure_repulsion_K(orc):
    K = 10 * G * M * M / D**2
    assert orc.pair_force(1e-12 * D, D, G, M, M) == pytest.approx(-K, rel=1e-10)


def test_interior_is_linear_in_r(orc):
    # inside the element the law is affine in r: equal steps give equal differences
    rs = np.linspace(0.05 * D, 0.95 * D, 7)
    f = np.array([orc.pair_force(r, D, G, M, M) for r in rs])
    d = np.diff(f)
    assert np.allclose(d, d[0], rtol=1e-10, atol=0)


def test_far_field_inverse_square(orc):
    f1 = orc.pair_force(3 * D, D, G, M, M)
    f2 = orc.pair_force(6 * D, D, G, M, M)
    assert f1 / f2 == pytest.approx(4.0, rel=1e-14)
    assert orc.pair_force(1.0, D, 2.0, 3.0, 5.0) == pytest.approx(30.0, rel=1e-15)


def test_potential_derivative_is_force(orc):
    # dU/dr = f by central differences on both branches, and U continuous at D
    for r in np.concatenate([np.linspace(0.02 * D, 0.98 * D, 9), np.linspace(1.02 * D, 5 * D, 9)]):
        h = 1e-6 * D
        dU = (orc.pair_potential(r + h, D, G, M, M) - orc.pair_potential(r - h, D, G, M, M)) / (2 * h)
        assert dU == pytest.approx(orc.pair_force(r, D, G, M, M), rel=1e-6, abs=1e-9 * G * M * M / D**2)
    below = orc.pair_potential(D * (1 - 1e-13), D, G, M, M)
    assert below == pytest.approx(-G * M * M / D, rel=1e-11)


def _accel(orc, pos, n1, D1, D2, m=M):
    return orc.accel(np.asarray(pos, dtype=np.float64), n1, G, m, D1, D2)


def test_two_body_direction_and_magnitude(orc):
    # attraction pulls each element toward the other with |a| = f/m; antisymmetric
    rng = np.random.default_rng(1)
    for r in (0.5 * D, 0.95 * D, 2.0 * D):
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        pos = np.array([[0.1, -0.2, 0.3], [0.1, -0.2, 0.3] + r * u])
        a = _accel(orc, pos, 2, D, D)
        f = orc.pair_force(r, D, G, M, M)
        assert np.allclose(a[0], (f / M) * u, rtol=1e-12, atol=1e-15)
        assert np.array_equal(a[0], -a[1])


def test_three_body_symmetric_configurations(orc):
    r = 3 * D
    # collinear, equally spaced: middle element feels nothing; ends feel G m (1/r^2 + 1/(2r)^2)
    pos = np.array([[-r, 0, 0], [0, 0, 0], [r, 0, 0]])
    a = _accel(orc, pos, 3, D, D)
    assert np.abs(a[1]).max() < 1e-12
    assert a[0][0] == pytest.approx(G * M * (1 / r**2 + 1 / (2 * r) ** 2), rel=1e-14)
    # equilateral triangle: sqrt(3) G m / r^2 toward the centroid
    pos = np.array([[0, 0, 0], [r, 0, 0], [r / 2, r * math.sqrt(3) / 2, 0]])
    a = _accel(orc, pos, 3, D, D)
    cen = pos.mean(axis=0)
    for i in range(3):
        u = (cen - pos[i]) / np.linalg.norm(cen - pos[i])
        assert np.allclose(a[i], math.sqrt(3) * G * M / r**2 * u, rtol=1e-13)


def test_cross_star_pairs_use_mean_diameter(orc):
    D1, D2 = 0.1, 0.3  # D12 = 0.2; 10/11 of D12 = 0.1818, of D2 = 0.2727
    for r, attract in ((0.15, False), (0.25, True)):
        pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        a = _accel(orc, pos, 1, D1, D2)  # element 0 in star 1, element 1 in star 2
        f = orc.pair_force(r, 0.2, G, M, M)
        assert (a[0][0] > 0) == attract
        assert a[0][0] == pytest.approx(f / M, rel=1e-14)
    # same-star pairs keep their own diameter
    pos = np.array([[0.0, 0.0, 0.0], [0.25, 0.0, 0.0]])
    assert _accel(orc, pos, 0, D1, D2)[0][0] < 0  # both in star 2: D2 = 0.3, repulsive
    assert _accel(orc, pos, 2, D1, D2)[0][0] > 0  # both in star 1: D1 = 0.1, Newton


def test_pairwise_antisymmetry_bitwise(orc):
    ic = synth.make_binary(2048, 0.5, seed=0)
    p, _ = ic.f32_as_f64()
    rng = np.random.default_rng(7)
    for _ in range(200):
        i, j = rng.integers(0, ic.n, size=2)
        fij = orc.pair_vector(p, ic.n1, G, ic.m, ic.D1, ic.D2, i, j)
        fji = orc.pair_vector(p, ic.n1, G, ic.m, ic.D1, ic.D2, j, i)
        assert np.array_equal(fij, -fji)


def test_total_force_vanishes(orc):
    ic = synth.make_binary(2048, 0.5, seed=0)
    p, _ = ic.f32_as_f64()
    a = orc.accel(p, ic.n1, G, ic.m, ic.D1, ic.D2)
    # momentum change rate sum_i m a_i = 0 up to rounding of the row sums
    scale = np.abs(a).sum()
    assert np.abs(a.sum(axis=0)).max() < 1e-13 * scale


def test_rows_subset_matches_full(orc):
    ic = synth.make_binary(700, 0.8, seed=3)
    p, _ = ic.f32_as_f64()
    full = orc.accel(p, ic.n1, G, ic.m, ic.D1, ic.D2)
    rows = np.array([0, 5, ic.n1 - 1, ic.n1, ic.n - 1])
    sub = orc.accel(p, ic.n1, G, ic.m, ic.D1, ic.D2, rows=rows)
    assert np.array_equal(sub, full[rows])


def test_c_oracle_matches_numpy_transcription(orc):
    from oracle import np_ref

    for n, q, seed in ((512, 0.5, 0), (333, 0.3, 5), (64, 1.0, 2)):
        ic = synth.make_binary(n, q, seed=seed)
        p, _ = ic.f32_as_f64()
        a = orc.accel(p, ic.n1, G, ic.m, ic.D1, ic.D2)
        b = np_ref.accel_dense(p, ic.n1, G, ic.m, ic.D1, ic.D2)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_potential_energy_pairs(orc):
    # the diagnostics' PE of two elements is the pair potential
    for r in (0.3 * D, 0.99 * D, 4 * D):
        pos = np.array([[0.0, 0.0, 0.0], [0.0, r, 0.0]])
        d = orc.diag(pos, np.zeros((2, 3)), 2, G, M, D, D, with_pe=True)
        assert d["PE"] == pytest.approx(orc.pair_potential(r, D, G, M, M), rel=1e-15)
