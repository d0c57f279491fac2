"""Pins of the oracle's accretor-side retention count (transferred donor elements that are bound
to the accretor as a point mass at its centre of mass, moving with its mean velocity)."""

import math

import numpy as np

import oracle


def _system(test_pos, test_vel, q=0.5, G=1.0, m=1e-3, n1=400, n2=600, seed=0):
    """Accretor: n1 elements in +/- pairs about the origin (centre exactly 0, mean velocity
    exactly 0). Donor bulk: n2 elements in +/- pairs about (1, 0, 0), at rest. Test elements are
    appended to the donor; the returned arrays put the accretor first."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(-0.02, 0.02, size=(n1 // 2, 3))
    acc = np.concatenate([h, -h])
    hv = rng.normal(0.0, 0.1, size=(n1 // 2, 3))
    accv = np.concatenate([hv, -hv])
    d = rng.uniform(-0.02, 0.02, size=(n2 // 2, 3))
    don = np.concatenate([d, -d]) + np.array([1.0, 0.0, 0.0])
    pos = np.concatenate([acc, don, np.asarray(test_pos, dtype=float).reshape(-1, 3)])
    vel = np.concatenate([accv, np.zeros_like(don), np.asarray(test_vel, dtype=float).reshape(-1, 3)])
    return pos, vel, n1, G, m, q


def _vesc(G, m, n1, r):
    return math.sqrt(2.0 * G * m * n1 / r)


def test_hand_placed_bound_unbound_and_not_past():
    G, m, n1 = 1.0, 1e-3, 400
    r = 0.2
    ve = _vesc(G, m, n1, r)
    test_pos = [[r, 0, 0], [0, r, 0], [r, 0, 0], [0.95, 0.0, 0.0], [-r, 0, 0]]
    test_vel = [[0, 0.5 * ve, 0], [0.3 * ve, 0, 0], [0, 0, 2.0 * ve], [0, 0, 0], [0, 1.5 * ve, 0]]
    pos, vel, n1, G, m, q = _system(test_pos, test_vel)
    # past L1 (L1 sits about 0.57 of the way to the donor): the first three and the last;
    # bound: the first two
    assert oracle.retention(pos, vel, n1, G, m, q) == (4, 2)


def test_threshold_is_the_escape_speed():
    G, m, n1, r = 1.0, 1e-3, 400, 0.15
    ve = _vesc(G, m, n1, r)
    for f, bound in ((0.999, 1), (1.001, 0)):
        pos, vel, n1_, G_, m_, q = _system([[0.0, 0.0, r]], [[f * ve, 0.0, 0.0]])
        assert oracle.retention(pos, vel, n1_, G_, m_, q) == (1, bound)


def test_velocity_relative_to_accretor_mean():
    """A uniform boost of every element changes nothing; boosting only the accretor does."""
    G, m, n1, r = 1.0, 1e-3, 400, 0.2
    ve = _vesc(G, m, n1, r)
    pos, vel, n1, G, m, q = _system([[r, 0, 0]], [[0, 0.6 * ve, 0]])
    assert oracle.retention(pos, vel, n1, G, m, q) == (1, 1)
    boost = np.array([3.0, -2.0, 1.0])
    assert oracle.retention(pos, vel + boost, n1, G, m, q) == (1, 1)
    vel2 = vel.copy()
    vel2[:n1] += np.array([0.0, -0.6 * ve, 0.0])  # now the element moves at 1.2 v_esc relative
    assert oracle.retention(pos, vel2, n1, G, m, q) == (1, 0)


def test_rotation_and_translation_invariance():
    rng = np.random.default_rng(4)
    G, m, n1 = 1.0, 1e-3, 400
    tp = rng.uniform(-0.3, 0.7, size=(60, 3)) * np.array([1.0, 0.4, 0.4])
    tv = rng.normal(0.0, 1.5, size=(60, 3))
    pos, vel, n1, G, m, q = _system(tp, tv)
    base = oracle.retention(pos, vel, n1, G, m, q)
    assert base[0] > 5 and 0 < base[1] < base[0]
    a = 0.7
    R = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0],
                  [0.0, 0.0, 1.0]])
    b = 1.1
    R = R @ np.array([[1.0, 0.0, 0.0], [0.0, math.cos(b), -math.sin(b)],
                      [0.0, math.sin(b), math.cos(b)]])
    assert oracle.retention(pos @ R.T + np.array([5.0, -3.0, 2.0]), vel @ R.T, n1, G, m, q) == base


def test_degenerate_systems():
    rng = np.random.default_rng(1)
    pos = rng.normal(size=(50, 3))
    vel = rng.normal(size=(50, 3))
    assert oracle.retention(pos, vel, 0, 1.0, 1e-2, 0.5) == (0, 0)
    assert oracle.retention(pos, vel, 50, 1.0, 1e-2, 0.5) == (0, 0)
    assert oracle.retention(np.zeros((0, 3)), np.zeros((0, 3)), 0, 1.0, 1e-2, 0.5) == (0, 0)


def test_past_count_agrees_with_l1_count():
    rng = np.random.default_rng(9)
    G, m, n1 = 1.0, 1e-3, 400
    tp = rng.uniform(-0.3, 1.0, size=(200, 3)) * np.array([1.0, 0.3, 0.3])
    pos, vel, n1, G, m, q = _system(tp, np.zeros_like(tp))
    assert oracle.retention(pos, vel, n1, G, m, q)[0] == oracle.l1_count(pos, n1, q)[0]
