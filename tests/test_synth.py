"""Checks of the seeded input generator (counts, centring, rigid rotation, frozen samples)."""

import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ic_checksums.json")


def test_counts_follow_mass_ratio():
    assert synth.particle_counts(2048, 0.5) == (1366, 682)
    assert synth.particle_counts(262144, 0.3) == (201650, 60494)
    assert synth.particle_counts(131072, 0.8) == (72818, 58254)
    assert synth.particle_counts(65536, 0.5) == (43691, 21845)
    assert synth.particle_counts(0, 0.5) == (0, 0)


def test_c1_layout():
    ic = synth.make_binary(2048, 0.5, seed=0)
    assert ic.m == pytest.approx(1.5 / 2048, rel=1e-15)
    assert ic.D1 == pytest.approx(0.6 * (0.74 / 1366) ** (1 / 3), rel=1e-14)
    assert ic.D2 == pytest.approx(0.4 * (0.74 / 682) ** (1 / 3), rel=1e-14)
    assert ic.omega == pytest.approx(math.sqrt(1.5), rel=1e-15)
    # centres of mass of the stars at the barycentric positions, total COM at the origin
    M1, M2 = ic.n1 * ic.m, ic.n2 * ic.m
    c1 = ic.pos[: ic.n1].mean(axis=0)
    c2 = ic.pos[ic.n1:].mean(axis=0)
    assert np.allclose(c1, [-M2 / (M1 + M2), 0, 0], atol=1e-15)
    assert np.allclose(c2, [M1 / (M1 + M2), 0, 0], atol=1e-15)
    assert np.abs((ic.m * ic.pos).sum(axis=0)).max() < 1e-15
    # rigid rotation: zero net momentum, v = omega z x r
    assert np.abs((ic.m * ic.vel).sum(axis=0)).max() < 1e-14
    assert np.allclose(ic.vel[:, 0], -ic.omega * ic.pos[:, 1])
    # inside the balls (up to the shift that re-centres each sample)
    r1 = np.linalg.norm(ic.pos[: ic.n1] - c1, axis=1)
    assert 0.29 < r1.max() < 0.32


def test_deterministic_and_seeded():
    a = synth.make_binary(500, 0.3, seed=4)
    b = synth.make_binary(500, 0.3, seed=4)
    c = synth.make_binary(500, 0.3, seed=5)
    assert a.checksum() == b.checksum() != c.checksum()


def test_golden_checksums():
    with open(GOLDEN) as f:
        gold = json.load(f)
    for key, digest in gold["checksums"].items():
        n, q, seed = key.split(":")
        assert synth.make_binary(int(n), float(q), int(seed)).checksum() == digest, key


def test_trace_shape():
    tr = synth.make_trace()
    assert len(tr) == 256
    assert tr[0].t_arrive == 0.0
    assert all(t.n % 64 == 0 and 4096 <= t.n <= 131072 for t in tr)
    assert all(0.1 <= t.q <= 1.0 for t in tr)
    assert [t.seed for t in tr] == list(range(256))
    span = tr[-1].t_arrive
    assert 8.0 < span < 18.0  # 255 gaps of mean 1/20 s


def test_paper_law_recipe_has_one_equilibrium_inside_contact():
    """The eqs. (4)-(6) parameter recipe: the oracle's pair force is repulsive from r = 0 up to
    one equilibrium just inside D and attractive beyond, for converging and separating pairs."""
    import oracle

    ic = synth.make_binary(2048, 0.5, seed=0)
    kw = synth.paper_law_params(ic)
    R = 0.5 * ic.D1
    xs = np.linspace(1e-4, 2.0, 4001) * ic.D1
    for vr in (-1.0, 1.0):
        f = np.array([oracle.paper_force(r, vr, R, ic.G, ic.m, ic.m, kw["eps"], kw["gamma"],
                                         kw["beta"]) for r in xs])
        flips = np.flatnonzero(np.diff(np.sign(f)) != 0)
        assert len(flips) == 1
        assert 0.9 < xs[flips[0]] / ic.D1 < 0.97
        assert f[0] < 0 and f[-1] > 0
