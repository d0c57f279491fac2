"""Bands of 1, 2 and 4 tile rows per work unit in the FP32 Kahan symmetric kernel.

A band of k rows evaluates k tile rows against each staged j tile, keeps one i element of every
row per lane and stores one reaction block per (band, later tile). Every band height must give
oracle parity for both element laws, at ragged sizes (a short last band, a short last tile, a
band across the star boundary) and at full size, and a batch that mixes band heights must give
each system bitwise the result it gets alone.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import force_error, print_case, require_gpu, sample_rows

pytestmark = pytest.mark.gpu

K = 1  # NB_FP32_KAHAN


def _with_rows(nb, n, rows, nsplit, law="contact"):
    nb.nb_tile_override(n, n, K, nsplit, rows, law=nb.LAWS[law])


def _clear(nb, n, law="contact"):
    nb.nb_tile_override(n, n, K, 0, 1, law=nb.LAWS[law])


def _law(ic, law):
    if law == "paper":
        ic = synth.with_velocity_noise(ic, 0.05, 77)
        return ic, synth.paper_law_params(ic)
    return ic, {}


def _oracle_forces(ic, kw, rows=None):
    p, v = (x.astype(np.float64) for x in ic.f32())
    if kw:
        return oracle.accel_paper(p, v, ic.n1, ic.G, ic.m, ic.D1, ic.D2, kw["eps"], kw["gamma"],
                                  kw["beta"], rows=rows)
    return oracle.accel(p, ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)


@pytest.mark.parametrize("law", ["contact", "paper"])
@pytest.mark.parametrize("rows", [1, 2, 4])
@pytest.mark.parametrize("n,q,nsplit", [(2048, 0.5, 3), (3001, 0.3, 1), (12345, 0.6, 5),
                                        (700, 0.9, 2)])
def test_band_forces_match_oracle(n, q, nsplit, rows, law):
    nb = require_gpu()
    ic, kw = _law(synth.make_binary(n, q, seed=5), law)
    print_case("band forces", n, q, nsplit, rows, law)
    _with_rows(nb, n, rows, nsplit, law)
    try:
        cfg = nb.nb_tile_config(n, ic.n1, K, nb.LAWS[law])
        assert cfg["rows"] == rows
        s = nb.System.from_ic(ic, mode="kahan", **kw)
        a = s.accelerations()
        s.forces()
        a2 = s.accelerations()
        s.close()
    finally:
        _clear(nb, n, law)
    assert np.array_equal(a, a2)  # deterministic
    assert force_error(a, _oracle_forces(ic, kw)) <= 1e-5


@pytest.mark.parametrize("rows", [2, 4])
def test_band_trajectory_100_steps(rows):
    """The 2048-element system over 100 steps with bands of 2 and 4 rows, at the same bars as
    the one-row kernel: positions within 1e-5 a, velocities within 1e-4 max|v|, the growing
    donor diameter exactly."""
    nb = require_gpu()
    ic = synth.make_binary(2048, 0.5, seed=0)
    print_case("band trajectory", rows)
    _with_rows(nb, 2048, rows, 2)
    try:
        s = nb.System.from_ic(ic, mode="kahan")
    finally:
        _clear(nb, 2048)
    p, v = ic.f32_as_f64()
    run = oracle.Run(p, v, ic.n1, ic.G, ic.m, 1e-4, ic.D1, ic.D2, ic.q, R2_0=ic.R2)
    s.step(100)
    run.advance(100)
    d = s.diagnostics()
    pos, vel = s.positions(), s.velocities()
    s.close()
    assert np.abs(pos - run.pos).max() <= 1e-5 * ic.a
    assert np.abs(vel - run.vel).max() <= 1e-4 * np.abs(run.vel).max()
    assert d["step"] == 100
    assert d["D2"] == run.D2  # bitwise: the same FP64 operations on both sides


def test_mixed_band_heights_alone_equals_batch():
    """Systems with bands of 1, 2 and 4 rows in one batch (nb_step, a replayed graph and
    nb_step_static): each ends bitwise equal to its run alone."""
    nb = require_gpu()
    cases = [(3000, 0.3, 1, 2), (5000, 0.7, 2, 3), (2048, 0.5, 4, 1), (4160, 0.2, 2, 4),
             (6000, 0.9, 4, 2)]
    for n, _, rows, ns in cases:
        _with_rows(nb, n, rows, ns)
    try:
        def make():
            return [nb.System.from_ic(synth.make_binary(n, q, seed=n), mode="kahan")
                    for n, q, _, _ in cases]
        alone, mix, graph, sta = make(), make(), make(), make()
    finally:
        for n, _, _, _ in cases:
            _clear(nb, n)
    print_case("mixed band heights", [c[2] for c in cases])
    for s in alone:
        s.step(6)
    nb.step_many(mix, 6)
    g = nb.nb_graph_create([s.handle for s in graph], 3, graph[0].stream)
    nb.nb_graph_launch(g, graph[0].stream)
    nb.nb_graph_launch(g, graph[0].stream)
    graph[0].synchronize()
    nb.nb_graph_destroy(g)
    nb.nb_step_static([s.handle for s in sta], 6, sta[0].stream)
    for k in range(len(cases)):
        ref = alone[k].positions()
        for other in (mix, graph, sta):
            assert np.array_equal(other[k].positions(), ref)
            assert np.array_equal(other[k].velocities(), alone[k].velocities())
            assert other[k].diagnostics()["step"] == 6
    for s in alone + mix + graph + sta:
        s.close()


@pytest.mark.parametrize("rows", [2, 4])
def test_band_full_size_sampled_rows(rows):
    """N = 262,144 (q = 0.3) with bands of 2 and 4 rows, on sampled rows against the oracle."""
    nb = require_gpu()
    n, q = 262144, 0.3
    ic = synth.make_binary(n, q, seed=0)
    print_case("band full size", rows)
    _with_rows(nb, n, rows, 57)
    try:
        s = nb.System.from_ic(ic, mode="kahan")
    finally:
        _clear(nb, n)
    a = s.accelerations()
    s.close()
    rows_s = sample_rows(n, ic.n1, 96, seed=rows)
    ref = _oracle_forces(ic, {}, rows=rows_s)
    scale = np.linalg.norm(ref, axis=1).max()
    err = np.linalg.norm(a[rows_s] - ref, axis=1).max() / scale
    assert err <= 1e-5


@pytest.mark.parametrize("mode,tol", [("kahan", 1e-5), ("fp64", 1e-12)])
def test_split_coarsened_by_the_workspace_budget(mode, tol):
    """A system created under a workspace budget below its requested split's workspace gets a
    coarser split (taller bands, then fewer chunks) and still oracle parity."""
    nb = require_gpu()
    n = 12345
    ic = synth.make_binary(n, 0.6, seed=9)
    M = nb.MODES[mode]
    nb.nb_tile_override(n, n, M, 12, 1)
    try:
        req = nb.nb_tile_config(n, ic.n1, M)
        p = nb.NbParams(n=n, n1=ic.n1, G=ic.G, m=ic.m, dt=1e-4, D1=ic.D1, D2=ic.D2, q=ic.q,
                        a=ic.a, R2_0=ic.R2, growth_rate=1e-4, growth_on=1, mode=M, law=0, pad=0,
                        eps=0.0, gamma=0.0, beta=1.0)
        full = nb.nb_scratch_bytes(p)
        nb.nb_set_workspace_budget(full * 2 // 3)
        try:
            cfg = nb.nb_tile_config(n, ic.n1, M)
            s = nb.System.from_ic(ic, mode=mode)
            # the FP32 Kahan split fits; the FP64 one (one row per band) shrinks as far as a
            # single chunk allows, still above the budget
            small = nb.nb_scratch_bytes(p)
            assert small <= full * 2 // 3 if mode == "kahan" else small < full
        finally:
            nb.nb_set_workspace_budget(0)
        assert nb.nb_scratch_bytes(p) == full  # budget lifted: the requested split again
    finally:
        nb.nb_tile_override(n, n, M, 0, 1)
    print_case("budget", mode, req, cfg)
    assert cfg != req
    a = s.accelerations()
    s.close()
    p64, _ = ic.f32_as_f64()
    ref = oracle.accel(p64, ic.n1, ic.G, ic.m, ic.D1, ic.D2)
    assert force_error(a, ref) <= tol
