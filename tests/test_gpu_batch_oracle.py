"""Batched paths against the FP64 oracle.

Every way the library advances several systems together -- nb_step over a segment table of
several systems, a replayed multi-system graph, and the continuous-batching server -- is compared
here system by system with that system's own oracle run, over the same 100-step horizon and with
the same bars as one system alone: max|dx| <= 1e-5 a and max|dv| <= 1e-4 max|v| in FP32 Kahan
mode, 1e-11 a and 1e-10 max|v| in FP64 mode. Donor diameters are FP64 with the same operations on
both sides (bitwise equal); in FP64 mode the per-step L1 record must equal the oracle's exactly.
Under eqs. (4)-(6) with beta < 1 the FP32 velocity bar is 2e-3 max|v| (a contact pair near a
sign tie may take the other branch for a step; see tests/test_gpu_paper_law.py).
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import print_case, require_gpu

pytestmark = pytest.mark.gpu

# ragged sizes (none a multiple of 256 but the first), different mass ratios, one system small
# enough for a single tile row per star
CASES = [(2048, 0.5, 21), (3001, 0.3, 22), (700, 0.9, 23)]
STEPS = 100
BARS = {"kahan": (1e-5, 1e-4), "fp64": (1e-11, 1e-10)}


def _ics(law):
    ics = []
    for n, q, seed in CASES:
        ic = synth.make_binary(n, q, seed=seed)
        if law == "paper":
            ic = synth.with_velocity_noise(ic, 0.05, seed + 1000)
        ics.append(ic)
    return ics


def _law_kw(ic, law):
    return synth.paper_law_params(ic, beta=0.5) if law == "paper" else {}


def _oracle_run(ic, law):
    p, v = ic.f32_as_f64()
    kw = {}
    if law == "paper":
        lp = _law_kw(ic, law)
        kw = dict(law=1, eps=lp["eps"], gamma=lp["gamma"], beta=lp["beta"])
    run = oracle.Run(p, v, ic.n1, ic.G, ic.m, 1e-4, ic.D1, ic.D2, ic.q, a=ic.a, R2_0=ic.R2, **kw)
    counts, d2 = run.advance(STEPS)
    return run, counts


def _check(tag, ic, law, mode, xg, vg, d2=None, l1=None):
    run, counts = _oracle_run(ic, law)
    xtol, vtol = BARS[mode]
    if law == "paper" and mode == "kahan":
        vtol = 2e-3
    dx = np.abs(xg - run.pos).max()
    dv = np.abs(vg - run.vel).max() / np.abs(run.vel).max()
    print(tag, "n", ic.n, "q", ic.q, "max|dx|", dx, "max|dv|/max|v|", dv, flush=True)
    assert dx <= xtol * ic.a, (tag, ic.n)
    assert dv <= vtol, (tag, ic.n)
    if d2 is not None:
        assert d2 == run.D2, (tag, ic.n)
    if l1 is not None and mode == "fp64":
        assert l1.shape == (STEPS, 4)
        assert np.array_equal(l1[:, 0], np.arange(1, STEPS + 1))
        assert np.array_equal(l1[:, 1:], counts), (tag, ic.n)


def _systems(nb, ics, mode, law):
    return [nb.System.from_ic(ic, mode=mode, **_law_kw(ic, law)) for ic in ics]


def _finish(tag, systems, ics, law, mode):
    for s, ic in zip(systems, ics):
        d = s.diagnostics()
        assert d["step"] == STEPS
        assert d["nonfinite"] == 0
        _check(tag, ic, law, mode, s.positions(), s.velocities(), d["D2"], s.l1_log(STEPS))
        s.close()


@pytest.mark.parametrize("mode,law", [("kahan", "contact"), ("fp64", "contact"),
                                      ("kahan", "paper"), ("fp64", "paper")])
def test_multi_system_step_matches_oracle(mode, law):
    nb = require_gpu()
    print_case("batched nb_step vs oracle", mode, law)
    ics = _ics(law)
    systems = _systems(nb, ics, mode, law)
    # uneven chunks: the segment table is built once and reused across calls
    for k in (1, 29, 70):
        nb.step_many(systems, k)
    systems[0].synchronize()
    _finish("step_many", systems, ics, law, mode)


@pytest.mark.parametrize("mode,law", [("kahan", "contact"), ("fp64", "contact"),
                                      ("kahan", "paper")])
def test_multi_system_graph_matches_oracle(mode, law):
    nb = require_gpu()
    print_case("batched graph vs oracle", mode, law)
    ics = _ics(law)
    systems = _systems(nb, ics, mode, law)
    st = systems[0].stream
    g = nb.nb_graph_create([s.handle for s in systems], 10, st)
    for _ in range(STEPS // 10):
        nb.nb_graph_launch(g, st)
    st.synchronize()
    nb.nb_graph_destroy(g)
    _finish("graph", systems, ics, law, mode)


@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_server_results_match_oracle(mode):
    """Four requests arriving over 30 ms, served by continuous batching with graphs; each final
    state against the oracle's run of the same request."""
    require_gpu()
    from paper_2303_12166_amd import serve

    print_case("server vs oracle", mode)
    cases = CASES + [(4160, 0.75, 24)]
    trace = [synth.Request(rid=k, t_arrive=0.01 * k, n=n, q=q, steps=STEPS, seed=seed)
             for k, (n, q, seed) in enumerate(cases)]
    server = serve.BatchServer(budget_bytes=4 << 30, round_steps=10, mode=mode, fill=1e7,
                               keep_states=True)
    recs = server.run(trace)
    assert server.rounds > STEPS // 10  # several rounds, systems joining while others run
    for rec, (n, q, seed) in zip(recs, cases):
        assert rec.status == "done", rec.rid
        xg, vg = rec.state
        _check("server", synth.make_binary(n, q, seed=seed), "contact", mode, xg, vg)
