"""Graph replays and the continuous-batching server on the GPU.

Graph replays must reproduce nb_step bitwise (the same kernels with the same arguments), with the
program's own eager work and synchronisations between replays. The server must produce, for
every request, the same final state as the one-at-a-time baseline.
"""

import numpy as np
import pytest

import synth
from gpu_common import print_case, require_gpu

pytestmark = pytest.mark.gpu


def _sys(nb, n, q, seed, mode="kahan"):
    return nb.System.from_ic(synth.make_binary(n, q, seed=seed), mode=mode)


@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_graph_replays_match_nb_step(mode):
    nb = require_gpu()
    print_case("graph vs step", mode)
    a = _sys(nb, 5000, 0.4, 1, mode)
    b = _sys(nb, 5000, 0.4, 1, mode)
    g = nb.nb_graph_create([b.handle], 5, b.stream)
    for k in range(4):
        a.step(5)
        nb.nb_graph_launch(g, b.stream)
        b.synchronize()
        d = b.diagnostics(with_pe=(k == 1))  # eager work (a reduction over many blocks) between
        assert d["step"] == 5 * (k + 1)        # replays
        # every replay against the eager steps
        assert np.array_equal(a.positions(), b.positions()), k
        assert np.array_equal(a.velocities(), b.velocities()), k
        assert np.array_equal(a.sides(), b.sides()), k
        assert a.diagnostics()["D2"] == d["D2"]
    nb.nb_graph_destroy(g)
    a.close()
    b.close()


def test_batched_graph_matches_systems_alone():
    nb = require_gpu()
    cases = [(3000, 0.3, 1), (20000, 0.8, 2), (4096, 0.1, 3)]
    alone = [_sys(nb, *c) for c in cases]
    for s in alone:
        s.step(12)
    mix = [_sys(nb, *c) for c in cases]
    g = nb.nb_graph_create([s.handle for s in mix], 4, mix[0].stream)
    for _ in range(3):
        nb.nb_graph_launch(g, mix[0].stream)
        mix[0].synchronize()
    nb.nb_graph_destroy(g)
    for x, y in zip(alone, mix):
        assert np.array_equal(x.positions(), y.positions())
        assert y.diagnostics()["step"] == 12
    for s in alone + mix:
        s.close()


def _small_trace(count=10, steps=30, rate=400.0, seed=5):
    return synth.make_trace(count=count, rate=rate, n_min=2048, n_max=12288, steps=steps,
                            seed=seed)


@pytest.mark.parametrize("policy,use_graphs,depth", [("srpt", True, 2), ("all", True, 2),
                                                     ("srpt", False, 2), ("srpt", True, 1)])
def test_server_results_equal_sequential_results(policy, use_graphs, depth):
    """Every policy, with captured graphs or plain multi-system steps, one or two rounds queued:
    each request's final state equals its one-at-a-time run bit for bit."""
    require_gpu()
    from paper_2303_12166_amd import serve

    print_case("serve", policy, "graphs" if use_graphs else "nb_step", "depth", depth)
    trace = _small_trace()
    server = serve.BatchServer(budget_bytes=8 << 30, round_steps=7, policy=policy, fill=2e8,
                               use_graphs=use_graphs, depth=depth)
    batched = server.run(trace)
    seq = serve.run_sequential(trace, chunk=11)
    assert all(r.status == "done" for r in batched)
    for rb, rs in zip(batched, seq):
        assert rb.rid == rs.rid
        assert rb.digest == rs.digest, rb.rid
        assert rb.t_done >= rb.t_arrive
    s = serve.summarize(batched)
    assert s["completed"] == len(trace)
    assert s["latency_p99_s"] >= s["latency_p50_s"] > 0
    assert (server.graphs_built >= 1) == use_graphs


def test_server_admission_under_small_budget():
    require_gpu()
    from paper_2303_12166_amd import serve

    trace = _small_trace(count=8, steps=20, seed=9)
    sizes = sorted(serve.footprint_bytes(r.n, r.q) for r in trace)
    budget = sizes[-1] + sizes[0] // 2  # the largest fits alone, pairs mostly do not
    server = serve.BatchServer(budget_bytes=budget, round_steps=5)
    recs = server.run(trace)
    assert all(r.status == "done" for r in recs)
    # the footprints bound what was admitted at once, and PyTorch's peak allocation over the
    # run stays within them up to the allocator's rounding (512 B per tensor, 11 per system)
    assert 0 < server.peak_footprint_bytes <= budget
    assert server.peak_allocated_bytes <= server.peak_footprint_bytes + 11 * 512 * len(trace)
    # admissions wait for memory: some request is admitted after an earlier one finished
    done_times = sorted(r.t_done for r in recs)
    assert any(r.t_admit >= done_times[0] for r in recs)
    # a request larger than the whole budget is rejected, the rest still complete
    big = synth.make_trace(count=3, rate=1000.0, n_min=4096, n_max=4096, steps=5, seed=1)
    tight = serve.BatchServer(budget_bytes=serve.footprint_bytes(4096, big[0].q) - 1,
                              round_steps=5)
    out = tight.run(big[:1])
    assert out[0].status == "rejected"


def test_nonfinite_system_is_evicted_and_the_others_are_unchanged():
    """A NaN written into one system's positions while its batch runs (queued on the compute
    stream after the third round): that request ends "failed" and leaves the server early; every
    other request still ends bit for bit as in its one-at-a-time run."""
    require_gpu()
    import torch

    from paper_2303_12166_amd import serve

    print_case("serve nonfinite eviction")
    trace = _small_trace(count=8, steps=40, rate=2000.0, seed=13)
    victim = trace[2].rid

    class Poisoning(serve.BatchServer):
        def __init__(self, *a, **kw):
            super().__init__(*a, **kw)
            self.by_handle = {}
            self.poisoned_at = None

        def build_system(self, req):
            s = super().build_system(req)
            self.by_handle[s.handle.value] = req.rid
            return s

        def on_round_queued(self, systems):
            if self.poisoned_at is None and self.rounds >= 2:
                for s in systems:
                    if self.by_handle.get(s.handle.value) == victim:
                        with torch.cuda.stream(self.compute):
                            s.x[5:6].fill_(float("nan"))
                        self.poisoned_at = self.rounds

    server = Poisoning(budget_bytes=8 << 30, round_steps=5, fill=1e9)
    recs = server.run(trace)
    seq = serve.run_sequential(trace, chunk=9)
    assert server.poisoned_at is not None
    assert server.evicted == 1
    by = {r.rid: r for r in recs}
    assert by[victim].status == "failed"
    assert by[victim].t_done >= by[victim].t_arrive
    for rb, rs in zip(recs, seq):
        if rb.rid == victim:
            continue
        assert rb.status == "done" and rs.status == "done"
        assert rb.digest == rs.digest, rb.rid
    s = serve.summarize(recs)
    assert s["completed"] == len(trace) - 1 and s["failed"] == 1
