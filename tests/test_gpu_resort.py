"""nb_resort: the force kernels' sorted order rebuilt from the current positions.

After a re-sort the order is a Morton order of the current positions (each star's elements once,
padding -1), forces keep oracle parity, and a system re-sorted at the same steps of its own run
gets the same bits alone and in a batch.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import force_error, print_case, require_gpu

pytestmark = pytest.mark.gpu


def test_resort_order_and_forces():
    nb = require_gpu()
    ic = synth.make_binary(6000, 0.4, seed=21)
    print_case("resort order and forces")
    s = nb.System.from_ic(ic, mode="kahan")
    s.step(40)
    before = nb.nb_sorted_order(s.handle, s.stream)
    s.resort()
    after = nb.nb_sorted_order(s.handle, s.stream)
    n1, n = ic.n1, ic.n
    p1 = -(-n1 // 256) * 256
    assert after.size == before.size
    assert sorted(after[:n1].tolist()) == list(range(n1))
    assert sorted(after[p1:p1 + n - n1].tolist()) == list(range(n1, n))
    assert np.all(after[n1:p1] == -1) and np.all(after[p1 + n - n1:] == -1)
    pos = s.positions()
    d2 = s.diagnostics()["D2"]  # the donor has grown for 40 steps
    s.forces()
    a = s.accelerations()
    s.close()
    assert not np.array_equal(before, after)
    ref = oracle.accel(pos.astype(np.float64), ic.n1, ic.G, ic.m, ic.D1, d2)
    assert force_error(a, ref) <= 1e-5


@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_resort_alone_equals_batch(mode):
    """Two systems re-sorted every 5 of their own steps: stepped alone and stepped together (one
    nb_step over both, re-sorting each at the same steps) they end bitwise equal."""
    nb = require_gpu()
    cases = [(3000, 0.3, 31), (5000, 0.8, 32)]
    print_case("resort alone vs batch", mode)

    def make():
        return [nb.System.from_ic(synth.make_binary(n, q, seed=sd), mode=mode)
                for n, q, sd in cases]

    alone, mix = make(), make()
    for s in alone:
        for _ in range(3):
            s.step(5)
            s.resort()
    for _ in range(3):
        nb.step_many(mix, 5)
        for s in mix:
            s.resort()
    for a, b in zip(alone, mix):
        assert np.array_equal(a.positions(), b.positions())
        assert np.array_equal(a.velocities(), b.velocities())
        assert np.array_equal(nb.nb_sorted_order(a.handle, a.stream),
                              nb.nb_sorted_order(b.handle, b.stream))
    for s in alone + mix:
        s.close()
