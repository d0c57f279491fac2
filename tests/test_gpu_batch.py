"""Multi-system steps: one launch per kernel over several systems' work (segment table).

Each system's result must be bitwise the same alone and in the mix: every system's work units,
tile shapes and reduction orders depend on its own size only.
"""

import numpy as np
import pytest

import synth
from gpu_common import print_case, require_gpu

pytestmark = pytest.mark.gpu

CASES = [(3000, 0.3, 1), (5000, 0.7, 2), (2048, 0.5, 3), (70000, 0.9, 4), (4096, 0.1, 5)]


def _make(nb, mode):
    return [nb.System.from_ic(synth.make_binary(n, q, seed=s), mode=mode) for n, q, s in CASES]


@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_alone_equals_mix_bitwise(mode):
    nb = require_gpu()
    print_case("alone vs mix", mode)
    alone = _make(nb, mode)
    for s in alone:
        s.step(15)
    mix = _make(nb, mode)
    nb.step_many(mix, 15)
    for a, b in zip(alone, mix):
        assert np.array_equal(a.positions(), b.positions())
        assert np.array_equal(a.velocities(), b.velocities())
        da, db = a.diagnostics(), b.diagnostics()
        assert da["D2"] == db["D2"] and da["n_past_L1"] == db["n_past_L1"]
        assert da["step"] == db["step"] == 15
    for s in alone + mix:
        s.close()


def test_changing_membership():
    nb = require_gpu()
    systems = _make(nb, "kahan")
    ref = _make(nb, "kahan")
    # steps in varying groupings; each system ends up with 6 steps
    nb.step_many(systems[:2], 2)
    nb.step_many(systems[1:4], 2)
    nb.step_many([systems[0], systems[3], systems[4]], 2)
    nb.step_many([systems[2], systems[4]], 4)
    nb.step_many([systems[0], systems[3]], 2)
    nb.step_many(systems[1:2], 2)
    for s in ref:
        s.step(6)
    for a, b in zip(systems, ref):
        assert a.diagnostics()["step"] == 6
        assert np.array_equal(a.positions(), b.positions())
    for s in systems + ref:
        s.close()


def test_mode_mismatch_and_duplicates_rejected():
    nb = require_gpu()
    a = nb.System.from_ic(synth.make_binary(1000, 0.5, seed=1), mode="kahan")
    b = nb.System.from_ic(synth.make_binary(1000, 0.5, seed=2), mode="fp64")
    with pytest.raises(nb.NbError) as e:
        nb.step_many([a, b], 1)
    assert e.value.status == nb.NB_E_MISMATCH
    with pytest.raises(nb.NbError) as e:
        nb.step_many([a, a], 1)
    assert e.value.status == nb.NB_E_INVAL
    a.close()
    b.close()


def test_batches_on_two_streams_concurrently():
    """Two threads step two different batches on two streams at once; each system ends bitwise
    equal to the same system stepped alone (each stream has its own segment table)."""
    import threading

    import torch

    nb = require_gpu()
    print_case("two streams, two batches")
    groups = [[(3000, 0.3, 11), (5000, 0.7, 12)], [(2048, 0.5, 13), (4096, 0.9, 14)]]
    alone = []
    for grp in groups:
        for n, q, seed in grp:
            s = nb.System.from_ic(synth.make_binary(n, q, seed=seed), mode="kahan")
            s.step(12)
            alone.append((s.positions(), s.velocities()))
            s.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    mixes = []
    for grp, st in zip(groups, streams):
        mixes.append([nb.System.from_ic(synth.make_binary(n, q, seed=seed), mode="kahan",
                                        stream=st) for n, q, seed in grp])
    torch.cuda.synchronize()
    errors = []

    def run(mix, st):
        try:
            for _ in range(12):
                nb.step_many(mix, 1, st)
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=run, args=(m, st)) for m, st in zip(mixes, streams)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors
    got = [(s.positions(), s.velocities()) for m in mixes for s in m]
    for (xa, va), (xb, vb) in zip(alone, got):
        assert np.array_equal(xa, xb)
        assert np.array_equal(va, vb)
    for m in mixes:
        for s in m:
            s.close()
