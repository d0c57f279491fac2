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
