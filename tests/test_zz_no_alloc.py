"""nb_step_static, the multi-system step that allocates nothing (its segment table lives in a
fixed per-GPU array), against nb_step on identical systems: bitwise the same state after two
calls in a row, the second on a smaller batch, in the FP32 Kahan and FP64 modes.

Both calls run the same kernels on the same segment-table contents, so equality is exact.
"""

import ctypes

import numpy as np
import pytest

import synth
from gpu_common import print_case, require_gpu

pytestmark = pytest.mark.gpu

# ragged sizes (several tiles, a short last tile), different q, one small enough for a single
# tile row per star
CASES = [(3000, 0.3, 11), (5000, 0.7, 12), (2048, 0.5, 13), (700, 0.9, 14)]


def _make(nb, mode, law="contact"):
    out = []
    for n, q, seed in CASES:
        ic = synth.make_binary(n, q, seed=seed)
        kw = {}
        if law == "paper":
            ic = synth.with_velocity_noise(ic, 0.05, seed + 100)
            kw = synth.paper_law_params(ic)
        out.append(nb.System.from_ic(ic, mode=mode, **kw))
    return out


def _same_state(a, b):
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.velocities(), b.velocities())
    assert np.array_equal(a.accelerations(), b.accelerations())
    da, db = a.diagnostics(), b.diagnostics()
    for key in ("step", "D2", "n_past_L1", "cross_fwd", "cross_bwd", "growth_stopped",
                "nonfinite"):
        assert da[key] == db[key], key


@pytest.mark.parametrize("mode,law", [("kahan", "contact"), ("fp64", "contact"),
                                      ("kahan", "paper")])
def test_static_step_equals_step(mode, law):
    nb = require_gpu()
    print_case("nb_step_static vs nb_step", mode, law)
    ref = _make(nb, mode, law)
    sta = _make(nb, mode, law)
    st = ref[0].stream
    # first call: all four systems
    nb.nb_step([s.handle for s in ref], 7, st)
    nb.nb_step_static([s.handle for s in sta], 7, st)
    for a, b in zip(ref, sta):
        _same_state(a, b)
        assert a.diagnostics()["step"] == 7
    # second call on a smaller batch, in another order: the table keeps the first call's
    # contents until it is rewritten, and nothing of them may leak into this one
    pick = [2, 0]
    nb.nb_step([ref[k].handle for k in pick], 4, st)
    nb.nb_step_static([sta[k].handle for k in pick], 4, st)
    for k, (a, b) in enumerate(zip(ref, sta)):
        _same_state(a, b)
        assert a.diagnostics()["step"] == (11 if k in pick else 7)
    for s in ref + sta:
        s.close()


def test_static_step_single_system_and_limit():
    nb = require_gpu()
    print_case("nb_step_static one system; limit")
    n, q, seed = CASES[1]
    a = nb.System.from_ic(synth.make_binary(n, q, seed=seed), mode="kahan")
    b = nb.System.from_ic(synth.make_binary(n, q, seed=seed), mode="kahan")
    a.step(5)
    nb.nb_step_static([b.handle], 5, b.stream)
    _same_state(a, b)
    lib = nb.load()
    many = (ctypes.c_void_p * (nb.NB_STATIC_MAX_SYS + 1))(*([b.handle.value] *
                                                           (nb.NB_STATIC_MAX_SYS + 1)))
    assert lib.nb_step_static(many, nb.NB_STATIC_MAX_SYS + 1, 1, None) == nb.NB_E_LIMIT
    assert b.diagnostics()["step"] == 5  # the refused call queued nothing
    a.close()
    b.close()
