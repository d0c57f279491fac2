"""GPU parity of the all-pairs force evaluation against the FP64 oracle, through the C ABI.

Bar: per-element error max_i |a_gpu,i - a_orc,i| / max_k |a_orc,k| <= 1e-5 for the FP32 modes,
<= 1e-12 for the FP64 mode. The oracle reads the same FP32-rounded positions, promoted to FP64,
so the metric measures force arithmetic only.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import force_error, print_case, require_gpu, sample_rows

pytestmark = pytest.mark.gpu

TOL = {"plain": 1e-5, "kahan": 1e-5, "fp64": 1e-12}


def _gpu_forces(nb, ic, mode, **kw):
    s = nb.System.from_ic(ic, mode=mode, **kw)
    a = s.accelerations()
    s.close()
    return a


def _oracle_input(ic, mode):
    p, _ = ic.f32_as_f64()
    return p


@pytest.mark.parametrize("mode", ["plain", "kahan", "fp64"])
def test_c1_every_row(mode):
    nb = require_gpu()
    ic = synth.make_binary(2048, 0.5, seed=0)
    print_case("c1 forces", mode)
    a = _gpu_forces(nb, ic, mode)
    ref = oracle.accel(_oracle_input(ic, mode), ic.n1, ic.G, ic.m, ic.D1, ic.D2)
    err = force_error(a, ref)
    print("c1", mode, "max rel err", err)
    assert err <= TOL[mode]


@pytest.mark.parametrize("n,q", [(1, 0.5), (2, 1.0), (3, 0.5), (63, 0.3), (64, 0.5), (65, 0.8),
                                 (255, 0.5), (257, 0.4), (511, 0.9), (512, 0.5), (513, 0.2),
                                 (1000, 0.7), (3001, 0.3), (5000, 0.6), (9000, 0.35)])
@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_ragged_sizes_every_row(n, q, mode):
    nb = require_gpu()
    ic = synth.make_binary(n, q, seed=n)
    print_case("ragged", n, q, mode)
    a = _gpu_forces(nb, ic, mode)
    ref = oracle.accel(_oracle_input(ic, mode), ic.n1, ic.G, ic.m, ic.D1, ic.D2)
    assert force_error(a, ref) <= TOL[mode]


@pytest.mark.parametrize("which", ["all_star1", "all_star2"])
@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_single_star_systems(which, mode):
    nb = require_gpu()
    rng = np.random.default_rng(3)
    n = 1500
    pos = rng.uniform(-0.2, 0.2, size=(n, 3)).astype(np.float32).astype(np.float64)
    n1 = n if which == "all_star1" else 0
    kw = dict(G=1.0, m=1.0 / n, dt=1e-4, D1=0.03, D2=0.02, q=0.5)
    print_case("single star", which, mode)
    s = nb.System(pos, np.zeros_like(pos), n1, mode=mode, **kw)
    a = s.accelerations()
    s.close()
    ref = oracle.accel(pos, n1, kw["G"], kw["m"], kw["D1"], kw["D2"])
    assert force_error(a, ref) <= TOL[mode]


def test_equilibrium_pair_and_collinear_triple():
    nb = require_gpu()
    D = 0.05
    for mode in ("kahan", "fp64"):
        # at r = 10D/11 the contact repulsion cancels the interior attraction
        pos = np.array([[0.0, 0.0, 0.0], [10 * D / 11, 0.0, 0.0]])
        s = nb.System(pos, np.zeros_like(pos), 2, G=1.0, m=0.01, dt=1e-4, D1=D, D2=D, q=1.0,
                      mode=mode)
        a = s.accelerations()
        s.close()
        assert np.abs(a).max() < 1e-5 * (1.0 * 0.01 / D**2)
        # collinear equally spaced triple: the middle element feels nothing
        pos = np.array([[-0.2, 0.0, 0.0], [0.0, 0.0, 0.0], [0.2, 0.0, 0.0]])
        s = nb.System(pos, np.zeros_like(pos), 3, G=1.0, m=0.01, dt=1e-4, D1=D, D2=D, q=1.0,
                      mode=mode)
        a = s.accelerations()
        s.close()
        ref = oracle.accel(pos, 3, 1.0, 0.01, D, D)
        assert np.abs(a[1]).max() <= 1e-6 * np.abs(ref).max()
        assert force_error(a, ref) <= TOL[mode]


@pytest.mark.parametrize("n,q", [(65536, 0.5), (131072, 0.8), (262144, 0.3)])
def test_full_size_sampled_rows_kahan(n, q):
    nb = require_gpu()
    ic = synth.make_binary(n, q, seed=0)
    print_case("full size sampled", n, q)
    a = _gpu_forces(nb, ic, "kahan")
    rows = sample_rows(n, ic.n1, 160, seed=n)
    ref = oracle.accel(_oracle_input(ic, "kahan"), ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)
    err = force_error(a[rows], ref)
    print("full size", n, q, "kahan max rel err", err)
    assert err <= 1e-5


def test_precision_study_rows_c4():
    """N=131072, q=0.8: FP64 GPU mode ~1e-12, Kahan within 1e-5 and better than plain."""
    nb = require_gpu()
    ic = synth.make_binary(131072, 0.8, seed=0)
    rows = sample_rows(ic.n, ic.n1, 96, seed=1)
    ref = oracle.accel(_oracle_input(ic, "kahan"), ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)
    errs = {}
    for mode in ("plain", "kahan", "fp64"):
        print_case("c4 precision", mode)
        a = _gpu_forces(nb, ic, mode)
        errs[mode] = force_error(a[rows], ref)
    print("c4 errors", errs)
    assert errs["fp64"] <= 1e-12
    assert errs["kahan"] <= 1e-5
    assert errs["kahan"] < errs["plain"]


def test_repeated_evaluation_is_bitwise_stable():
    nb = require_gpu()
    ic = synth.make_binary(20000, 0.4, seed=9)
    s = nb.System.from_ic(ic, mode="kahan")
    a0 = s.accelerations()
    for _ in range(3):
        s.forces()
        assert np.array_equal(s.accelerations(), a0)
    s.close()


@pytest.mark.parametrize("mode,rows,tol", [("kahan", 1, 1e-5), ("kahan", 2, 1e-5),
                                           ("kahan", 4, 1e-5), ("fp64", 1, 1e-12)])
@pytest.mark.parametrize("nsplit", [1, 2, 3, 7])
def test_j_split_choices_agree(nsplit, mode, rows, tol):
    """Every chunking and band height of the symmetric kernels (FP32 Kahan and FP64) gives
    oracle parity."""
    nb = require_gpu()
    n = 12345
    ic = synth.make_binary(n, 0.6, seed=2)
    nb.nb_tile_override(n, n, nb.MODES[mode], nsplit, rows)
    try:
        cfg = nb.nb_tile_config(n, ic.n1, nb.MODES[mode])
        assert cfg["rows"] == rows
        print_case("nsplit", nsplit, mode, cfg)
        a = _gpu_forces(nb, ic, mode)
    finally:
        nb.nb_tile_override(n, n, nb.MODES[mode], 0, 1)
    ref = oracle.accel(_oracle_input(ic, mode), ic.n1, ic.G, ic.m, ic.D1, ic.D2)
    assert force_error(a, ref) <= tol


def test_full_size_sampled_rows_fp64():
    """The FP64 symmetric kernel at N = 262,144 (q = 0.3) on sampled rows."""
    nb = require_gpu()
    n, q = 262144, 0.3
    ic = synth.make_binary(n, q, seed=0)
    print_case("full size sampled fp64", n, q)
    a = _gpu_forces(nb, ic, "fp64")
    rows = sample_rows(n, ic.n1, 96, seed=n + 1)
    ref = oracle.accel(_oracle_input(ic, "fp64"), ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)
    err = force_error(a[rows], ref)
    print("full size fp64 max rel err", err)
    assert err <= 1e-12


@pytest.mark.parametrize("blocks", [7, 512])
@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_persistent_launch_is_bitwise_identical(blocks, mode):
    nb = require_gpu()
    print_case("persistent grid", blocks, mode)
    ic = synth.make_binary(30000, 0.5, seed=4)
    a0 = _gpu_forces(nb, ic, mode)
    nb.nb_set_force_grid(blocks)
    try:
        a1 = _gpu_forces(nb, ic, mode)
    finally:
        nb.nb_set_force_grid(0)
    assert np.array_equal(a0, a1)
