"""GPU parity of the leap-frog step, donor growth, L1 count and FP64 diagnostics.

Trajectories: 100 kick-drift-kick steps at N=2048 against the FP64 oracle from the same
FP32-rounded start (positions within 1e-5 a, velocities within 1e-4 max|v|). Donor diameters
are FP64 on both sides with the same operations, so they must agree bitwise. L1 counts are
integers decided in FP64 on both sides from identical inputs (the GPU's FP32 state), so they
must agree exactly.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import print_case, require_gpu

pytestmark = pytest.mark.gpu


def _oracle_run(ic, dt=1e-4, growth_on=True, R2_0=None):
    p, v = ic.f32_as_f64()
    return oracle.Run(p, v, ic.n1, ic.G, ic.m, dt, ic.D1, ic.D2, ic.q, a=ic.a,
                      R2_0=ic.R2 if R2_0 is None else R2_0, growth_on=growth_on)


@pytest.mark.parametrize("mode,xtol,vtol", [("kahan", 1e-5, 1e-4), ("plain", 1e-5, 1e-4),
                                            ("fp64", 1e-11, 1e-10)])
def test_c1_trajectory_100_steps(mode, xtol, vtol):
    nb = require_gpu()
    ic = synth.make_binary(2048, 0.5, seed=0)
    print_case("c1 trajectory", mode)
    s = nb.System.from_ic(ic, mode=mode)
    s.step(100)
    xg, vg = s.positions(), s.velocities()
    dg = s.diagnostics()
    s.close()
    run = _oracle_run(ic)
    run.advance(100)
    dx = np.abs(xg - run.pos).max()
    dv = np.abs(vg - run.vel).max()
    vmax = np.abs(run.vel).max()
    print("c1", mode, "max |dx|", dx, "max |dv|/max|v|", dv / vmax)
    assert dx <= xtol * ic.a
    assert dv <= vtol * vmax
    assert dg["step"] == 100
    assert dg["D2"] == run.D2  # bitwise: same FP64 operations on both sides


def test_growth_stops_on_the_same_step_as_the_oracle():
    nb = require_gpu()
    ic = synth.make_binary(3000, 0.5, seed=4)
    rl = oracle.roche_lobe(0.5)
    R2_0 = rl * (1 - 7e-4)  # lobe reached after a handful of growth steps
    nstar = math.ceil(math.log(rl / R2_0) / math.log(1 + 1e-4))
    p, v = ic.f32()
    s = nb.System(p, v, ic.n1, G=ic.G, m=ic.m, dt=1e-4, D1=ic.D1, D2=ic.D2, q=0.5, R2_0=R2_0)
    run = _oracle_run(ic, R2_0=R2_0)
    _, d2_log = run.advance(nstar + 4)
    for k in range(nstar + 4):
        s.step(1)
        d = s.diagnostics()
        assert d["D2"] == d2_log[k], k
        assert d["growth_stopped"] == (k >= nstar)
    s.close()


def test_l1_counts_exact_on_identical_state():
    """Donor overflowing its lobe (R2 = 0.45): many donor elements sit past L1."""
    nb = require_gpu()
    ic = synth.make_binary(6000, 0.5, seed=5, R2=0.45)
    s = nb.System.from_ic(ic, mode="kahan")
    # initial sides come from the initial positions
    pos = s.positions().astype(np.float64)
    n0 = oracle.l1_count(pos, ic.n1, ic.q)[0]
    assert n0 > 0
    assert s.diagnostics()["n_past_L1"] == n0
    assert np.array_equal(s.sides()[ic.n1:], _past_flags(pos, ic)[ic.n1:])
    for k in range(12):
        s.step(5)
        pos = s.positions().astype(np.float64)
        assert s.diagnostics()["n_past_L1"] == oracle.l1_count(pos, ic.n1, ic.q)[0], k
        assert np.array_equal(s.sides()[ic.n1:], _past_flags(pos, ic)[ic.n1:]), k
    s.close()


def _past_flags(pos, ic):
    side = np.zeros(ic.n, dtype=np.int8)
    oracle.l1_count(pos, ic.n1, ic.q, side, init=True)
    return side


def test_l1_crossing_counts_step_by_step():
    """Rigid rotation alone moves nothing across the co-rotating L1 plane: an overfull donor
    (R2 = 0.6) with seeded random velocity kicks makes elements cross in both directions."""
    nb = require_gpu()
    ic = synth.make_binary(8000, 0.5, seed=6, R2=0.6)
    p, v = ic.f32()
    rng = np.random.default_rng(60)
    v = (v + rng.normal(0.0, 5.0, size=v.shape)).astype(np.float32)
    s = nb.System(p, v, ic.n1, G=ic.G, m=ic.m, dt=1e-4, D1=ic.D1, D2=ic.D2, q=ic.q, R2_0=ic.R2)
    side = np.zeros(ic.n, dtype=np.int8)
    oracle.l1_count(s.positions().astype(np.float64), ic.n1, ic.q, side, init=True)
    fwd = bwd = 0
    for k in range(40):
        s.step(1)
        pos = s.positions().astype(np.float64)
        expect = oracle.l1_count(pos, ic.n1, ic.q, side)
        d = s.diagnostics()
        assert (d["n_past_L1"], d["cross_fwd"], d["cross_bwd"]) == expect, k
        fwd += expect[1]
        bwd += expect[2]
    log = s.l1_log(40)
    s.close()
    print("L1 crossings over 40 steps: forward", fwd, "backward", bwd)
    assert fwd > 0 and bwd > 0
    assert log.shape == (40, 4)
    assert list(log[:, 0]) == list(range(1, 41))


def test_diagnostics_match_oracle_on_identical_state():
    nb = require_gpu()
    for mode in ("kahan", "fp64"):
        ic = synth.make_binary(4096, 0.6, seed=8)
        print_case("diagnostics", mode)
        s = nb.System.from_ic(ic, mode=mode)
        s.step(10)
        d = s.diagnostics(with_pe=True)
        pos, vel = s.positions().astype(np.float64), s.velocities().astype(np.float64)
        s.close()
        ref = oracle.diag(pos, vel, ic.n1, ic.G, ic.m, ic.D1, d["D2"])
        for key in ("KE", "PE", "E"):
            assert d[key] == pytest.approx(ref[key], rel=1e-12), key
        for key in ("com", "P", "L"):
            scale = {"com": 1.0, "P": ic.m * np.abs(vel).sum(), "L": np.abs(ref["L"]).max()}[key]
            assert np.abs(d[key] - ref[key]).max() <= 1e-12 * scale, key


def test_momentum_and_energy_drift_fp32():
    nb = require_gpu()
    ic = synth.make_binary(8192, 0.5, seed=10)
    s = nb.System.from_ic(ic, mode="kahan", growth_on=False)
    d0 = s.diagnostics(with_pe=True)
    s.step(200)
    d1 = s.diagnostics(with_pe=True)
    vel = s.velocities()
    s.close()
    dP = np.linalg.norm(d1["P"] - d0["P"]) / (ic.m * np.linalg.norm(vel, axis=1).sum())
    dE = abs(d1["E"] - d0["E"]) / abs(d0["E"])
    print("200 steps: dP", dP, "dE", dE)
    assert dP < 1e-5
    assert dE < 1e-4


def test_nonfinite_state_is_flagged():
    nb = require_gpu()
    ic = synth.make_binary(3000, 0.5, seed=12)
    s = nb.System.from_ic(ic, mode="kahan")
    s.x[17] = float("nan")
    s.step(1)
    d = s.diagnostics()
    s.close()
    assert d["status"] == nb.NB_E_NONFINITE
    assert d["nonfinite"] > 0


@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_growth_enters_the_force_one_step_later(mode):
    """Growing and non-growing runs from the same start: bitwise equal after one step (the first
    step's forces use the initial diameter; growth follows the second kick), equal positions
    and different donor velocities after two (the grown diameter first enters the force at the
    end of step 2), as in the oracle."""
    nb = require_gpu()
    ic = synth.make_binary(2048, 0.5, seed=0)
    print_case("growth ordering", mode)
    grow = nb.System.from_ic(ic, mode=mode, growth_on=True)
    keep = nb.System.from_ic(ic, mode=mode, growth_on=False)
    grow.step(1)
    keep.step(1)
    assert np.array_equal(grow.positions(), keep.positions())
    assert np.array_equal(grow.velocities(), keep.velocities())
    assert grow.diagnostics()["D2"] == ic.D2 * (1 + 1e-4)
    assert keep.diagnostics()["D2"] == ic.D2
    grow.step(1)
    keep.step(1)
    assert np.array_equal(grow.positions(), keep.positions())
    dv = np.abs(grow.velocities() - keep.velocities()).max(axis=1)
    grow.close()
    keep.close()
    assert (dv[ic.n1:] > 0).any()


@pytest.mark.parametrize("mode", ["kahan", "plain", "fp64"])
def test_l1_count_ballistic_hand_case(mode):
    """G = 0: straight-line motion. Star 1 at the origin, the donor centre held at x = 1 by two
    elements moving apart, so L1 (q = 0.5) is the plane x = 0.570752; the element leaving
    x = 0.60 at speed 0.05 with dt = 0.01 first lies past it after step 59. The per-step record
    has exactly that one forward crossing (the same case pins the oracle's run)."""
    nb = require_gpu()
    print_case("L1 ballistic", mode)
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.60, 0.0, 0.0], [1.40, 0.0, 0.0]])
    vel = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [-0.05, 0.0, 0.0], [0.05, 0.0, 0.0]])
    s = nb.System(pos, vel, 1, G=0.0, m=1e-3, dt=0.01, D1=0.01, D2=0.01, q=0.5, growth_on=False,
                  mode=mode)
    s.step(80)
    log = s.l1_log(80)
    s.close()
    assert np.array_equal(log[:, 0], np.arange(1, 81))
    past, fwd, bwd = log[:, 1], log[:, 2], log[:, 3]
    assert np.all(past[:58] == 0) and np.all(past[58:] == 1)
    assert fwd[58] == 1 and fwd.sum() == 1 and bwd.sum() == 0


@pytest.mark.parametrize("n1,D1,D2", [(2, 0.1, 0.1), (1, 0.08, 0.12)])
@pytest.mark.parametrize("mode,tol", [("fp64", 1e-12), ("kahan", 5e-6), ("plain", 5e-6)])
def test_contact_oscillation_matches_the_leapfrog_closed_form(mode, tol, n1, D1, D2):
    """Two elements in contact, both in star 1 (D = D1) or one in each star (D = (D1 + D2) / 2),
    moving apart at relative speed v0. Inside D the contact law is affine,
    f = (11 G m^2 / D^3) (r - 10 D / 11), so the separation u = r - r_eq
    obeys u'' = -w^2 u (w^2 = 22 G m / D^3), and the leap-frog map of a linear force is exactly
    u_k = u_0 cos(k theta) + (v_0 dt / sin theta) sin(k theta), cos theta = 1 - (w dt)^2 / 2
    (the oracle meets it to 1.6e-14). Bars, each the worst case of rounding errors adding up in
    one direction: FP64, a few roundings of 0.05-sized positions (1.1e-17 each) per step over
    2000 steps, 1e-13, with margin; FP32, half an ulp of 0.05 (1.9e-9) per step over 2000 steps
    plus the FP32 rounding of 11/D^3 and 10/D^2, about 4e-6 (measured: 1.6e-14 and 1.0e-7;
    amplitude 2.9e-3)."""
    nb = require_gpu()
    print_case("contact oscillator", mode)
    D, m, dt, u0, v0 = 0.1, 1e-3, 1e-3, 0.002, 0.01
    r_eq = 10.0 * D / 11.0
    r0 = r_eq + u0
    pos = np.array([[-0.5 * r0, 0.0, 0.0], [0.5 * r0, 0.0, 0.0]])
    vel = np.array([[-0.5 * v0, 0.0, 0.0], [0.5 * v0, 0.0, 0.0]])
    theta = math.acos(1.0 - 22.0 * m / D ** 3 * dt * dt / 2.0)
    s = nb.System(pos, vel, n1, G=1.0, m=m, dt=dt, D1=D1, D2=D2, q=0.5, growth_on=False,
                  mode=mode)
    done, worst = 0, 0.0
    for k in (1, 250, 1000, 2000):
        s.step(k - done)
        done = k
        p = s.positions().astype(np.float64)
        u = (p[1, 0] - p[0, 0]) - r_eq
        exact = u0 * math.cos(k * theta) + v0 * dt / math.sin(theta) * math.sin(k * theta)
        worst = max(worst, abs(u - exact))
    s.close()
    print("worst |u - closed form| = %.3e" % worst)
    assert worst < tol


def test_l1_log_keeps_the_last_4096_steps():
    """The per-step L1 record is a ring of NB_L1_LOG_CAP = 4096 rows: after 4100 steps the
    oldest rows are gone, the rows come back oldest first with contiguous step numbers, a shorter
    request returns the most recent rows, and the newest row equals the last step's counts that
    nb_diagnostics reports."""
    nb = require_gpu()
    print_case("L1 log ring")
    ic = synth.make_binary(512, 0.5, seed=4)
    s = nb.System.from_ic(ic, mode="kahan", dt=1e-3)
    s.step(4100)
    full = s.l1_log(5000)
    last = s.l1_log(10)
    d = s.diagnostics()
    s.close()
    assert full.shape == (nb.NB_L1_LOG_CAP, 4)
    assert np.array_equal(full[:, 0], np.arange(4100 - 4096 + 1, 4101))
    assert np.array_equal(last, full[-10:])
    assert d["step"] == 4100
    assert tuple(full[-1, 1:]) == (d["n_past_L1"], d["cross_fwd"], d["cross_bwd"])
    # every row is a consistent count: the past count changes by forward minus backward
    assert np.array_equal(np.diff(full[:, 1]), full[1:, 2] - full[1:, 3])


def test_no_growth_when_the_donor_starts_beyond_its_lobe():
    """q = 0.1: r_L = 0.1992 < R2_0 = 0.2, so the first step stops growth and D2 stays D2_0, as
    in the oracle."""
    nb = require_gpu()
    print_case("no growth at q = 0.1")
    ic = synth.make_binary(2048, 0.1, seed=0)
    s = nb.System.from_ic(ic, mode="kahan")
    s.step(1)
    d1 = s.diagnostics()
    s.step(4)
    d5 = s.diagnostics()
    s.close()
    assert d1["growth_stopped"] and d5["growth_stopped"]
    assert d1["D2"] == ic.D2 and d5["D2"] == ic.D2
