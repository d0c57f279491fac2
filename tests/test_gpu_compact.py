"""Compact-accretor systems (unequal radii and element diameters per star) on the GPU.

A white-dwarf-like accretor (R1 = 0.02-0.03, so D1 is an order of magnitude below D2) packs star
1's elements into a few tiles whose boxes all overlap: nearly every star-1 tile is near, nearly
every cross tile is far. Forces against the FP64 oracle at the usual bars (1e-5 FP32 Kahan,
1e-12 FP64), for both element laws, and a short trajectory.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import force_error, print_case, require_gpu, sample_rows

pytestmark = pytest.mark.gpu

TOL = {"kahan": 1e-5, "fp64": 1e-12}


@pytest.mark.parametrize("mode", ["kahan", "fp64"])
@pytest.mark.parametrize("R1", [0.02, 0.05])
def test_compact_accretor_every_row(mode, R1):
    nb = require_gpu()
    ic = synth.make_binary(4096, 0.6, seed=13, R1=R1, R2=0.35)
    print_case("compact accretor", mode, R1)
    s = nb.System.from_ic(ic, mode=mode)
    a = s.accelerations()
    s.close()
    p, _ = ic.f32_as_f64()
    ref = oracle.accel(p, ic.n1, ic.G, ic.m, ic.D1, ic.D2)
    err = force_error(a, ref)
    print("compact", mode, R1, "D1/D2", ic.D1 / ic.D2, "err", err)
    assert err <= TOL[mode]


def test_compact_accretor_sampled_rows_n131072():
    nb = require_gpu()
    ic = synth.make_binary(131072, 0.8, seed=17, R1=0.03, R2=0.3)
    print_case("compact accretor N=131072 kahan")
    s = nb.System.from_ic(ic, mode="kahan")
    a = s.accelerations()
    s.close()
    p, _ = ic.f32_as_f64()
    rows = sample_rows(ic.n, ic.n1, 128, seed=2)
    ref = oracle.accel(p, ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)
    err = force_error(a[rows], ref)
    print("compact N=131072 err", err)
    assert err <= TOL["kahan"]


@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_compact_accretor_paper_law(mode):
    nb = require_gpu()
    ic = synth.with_velocity_noise(synth.make_binary(3000, 0.5, seed=19, R1=0.03, R2=0.3),
                                   0.05, 1019)
    kw = synth.paper_law_params(ic)
    print_case("compact accretor paper law", mode)
    s = nb.System.from_ic(ic, mode=mode, **kw)
    a = s.accelerations()
    s.close()
    if mode == "fp64":
        p, v = ic.f32_as_f64()
    else:
        p, v = (x.astype(np.float64) for x in ic.f32())
    ref = oracle.accel_paper(p, v, ic.n1, ic.G, ic.m, ic.D1, ic.D2, kw["eps"], kw["gamma"],
                             kw["beta"])
    err = force_error(a, ref)
    print("compact paper", mode, "err", err)
    assert err <= {"kahan": 1e-5, "fp64": 1e-11}[mode]


@pytest.mark.parametrize("mode,xtol", [("kahan", 1e-5), ("fp64", 1e-11)])
def test_compact_accretor_trajectory(mode, xtol):
    nb = require_gpu()
    ic = synth.make_binary(2048, 0.5, seed=23, R1=0.03, R2=0.3)
    print_case("compact accretor trajectory", mode)
    s = nb.System.from_ic(ic, mode=mode)
    s.step(50)
    xg = s.positions()
    s.close()
    p, v = ic.f32_as_f64()
    run = oracle.Run(p, v, ic.n1, ic.G, ic.m, 1e-4, ic.D1, ic.D2, ic.q, a=ic.a, R2_0=ic.R2)
    run.advance(50)
    dx = np.abs(xg - run.pos).max()
    print("compact trajectory", mode, "max|dx|", dx)
    assert dx <= xtol * ic.a
