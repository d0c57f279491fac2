"""Edge cases of the GPU path: an empty system alone and inside a batch, the largest size tried
(N = 1,048,576: bands of four tile rows by the built-in rule, about 9.5 GB of workspace in Kahan
mode) against the oracle on sampled rows, a system whose stars are both a single element, and
the sorted layout the force kernels work in."""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import force_error, print_case, require_gpu, sample_rows

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["plain", "kahan", "fp64"])
def test_empty_system(mode):
    nb = require_gpu()
    print_case("empty system", mode)
    z = np.zeros((0, 3))
    s = nb.System(z, z, 0, G=1.0, m=1e-3, dt=1e-4, D1=0.01, D2=0.01, q=0.5, mode=mode)
    s.forces()
    s.step(3)
    d = s.diagnostics(with_pe=True)
    assert d["step"] == 3 and d["nonfinite"] == 0 and d["n_past_L1"] == 0
    assert d["KE"] == 0.0 and d["PE"] == 0.0
    assert s.retention() == (0, 0)
    assert s.positions().shape == (0, 3)
    s.close()


@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_empty_system_inside_a_batch(mode):
    nb = require_gpu()
    print_case("empty system in batch", mode)
    ic = synth.make_binary(3000, 0.5, seed=8)
    z = np.zeros((0, 3))

    def empty():
        return nb.System(z, z, 0, G=1.0, m=1e-3, dt=1e-4, D1=0.01, D2=0.01, q=0.5, mode=mode)

    alone = nb.System.from_ic(ic, mode=mode)
    alone.step(6)
    e1, full, e2 = empty(), nb.System.from_ic(ic, mode=mode), empty()
    nb.step_many([e1, full, e2], 6)
    assert np.array_equal(alone.positions(), full.positions())
    assert np.array_equal(alone.velocities(), full.velocities())
    assert e1.diagnostics()["step"] == 6 and e2.diagnostics()["step"] == 6
    for s in (alone, e1, full, e2):
        s.close()


@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_one_element_per_star(mode):
    nb = require_gpu()
    print_case("one element per star", mode)
    pos = np.array([[-0.3, 0.0, 0.0], [0.7, 0.0, 0.0]])
    vel = np.array([[0.0, -0.5, 0.0], [0.0, 1.0, 0.0]])
    s = nb.System(pos, vel, 1, G=1.0, m=0.5, dt=1e-4, D1=0.05, D2=0.04, q=0.5, mode=mode)
    a = s.accelerations()
    s.close()
    ref = oracle.accel(pos, 1, 1.0, 0.5, 0.05, 0.04)
    assert force_error(a, ref) <= (1e-6 if mode == "kahan" else 1e-14)
    # Newton: equal and opposite
    assert np.allclose(a[0], -a[1], rtol=1e-6, atol=0)


def test_largest_size_sampled_rows_kahan():
    nb = require_gpu()
    n, q = 1048576, 0.5
    ic = synth.make_binary(n, q, seed=0)
    print_case("largest size", n, q)
    s = nb.System.from_ic(ic, mode="kahan")
    a = s.accelerations()
    s.close()
    rows = sample_rows(n, ic.n1, 64, seed=3)
    p, _ = ic.f32_as_f64()
    ref = oracle.accel(p, ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)
    err = force_error(a[rows], ref)
    print("N=1048576 kahan max rel err", err)
    assert err <= 1e-5


@pytest.mark.parametrize("law", ["contact", "paper", "paper-eps0"])
@pytest.mark.parametrize("mode", ["kahan", "fp64"])
def test_coincident_elements(mode, law):
    """Distinct elements at exactly the same position (in different tiles and in the same tile):
    the pair has d = 0 and contributes nothing, as the oracle's r = 0 rule says; nothing becomes
    non-finite. "paper-eps0" takes eqs. (4)-(6) without softening, where the pair scalar of
    coincident elements is largest."""
    nb = require_gpu()
    ic = synth.with_velocity_noise(synth.make_binary(1500, 0.5, seed=5), 0.05, 1005)
    p, v = ic.f32()
    p = p.copy()
    p[700] = p[3]        # same star, far apart in the sorted order
    p[1400] = p[1401]    # donor, neighbours
    p[1100] = p[10]      # across the stars' index ranges
    kw = synth.paper_law_params(ic) if law != "contact" else {}
    if law == "paper-eps0":
        kw["eps"] = 0.0
    print_case("coincident elements", mode, law)
    cast = np.float64 if mode == "fp64" else np.float32
    s = nb.System(p.astype(cast), v.astype(cast), ic.n1, G=ic.G, m=ic.m, dt=1e-4, D1=ic.D1,
                  D2=ic.D2, q=ic.q, mode=mode, **kw)
    a = s.accelerations()
    s.step(2)
    d = s.diagnostics()
    s.close()
    assert np.isfinite(a).all() and d["nonfinite"] == 0
    p64, v64 = p.astype(np.float64), v.astype(np.float64)
    if law != "contact":
        ref = oracle.accel_paper(p64, v64, ic.n1, ic.G, ic.m, ic.D1, ic.D2, kw["eps"],
                                 kw["gamma"], kw["beta"])
    else:
        ref = oracle.accel(p64, ic.n1, ic.G, ic.m, ic.D1, ic.D2)
    assert force_error(a, ref) <= (1e-5 if mode == "kahan" else 1e-11)


def test_create_refuses_host_memory():
    """Buffers in pinned host memory (device-accessible, so a missed check would not fault) are
    refused by nb_create with NB_E_INVAL before any copy or launch, the failed pointer query
    leaves no error behind for the next HIP call, and a valid system builds afterwards."""
    nb = require_gpu()
    import torch

    print_case("host buffers refused")
    ic = synth.make_binary(600, 0.5, seed=12)
    p = nb.NbParams(n=ic.n, n1=ic.n1, G=ic.G, m=ic.m, dt=1e-4, D1=ic.D1, D2=ic.D2, q=ic.q, a=1.0,
                    R2_0=0.2, growth_rate=1e-4, growth_on=1, mode=nb.NB_FP32_KAHAN, law=0, pad=0,
                    eps=0.0, gamma=0.0, beta=1.0)
    nbytes = nb.nb_scratch_bytes(p)
    dev = [torch.zeros(ic.n, dtype=torch.float32, device="cuda") for _ in range(9)]
    host = [torch.zeros(ic.n, dtype=torch.float32, pin_memory=True) for _ in range(9)]
    side_d = torch.zeros(ic.n, dtype=torch.int8, device="cuda")
    side_h = torch.zeros(ic.n, dtype=torch.int8, pin_memory=True)
    scr_d = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    scr_h = torch.empty(nbytes + 256, dtype=torch.uint8, pin_memory=True)

    def bufs(arrays, side, scr):
        base = scr.data_ptr()
        names = ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az")
        kw = {k: t.data_ptr() for k, t in zip(names, arrays)}
        return nb.NbBuffers(side=side.data_ptr(), scratch=base + (-base) % 256,
                            scratch_bytes=nbytes, **kw)

    for arrays, side, scr in ((host, side_d, scr_d), (dev[:3] + host[3:], side_d, scr_d),
                              (dev, side_h, scr_d), (dev, side_d, scr_h)):
        with pytest.raises(nb.NbError) as e:
            nb.nb_create(p, bufs(arrays, side, scr))
        assert e.value.status == nb.NB_E_INVAL
    torch.cuda.synchronize()
    (dev[0] + 1.0).sum().item()  # no stale HIP error surfaces in torch
    s = nb.System.from_ic(ic, mode="kahan")
    a = s.accelerations()
    s.close()
    assert np.isfinite(a).all()


def test_force_timing_counts_exactly_the_timed_launches():
    """nb_timing_*: while enabled, each force launch of nb_forces and nb_step is timed once;
    nothing is counted while disabled, graph replays are not counted, and a reset clears the
    totals."""
    nb = require_gpu()
    print_case("force timing")
    ic = synth.make_binary(4096, 0.5, seed=2)
    s = nb.System.from_ic(ic, mode="kahan")
    nb.nb_timing_reset()
    nb.nb_timing_enable(True)
    s.forces()
    s.forces()
    s.step(3)
    g = nb.nb_graph_create([s.handle], 2, s.stream)
    nb.nb_graph_launch(g, s.stream)
    nb.nb_timing_enable(False)
    s.forces()
    s.step(2)
    s.synchronize()
    ms, n = nb.nb_timing_read()
    nb.nb_graph_destroy(g)
    s.close()
    assert n == 5
    assert 0.0 < ms < 1000.0
    nb.nb_timing_reset()
    assert nb.nb_timing_read() == (0.0, 0)


@pytest.mark.parametrize("n,q", [(3001, 0.3), (700, 0.9), (1, 0.5)])
def test_sorted_order_is_a_per_star_permutation(n, q):
    """nb_sorted_order: star 1's elements fill slots [0, n1) and star 2's start at
    roundup(n1, 256), each exactly once, every other slot is padding (-1), and the slot count is
    a whole number of 256-slot tiles."""
    nb = require_gpu()
    ic = synth.make_binary(n, q, seed=3)
    print_case("sorted order", n, q)
    s = nb.System.from_ic(ic, mode="kahan")
    perm = nb.nb_sorted_order(s.handle, s.stream)
    s.close()
    n1 = ic.n1
    p1 = -(-n1 // 256) * 256
    n2 = n - n1
    assert perm.size == p1 + -(-n2 // 256) * 256 and perm.size % 256 == 0
    assert sorted(perm[:n1].tolist()) == list(range(n1))
    assert np.all(perm[n1:p1] == -1)
    assert sorted(perm[p1:p1 + n2].tolist()) == list(range(n1, n))
    assert np.all(perm[p1 + n2:] == -1)
