"""FP64 CPU oracle for the binary-star element model -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with the GPU library (``paper_2303_12166_amd``) and never imports it.

The arithmetic lives in ``nbody_oracle.c`` (plain C, FP64, OpenMP over rows only); this module
compiles it with gcc and marshals arrays through ctypes. ``np_ref`` holds a second, NumPy
transcription of the all-pairs sum used to cross-check the C code on small inputs.

Pins (tests/test_oracle_*.py): pair-law closed forms (continuity at D, zero at 10D/11, the r->0
limit), Newton far field, dU/dr = f by finite differences, exact antisymmetry and momentum
conservation, two-body Kepler orbits (circular and eccentric, via Kepler's equation), second-order
energy error of the leap-frog, eq. (3) limits, the L1 root's symmetry and Hill limit, the donor
growth stop step in closed form, and hand-placed L1 counts; under eqs. (4)-(6) the lens
volume (closed form and Monte Carlo), elastic and inelastic head-on collisions, and the potential
energy sum against hand-integrated contact energies and a quadrature of the lens volume.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i8p = ctypes.POINTER(ctypes.c_int8)


class OrcState(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("n1", ctypes.c_int64),
        ("G", ctypes.c_double),
        ("m", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("D1", ctypes.c_double),
        ("D2", ctypes.c_double),
        ("q", ctypes.c_double),
        ("a", ctypes.c_double),
        ("R2_0", ctypes.c_double),
        ("D2_0", ctypes.c_double),
        ("growth_rate", ctypes.c_double),
        ("growth_on", ctypes.c_int32),
        ("growth_stopped", ctypes.c_int32),
        ("step", ctypes.c_int64),
        ("law", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("beta", ctypes.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liborc.so``."""
    global _lib
    with _lock:
        if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
            return _LIB
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(_LIB)
            lib.orc_pair_force.restype = ctypes.c_double
            lib.orc_pair_force.argtypes = [ctypes.c_double] * 5
            lib.orc_pair_potential.restype = ctypes.c_double
            lib.orc_pair_potential.argtypes = [ctypes.c_double] * 5
            lib.orc_overlap_volume.restype = ctypes.c_double
            lib.orc_overlap_volume.argtypes = [ctypes.c_double] * 2
            lib.orc_paper_force.restype = ctypes.c_double
            lib.orc_paper_force.argtypes = [ctypes.c_double] * 9
            lib.orc_paper_potential.restype = ctypes.c_double
            lib.orc_paper_potential.argtypes = [ctypes.c_double] * 7
            lib.orc_accel_rows_paper.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int64,
                                                 ctypes.c_int64] + [ctypes.c_double] * 7 + [
                                                 _i64p, ctypes.c_int64, _dp, _dp, _dp]
            lib.orc_paper_pe.restype = ctypes.c_double
            lib.orc_paper_pe.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_int64] + [
                ctypes.c_double] * 6
            lib.orc_roche_lobe.restype = ctypes.c_double
            lib.orc_roche_lobe.argtypes = [ctypes.c_double]
            lib.orc_l1_point.restype = ctypes.c_double
            lib.orc_l1_point.argtypes = [ctypes.c_double]
            lib.orc_max_threads.restype = ctypes.c_int
            lib.orc_set_threads.argtypes = [ctypes.c_int]
            lib.orc_accel_rows.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, _i64p, ctypes.c_int64, _dp, _dp, _dp]
            lib.orc_pair_vector.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int64, ctypes.c_int64, _dp]
            lib.orc_l1_count.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_double, _i8p, ctypes.c_int, _i32p]
            lib.orc_retention.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, _i32p]
            lib.orc_retention.restype = None
            lib.orc_diag.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, _dp]
            lib.orc_run.argtypes = [ctypes.POINTER(OrcState), _dp, _dp, _dp, _dp, _dp, _dp, _i8p,
                                    ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int64,
                                    _i32p, _dp]
            _lib = lib
    return _lib


def _col(a: np.ndarray, k: int) -> np.ndarray:
    return np.ascontiguousarray(a[:, k], dtype=np.float64)


def _p(a: np.ndarray, t=_dp):
    return a.ctypes.data_as(t)


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def pair_force(r: float, D: float, G: float = 1.0, mi: float = 1.0, mj: float = 1.0) -> float:
    """Attractive magnitude of the pair force (negative = repulsion)."""
    return float(_load().orc_pair_force(r, D, G, mi, mj))


def pair_potential(r: float, D: float, G: float = 1.0, mi: float = 1.0, mj: float = 1.0) -> float:
    return float(_load().orc_pair_potential(r, D, G, mi, mj))


def overlap_volume(r: float, R: float) -> float:
    """Lens volume of two spheres of radius R at centre distance r (eqs. 5-6, read with r^3/12)."""
    return float(_load().orc_overlap_volume(r, R))


def paper_force(r: float, vr: float, R: float, G: float = 1.0, mi: float = 1.0, mj: float = 1.0,
                eps: float = 0.0, gamma: float = 0.0, beta: float = 1.0) -> float:
    """Attractive magnitude of eqs. (4)-(6); vr < 0 means the pair converges."""
    return float(_load().orc_paper_force(r, vr, R, G, mi, mj, eps, gamma, beta))


def paper_potential(r: float, R: float, G: float = 1.0, mi: float = 1.0, mj: float = 1.0,
                    eps: float = 0.0, gamma: float = 0.0) -> float:
    return float(_load().orc_paper_potential(r, R, G, mi, mj, eps, gamma))


def accel_paper(pos, vel, n1, G, m, D1, D2, eps, gamma, beta, rows=None) -> np.ndarray:
    """All-pairs acceleration under eqs. (4)-(6); returns (k, 3) float64."""
    lib = _load()
    pos = np.asarray(pos, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    n = pos.shape[0]
    cols = [_col(pos, 0), _col(pos, 1), _col(pos, 2), _col(vel, 0), _col(vel, 1), _col(vel, 2)]
    if rows is None:
        k, rp = n, None
    else:
        rr = np.ascontiguousarray(rows, dtype=np.int64)
        if rr.size and (rr.min() < 0 or rr.max() >= n):
            raise IndexError("row index out of range")
        k, rp = rr.size, _p(rr, _i64p)
    ax, ay, az = np.zeros(k), np.zeros(k), np.zeros(k)
    if k:
        lib.orc_accel_rows_paper(*[_p(c) for c in cols], n, int(n1), G, m, D1, D2, eps, gamma,
                                 beta, rp, k, _p(ax), _p(ay), _p(az))
    return np.stack([ax, ay, az], axis=1)


def paper_pe(pos, n1, G, m, D1, D2, eps, gamma) -> float:
    lib = _load()
    pos = np.asarray(pos, dtype=np.float64)
    cols = [_col(pos, 0), _col(pos, 1), _col(pos, 2)]
    return float(lib.orc_paper_pe(*[_p(c) for c in cols], pos.shape[0], int(n1), G, m, D1, D2,
                                  eps, gamma))


def roche_lobe(q: float) -> float:
    """eq. (3): Roche-lobe radius over separation for mass ratio q."""
    return float(_load().orc_roche_lobe(q))


def l1_point(q: float) -> float:
    """Distance of L1 from the accretor in units of the separation."""
    return float(_load().orc_l1_point(q))


def accel(pos: np.ndarray, n1: int, G: float, m: float, D1: float, D2: float,
          rows=None) -> np.ndarray:
    """All-pairs acceleration for the given rows (all rows if None); returns (k, 3) float64."""
    lib = _load()
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    x, y, z = _col(pos, 0), _col(pos, 1), _col(pos, 2)
    if rows is None:
        k = n
        rp = None
        rr = None
    else:
        rr = np.ascontiguousarray(rows, dtype=np.int64)
        if rr.size and (rr.min() < 0 or rr.max() >= n):
            raise IndexError("row index out of range")
        k = rr.size
        rp = _p(rr, _i64p)
    ax, ay, az = np.zeros(k), np.zeros(k), np.zeros(k)
    if k:
        lib.orc_accel_rows(_p(x), _p(y), _p(z), n, int(n1), G, m, D1, D2, rp, k,
                           _p(ax), _p(ay), _p(az))
    return np.stack([ax, ay, az], axis=1)


def pair_vector(pos: np.ndarray, n1: int, G: float, m: float, D1: float, D2: float,
                i: int, j: int) -> np.ndarray:
    lib = _load()
    pos = np.asarray(pos, dtype=np.float64)
    x, y, z = _col(pos, 0), _col(pos, 1), _col(pos, 2)
    out = np.zeros(3)
    lib.orc_pair_vector(_p(x), _p(y), _p(z), int(n1), G, m, D1, D2, int(i), int(j), _p(out))
    return out


def l1_count(pos: np.ndarray, n1: int, q: float, side=None, init: bool = False):
    """Returns (n_past, forward, backward); ``side`` (int8, n) is updated in place if given."""
    lib = _load()
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    x, y, z = _col(pos, 0), _col(pos, 1), _col(pos, 2)
    out = np.zeros(3, dtype=np.int32)
    sp = None
    if side is not None:
        if side.dtype != np.int8 or not side.flags.c_contiguous or side.shape != (n,):
            raise ValueError("side must be a contiguous int8 array of length n")
        sp = _p(side, _i8p)
    lib.orc_l1_count(_p(x), _p(y), _p(z), n, int(n1), q, sp, int(bool(init)), _p(out, _i32p))
    return int(out[0]), int(out[1]), int(out[2])


def retention(pos: np.ndarray, vel: np.ndarray, n1: int, G: float, m: float, q: float):
    """Returns (n_past, n_bound): donor elements past L1, and those of them bound to the accretor."""
    lib = _load()
    pos = np.asarray(pos, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    n = pos.shape[0]
    cols = [_col(pos, 0), _col(pos, 1), _col(pos, 2), _col(vel, 0), _col(vel, 1), _col(vel, 2)]
    out = np.zeros(2, dtype=np.int32)
    lib.orc_retention(*[_p(c) for c in cols], n, int(n1), G, m, q, _p(out, _i32p))
    return int(out[0]), int(out[1])


def diag(pos: np.ndarray, vel: np.ndarray, n1: int, G: float, m: float, D1: float, D2: float,
         with_pe: bool = True) -> dict:
    lib = _load()
    pos = np.asarray(pos, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    n = pos.shape[0]
    cols = [_col(pos, 0), _col(pos, 1), _col(pos, 2), _col(vel, 0), _col(vel, 1), _col(vel, 2)]
    out = np.zeros(12)
    lib.orc_diag(*[_p(c) for c in cols], n, int(n1), G, m, D1, D2, int(bool(with_pe)), _p(out))
    return {"com": out[0:3].copy(), "P": out[3:6].copy(), "L": out[6:9].copy(),
            "KE": float(out[9]), "PE": float(out[10]), "E": float(out[11])}


class Run:
    """FP64 kick-drift-kick run with donor growth and L1 counting."""

    def __init__(self, pos, vel, n1, G, m, dt, D1, D2, q, a=1.0, R2_0=0.2, growth_rate=1e-4,
                 growth_on=True, D2_0=None, law=0, eps=0.0, gamma=0.0, beta=1.0):
        pos = np.asarray(pos, dtype=np.float64)
        vel = np.asarray(vel, dtype=np.float64)
        self.n = pos.shape[0]
        self.cols = [_col(pos, 0), _col(pos, 1), _col(pos, 2),
                     _col(vel, 0), _col(vel, 1), _col(vel, 2)]
        self.side = np.zeros(self.n, dtype=np.int8)
        # acceleration of the current state, carried from one advance() to the next
        self.acc = [np.zeros(max(self.n, 1)) for _ in range(3)]
        self.state = OrcState(n=self.n, n1=int(n1), G=G, m=m, dt=dt, D1=D1, D2=D2, q=q, a=a,
                              R2_0=R2_0, D2_0=D2 if D2_0 is None else D2_0,
                              growth_rate=growth_rate, growth_on=int(bool(growth_on)),
                              growth_stopped=0, step=0, law=int(law), pad=0, eps=eps,
                              gamma=gamma, beta=beta)
        self._inited = False

    def advance(self, steps: int):
        """Returns (counts (steps, 3) int32, d2_log (steps,) float64)."""
        lib = _load()
        counts = np.zeros((max(steps, 1), 3), dtype=np.int32)
        d2 = np.zeros(max(steps, 1))
        lib.orc_run(ctypes.byref(self.state), *[_p(c) for c in self.cols], _p(self.side, _i8p),
                    int(not self._inited), *[_p(a) for a in self.acc], int(self._inited),
                    int(steps), _p(counts, _i32p), _p(d2))
        self._inited = True
        return counts[:steps], d2[:steps]

    @property
    def pos(self) -> np.ndarray:
        return np.stack(self.cols[0:3], axis=1)

    @property
    def vel(self) -> np.ndarray:
        return np.stack(self.cols[3:6], axis=1)

    @property
    def D2(self) -> float:
        return float(self.state.D2)

    @property
    def growth_stopped(self) -> bool:
        return bool(self.state.growth_stopped)
