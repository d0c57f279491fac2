"""Second, NumPy transcription of the all-pairs acceleration -- TEST INFRASTRUCTURE ONLY.

Vectorised FP64 over a dense (n, n) distance matrix, so only for small n. It exists to catch
coding mistakes in the C oracle (index ranges, signs, the cross-star diameter), not as a pin of
the physics: the physics pins are the closed forms and invariants in tests/test_oracle_*.py.
"""

from __future__ import annotations

import numpy as np


def accel_dense(pos: np.ndarray, n1: int, G: float, m: float, D1: float, D2: float) -> np.ndarray:
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    star = (np.arange(n) >= n1).astype(np.int64)
    Dtab = np.array([[D1, 0.5 * (D1 + D2)], [0.5 * (D1 + D2), D2]])
    D = Dtab[star[:, None], star[None, :]]
    d = pos[None, :, :] - pos[:, None, :]  # d[i, j] = r_j - r_i
    r = np.sqrt((d * d).sum(axis=2))
    valid = r > 0.0
    rs = np.where(valid, r, 1.0)
    newton = G * m * m / rs**2
    K = 10.0 * G * m * m / D**2
    inner = G * m * m * rs / D**3 - K * (1.0 - rs / D)
    f = np.where(rs >= D, newton, inner)
    g = np.where(valid, f / m / rs, 0.0)
    return (g[:, :, None] * d).sum(axis=1)


def accel_dense_paper(pos, vel, n1, G, m, D1, D2, eps, gamma, beta) -> np.ndarray:
    """NumPy transcription of the eqs. (4)-(6) pair sum (small n only)."""
    pos = np.asarray(pos, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    n = pos.shape[0]
    star = (np.arange(n) >= n1).astype(np.int64)
    Dtab = np.array([[D1, 0.5 * (D1 + D2)], [0.5 * (D1 + D2), D2]])
    R = 0.5 * Dtab[star[:, None], star[None, :]]
    d = pos[None, :, :] - pos[:, None, :]
    dv = vel[None, :, :] - vel[:, None, :]
    r = np.sqrt((d * d).sum(axis=2))
    valid = r > 0.0
    rs = np.where(valid, r, 1.0)
    vr = (dv * d).sum(axis=2) / rs
    vol = np.where(rs < 2 * R, np.pi * (4.0 / 3.0 * R**3 - R**2 * rs + rs**3 / 12.0), 0.0)
    g = np.where(vr < 0.0, gamma, gamma * beta)
    f = G * m * m / (rs + eps) ** 2 - g * vol
    coef = np.where(valid, f / m / rs, 0.0)
    return (coef[:, :, None] * d).sum(axis=1)
