"""Two-star initial conditions for the element model (Methodology section).

A star is a ball of N_k elements of one common mass and one common diameter. The element mass is
the star mass over the element count, and the diameter follows from the packing of the ball; both
rules come from the paragraph of the Methodology section that sets up the binary.

Recipe (fixed here because the paper gives no sampling procedure):

* counts: N2 = floor(N q / (1 + q)), N1 = N - N2 (star 1 = accretor of mass 1, star 2 = donor of
  mass q, q = m2/m1 as in the definition next to eq. 3);
* every element has mass m = (1 + q) / N, so the total mass is exactly 1 + q;
* element diameter per star: D_k = 2 R_k (0.74 / N_k)^(1/3) (spheres at 74 % packing fill the
  ball); cross-star pairs use (D1 + D2) / 2;
* positions: ``numpy.random.Generator(PCG64(seed))``, star 1 then star 2. Per star draw an
  (N_k, 3) block of standard normals (directions, normalised), then N_k uniforms u; the radius is
  R_k u^(1/3). The sample mean is subtracted and the star centre added, so each star's centre of
  mass sits exactly on its centre: c1 = -a M2 / (M1 + M2), c2 = +a M1 / (M1 + M2) on the x axis;
* velocities: rigid rotation about the barycentre at the circular-orbit rate
  omega = sqrt(G (1 + q) / a^3), i.e. v = omega z_hat x r (orbit plus co-rotation).

Everything is float64. Consumers that run in FP32 round once with :meth:`BinaryIC.f32` and the
oracle is handed those same rounded values promoted back to float64.
"""

from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

PACKING = 0.74


def particle_counts(n: int, q: float) -> tuple[int, int]:
    """Element counts (N1, N2) of accretor and donor, proportional to mass."""
    if n < 0:
        raise ValueError("n must be >= 0")
    n2 = int(math.floor(n * q / (1.0 + q)))
    return n - n2, n2


def element_diameter(radius: float, count: int, packing: float = PACKING) -> float:
    """Common element diameter of a ball of ``count`` elements filling ``radius`` at ``packing``."""
    if count <= 0:
        return 2.0 * radius
    return 2.0 * radius * (packing / count) ** (1.0 / 3.0)


def orbital_omega(q: float, a: float = 1.0, G: float = 1.0) -> float:
    """Circular-orbit angular rate of two point masses 1 and q at separation a."""
    return math.sqrt(G * (1.0 + q) / a**3)


@dataclasses.dataclass
class BinaryIC:
    n: int
    n1: int
    q: float
    G: float
    a: float
    R1: float
    R2: float
    m: float
    D1: float
    D2: float
    omega: float
    seed: int
    pos: np.ndarray  # (n, 3) float64
    vel: np.ndarray  # (n, 3) float64

    @property
    def n2(self) -> int:
        return self.n - self.n1

    def f32(self) -> tuple[np.ndarray, np.ndarray]:
        """Positions and velocities rounded once to float32, as (n, 3) arrays."""
        return self.pos.astype(np.float32), self.vel.astype(np.float32)

    def f32_as_f64(self) -> tuple[np.ndarray, np.ndarray]:
        """The float32-rounded state promoted back to float64 (what the oracle consumes)."""
        p, v = self.f32()
        return p.astype(np.float64), v.astype(np.float64)

    def checksum(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.pos).tobytes())
        h.update(np.ascontiguousarray(self.vel).tobytes())
        return h.hexdigest()


def _uniform_ball(rng: np.random.Generator, count: int, radius: float) -> np.ndarray:
    if count == 0:
        return np.zeros((0, 3))
    d = rng.standard_normal((count, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = rng.random(count)
    return d * (radius * np.cbrt(u))[:, None]


def make_binary(
    n: int,
    q: float,
    seed: int = 0,
    R1: float = 0.30,
    R2: float = 0.20,
    a: float = 1.0,
    G: float = 1.0,
) -> BinaryIC:
    """Draw a two-star system of ``n`` elements with mass ratio ``q`` (see module docstring)."""
    if not (q > 0.0):
        raise ValueError("q must be > 0")
    n1, n2 = particle_counts(n, q)
    m = (1.0 + q) / n if n > 0 else 0.0
    M1, M2 = n1 * m, n2 * m
    Mt = M1 + M2
    c1 = -a * M2 / Mt if Mt > 0 else 0.0
    c2 = a * M1 / Mt if Mt > 0 else 0.0
    rng = np.random.Generator(np.random.PCG64(seed))
    stars = []
    for count, radius, cx in ((n1, R1, c1), (n2, R2, c2)):
        p = _uniform_ball(rng, count, radius)
        if count:
            p -= p.mean(axis=0)
            p[:, 0] += cx
        stars.append(p)
    pos = np.concatenate(stars, axis=0) if n else np.zeros((0, 3))
    omega = orbital_omega(q, a, G)
    vel = np.zeros_like(pos)
    vel[:, 0] = -omega * pos[:, 1]
    vel[:, 1] = omega * pos[:, 0]
    return BinaryIC(
        n=n,
        n1=n1,
        q=q,
        G=G,
        a=a,
        R1=R1,
        R2=R2,
        m=m,
        D1=element_diameter(R1, n1),
        D2=element_diameter(R2, n2),
        omega=omega,
        seed=seed,
        pos=pos,
        vel=vel,
    )


def with_velocity_noise(ic: BinaryIC, sigma: float, seed: int) -> BinaryIC:
    """A copy of ``ic`` whose velocities carry extra isotropic Gaussian noise of std ``sigma``.

    Rigid rotation gives every pair exactly zero radial relative velocity, which would leave the
    converging/separating choice of eqs. (5)-(6) to rounding; the noise gives each pair a definite
    sign. Drawn from PCG64(seed), independent of the positions' stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    vel = ic.vel + sigma * rng.standard_normal(ic.vel.shape)
    return dataclasses.replace(ic, vel=vel)


def paper_law_params(ic: BinaryIC, strength: float = 200.0, beta: float = 0.5,
                     eps_frac: float = 0.1) -> dict:
    """Parameters of the eqs. (4)-(6) element law for the system ``ic`` (an input recipe).

    The paper gives no values. gamma = strength G m^2 / (D1^2 pi R^3), R = D1 / 2, and
    eps = eps_frac D1. With the defaults the net pair force is repulsive from r = 0 up to a single
    equilibrium near 0.95 D1 (0.93 D1 for separating pairs at beta = 1/2) and attractive beyond,
    like the contact law's 10 D / 11; a much weaker gamma or smaller eps lets the softened
    attraction win at small r, so close pairs collapse towards r ~ eps.
    """
    R = 0.5 * ic.D1
    gamma = strength * ic.G * ic.m * ic.m / (ic.D1 ** 2 * math.pi * R ** 3) if ic.n else 0.0
    return {"law": "paper", "eps": eps_frac * ic.D1, "gamma": gamma, "beta": beta}
