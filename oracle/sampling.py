"""FP64 oracle of the orientation samplers (Sec. IV-C of the paper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module; the HIP path never does.

* Quaternion distance d(q1, q2) = arccos |<q1, q2>| (half the relative rotation
  angle) and the geodesic ball B(q0, theta) = {q : d(q, q0) <= theta}.
* Global sampler: the Super-Fibonacci sequence the paper adopts (the cited
  construction): for s = i + 1/2, r = sqrt(s/n), R = sqrt(1 - s/n),
  alpha = 2 pi s / phi, beta = 2 pi s / psi,
  q = (r sin alpha, r cos alpha, R sin beta, R cos beta), with phi = sqrt 2
  and psi the real root of psi^4 = psi + 4 above 1.
* Local sampler GeoBall-SF (Alg. geoball-sf): in coordinates
  q = (R cos a, R sin a, r cos b, r sin b), R = sqrt(1 - r^2), the ball around
  the identity is cos a >= cos(theta) / R, i.e. |a| <= L(r) / 2 with
  L(r) = 2 arccos(cos theta / R), and the uniform measure on S^3 is
  r dr da db.  The radius therefore has density rho(r) ~ r L(r) on
  [0, sin theta]; its distribution function F is tabulated numerically on a
  uniform grid of r (cumulative trapezoid rule) and inverted by linear
  interpolation.  The sample is q0 * q_local.

Readings taken (listed in the design notes): the paper leaves gamma undefined;
the default is gamma = n, which keeps the Super-Fibonacci stratification s/n of
the radial coordinate.  gamma is a parameter: gamma = 1.3247 (the plastic
number) reproduces the paper's 0.7 deg mean nearest-neighbour spacing at
n = 5000, theta = 5 deg, gamma = n gives 0.57 deg.  The radial table has
TABLE_POINTS points.
"""
from __future__ import annotations

import math

import numpy as np

PHI = math.sqrt(2.0)
TABLE_POINTS = 4096


def _psi() -> float:
    """Real root above 1 of x^4 = x + 4 (Newton from 1.5)."""
    x = 1.5
    for _ in range(60):
        x -= (x ** 4 - x - 4.0) / (4.0 * x ** 3 - 1.0)
    return x


PSI = _psi()


def quat_mul(a, b) -> np.ndarray:
    """Hamilton product, scalar first; broadcasts over leading axes."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    w1, x1, y1, z1 = np.moveaxis(a, -1, 0)
    w2, x2, y2, z2 = np.moveaxis(b, -1, 0)
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def quat_distance(q1, q2) -> np.ndarray:
    """d(q1, q2) = arccos |<q1, q2>| (radians), for unit quaternions."""
    dot = np.abs(np.sum(np.asarray(q1, dtype=np.float64) * np.asarray(q2, dtype=np.float64), axis=-1))
    return np.arccos(np.clip(dot, -1.0, 1.0))


def super_fibonacci(n: int) -> np.ndarray:
    """n unit quaternions (scalar first) of the Super-Fibonacci sequence."""
    s = np.arange(n, dtype=np.float64) + 0.5
    r = np.sqrt(s / n)
    R = np.sqrt(1.0 - s / n)
    alpha = 2.0 * math.pi * s / PHI
    beta = 2.0 * math.pi * s / PSI
    return np.stack([r * np.sin(alpha), r * np.cos(alpha), R * np.sin(beta), R * np.cos(beta)], axis=1)


def admissible_angle(r, theta: float) -> np.ndarray:
    """L(r) = 2 arccos(cos theta / sqrt(1 - r^2)): the range of the axial angle a
    at radius r inside B(1, theta) (zero at r = sin theta)."""
    r = np.asarray(r, dtype=np.float64)
    return 2.0 * np.arccos(np.clip(math.cos(theta) / np.sqrt(1.0 - r * r), -1.0, 1.0))


def radial_table(theta: float, points: int = TABLE_POINTS):
    """(r_j, F(r_j)): F(r) = int_0^r rho / Z with rho(r) = r L(r), on a uniform
    grid of [0, sin theta] by the cumulative trapezoid rule, F(sin theta) = 1."""
    r = np.linspace(0.0, math.sin(theta), points)
    rho = r * admissible_angle(r, theta)
    F = np.concatenate([[0.0], np.cumsum(0.5 * (rho[1:] + rho[:-1]) * np.diff(r))])
    return r, F / F[-1]


def geoball_sf(n: int, q0, theta: float, gamma: float | None = None) -> np.ndarray:
    """n unit quaternions (scalar first) in B(q0, theta) by GeoBall-SF."""
    g = float(n) if gamma is None else float(gamma)
    q0 = np.asarray(q0, dtype=np.float64)
    q0 = q0 / np.linalg.norm(q0)
    r_t, F_t = radial_table(theta)
    s = np.arange(n, dtype=np.float64) + 0.5
    u1 = np.mod(s / g, 1.0)
    u2 = np.mod(s / PHI, 1.0)
    u3 = np.mod(s / PSI, 1.0)
    r = np.interp(u1, F_t, r_t)
    R = np.sqrt(1.0 - r * r)
    a = (u2 - 0.5) * admissible_angle(r, theta)
    b = 2.0 * math.pi * u3
    local = np.stack([R * np.cos(a), R * np.sin(a), r * np.cos(b), r * np.sin(b)], axis=1)
    return quat_mul(q0, local)


def ball_volume_fraction(t, theta: float) -> np.ndarray:
    """Share of the uniform measure of B(q0, theta) within distance t of q0: the
    volume of a geodesic ball of radius t on S^3 is pi (2 t - sin 2 t)."""
    t = np.asarray(t, dtype=np.float64)
    return (2.0 * t - np.sin(2.0 * t)) / (2.0 * theta - math.sin(2.0 * theta))


def mean_nn_rotation_angle(q) -> float:
    """Mean over the samples of the rotation angle (2 d) to the nearest other
    sample (q and -q are the same rotation), by brute force."""
    q = np.asarray(q, dtype=np.float64)
    best = np.zeros(len(q))
    for i0 in range(0, len(q), 512):
        dots = np.abs(q[i0:i0 + 512] @ q.T)
        for j in range(dots.shape[0]):
            dots[j, i0 + j] = -1.0
        best[i0:i0 + 512] = dots.max(axis=1)
    return float(np.mean(2.0 * np.arccos(np.clip(best, -1.0, 1.0))))
