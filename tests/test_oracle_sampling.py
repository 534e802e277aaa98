"""Pins of the orientation-sampler oracle (Sec. IV-C) against what the paper
and the geometry of S^3 fix:

* the constants: phi^2 = 2, psi^4 = psi + 4;
* the uniform law on S^3: the share of Super-Fibonacci rotations within
  rotation angle 2t of any fixed rotation is (2t - sin 2t) / pi;
* the uniform law in the geodesic ball: the share of GeoBall-SF samples within
  distance t of q0 is (2t - sin 2t) / (2 theta - sin 2 theta), with every
  sample inside B(q0, theta) -- a wrong radial density or a wrong admissible
  axial angle breaks this law (both are planted below);
* the paper's printed spacings (Results): mean nearest-neighbour rotation
  angle 8.0 deg for 20000 global samples and 0.7 deg for 5000 local samples at
  theta = 5 deg (the latter with gamma = the plastic number, see the module's
  readings);
* the radial distribution function against an independent quadrature.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import sampling as S

PLASTIC = 1.324717957244746


def _ks(sample, cdf):
    x = np.sort(sample)
    emp = (np.arange(len(x)) + 0.5) / len(x)
    return float(np.max(np.abs(emp - cdf(x))))


def test_constants():
    assert abs(S.PHI ** 2 - 2.0) < 1e-15
    assert abs(S.PSI ** 4 - S.PSI - 4.0) < 1e-12 and S.PSI > 1.5


def test_super_fibonacci_is_uniform_on_s3():
    q = S.super_fibonacci(20000)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-14)
    rng = np.random.default_rng(3)
    for _ in range(3):
        c = rng.normal(size=4)
        c /= np.linalg.norm(c)
        d = S.quat_distance(q, c)   # in [0, pi/2]; rotation angle 2d
        ks = _ks(d, lambda t: (2 * t - np.sin(2 * t)) / math.pi)
        # a random set of this size has KS ~ 0.01; low discrepancy does better
        assert ks < 0.005, ks


def test_super_fibonacci_spacing_matches_the_paper():
    # 8.0 deg at 20000 samples (Results)
    spacing = math.degrees(S.mean_nn_rotation_angle(S.super_fibonacci(20000)))
    assert abs(spacing - 8.0) < 0.4, spacing


@pytest.mark.parametrize("gamma", [None, PLASTIC])
@pytest.mark.parametrize("theta_deg", [5.0, 20.0])
def test_geoball_samples_fill_the_ball_uniformly(gamma, theta_deg):
    theta = math.radians(theta_deg)
    rng = np.random.default_rng(int(theta_deg))
    q0 = rng.normal(size=4)
    q0 /= np.linalg.norm(q0)
    q = S.geoball_sf(5000, q0, theta, gamma)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-14)
    d = S.quat_distance(q, q0)
    assert d.max() <= theta + 1e-12
    ks = _ks(d, lambda t: S.ball_volume_fraction(t, theta))
    assert ks < 0.006, ks
    # the axial angle is symmetric about 0 and the ball is not lopsided
    local = S.quat_mul(np.array([q0[0], -q0[1], -q0[2], -q0[3]]), q)
    assert abs(np.mean(local[:, 1:], axis=0)).max() < 0.02 * math.sin(theta)


def test_geoball_spacing_matches_the_paper_with_the_plastic_number():
    q = S.geoball_sf(5000, [1.0, 0.0, 0.0, 0.0], math.radians(5.0), PLASTIC)
    spacing = math.degrees(S.mean_nn_rotation_angle(q))
    assert abs(spacing - 0.7) < 0.035, spacing


def test_radial_distribution_against_quadrature():
    theta = math.radians(5.0)
    r_t, F_t = S.radial_table(theta)
    rho = lambda r: r * 2.0 * math.acos(min(1.0, math.cos(theta) / math.sqrt(1.0 - r * r)))
    Z = integrate.quad(rho, 0.0, math.sin(theta), limit=200)[0]
    for frac in (0.1, 0.37, 0.5, 0.81, 0.99):
        r = frac * math.sin(theta)
        F = integrate.quad(rho, 0.0, r, limit=200)[0] / Z
        assert abs(np.interp(r, r_t, F_t) - F) < 2e-5, (frac, np.interp(r, r_t, F_t), F)


def test_planted_mistakes_are_caught(monkeypatch):
    # a radial density without the admissible-angle factor (rho ~ r) puts too
    # many samples near the boundary: the ball law fails
    theta = math.radians(20.0)
    orig = S.admissible_angle
    monkeypatch.setattr(S, "radial_table", lambda th, points=S.TABLE_POINTS: (
        np.linspace(0, math.sin(th), points), np.linspace(0, math.sin(th), points) ** 2 / math.sin(th) ** 2))
    d = S.quat_distance(S.geoball_sf(5000, [1, 0, 0, 0], theta), [1, 0, 0, 0])
    assert _ks(d, lambda t: S.ball_volume_fraction(t, theta)) > 0.02
    monkeypatch.undo()
    # half the admissible axial angle leaves the outer shell of the ball empty
    monkeypatch.setattr(S, "admissible_angle", lambda r, th: orig(r, th) / 2)
    d = S.quat_distance(S.geoball_sf(5000, [1, 0, 0, 0], theta), [1, 0, 0, 0])
    assert _ks(d, lambda t: S.ball_volume_fraction(t, theta)) > 0.02
    monkeypatch.undo()
    assert orig is S.admissible_angle
