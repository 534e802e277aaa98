"""GPU parity of the orientation samplers (Sec. IV-C) and of the local search
(Sec. IV-D) against the FP64 oracle, through the C ABI.

Samples: float32 output of FP64 arithmetic, compared element by element within
3e-7 (the float32 rounding of unit components plus the last bits of the
device's transcendental functions).  Local search: the GeoBall-SF set around
the global maximum replaces the handle's rotations; scores and peaks follow
the search's bar (1e-4 of the largest |score|, peak equal or tied within it).
"""
import math

import numpy as np
import pytest

import synth
from oracle import sampling as SA
from oracle import search as S

pytestmark = pytest.mark.gpu

PLASTIC = 1.324717957244746


def _lib():
    import paper_2605_21398_amd as rd
    rd.load_library()
    return rd


@pytest.mark.parametrize("n", [1, 7, 1000, 20000])
def test_super_fibonacci_matches_oracle(n):
    rd = _lib()
    got = rd.so3_super_fibonacci(n).cpu().numpy().astype(np.float64)
    ref = SA.super_fibonacci(n)
    assert np.abs(got - ref).max() <= 3e-7, np.abs(got - ref).max()


@pytest.mark.parametrize("n,theta_deg,gamma,seed", [(5000, 5.0, None, 0), (777, 40.0, PLASTIC, 1), (1, 90.0, None, 2),
                                                    (20000, 0.5, None, 3)])
def test_geoball_matches_oracle(n, theta_deg, gamma, seed):
    rd = _lib()
    g = np.random.default_rng(seed)
    q0 = g.normal(size=4)
    theta = math.radians(theta_deg)
    got = rd.so3_geoball_sf(n, q0, theta, 0.0 if gamma is None else gamma).cpu().numpy().astype(np.float64)
    ref = SA.geoball_sf(n, q0, theta, gamma)
    err = np.abs(got - ref).max()
    print(f"\nn={n} theta={theta_deg} deg: max |q_gpu - q_oracle| = {err:.2e}")
    assert err <= 3e-7
    # every device sample inside the ball (up to the float32 rounding)
    assert SA.quat_distance(got, q0 / np.linalg.norm(q0)).max() <= theta + 1e-6


def test_sampler_abi_errors():
    rd = _lib()
    for args in [(0, [1, 0, 0, 0], 0.1), (10, [0, 0, 0, 0], 0.1), (10, [1, 0, 0, 0], 0.0), (10, [1, 0, 0, 0], 2.0),
                 (10, [math.nan, 0, 0, 0], 0.1)]:
        with pytest.raises(rd.RegError):
            rd.so3_geoball_sf(*args)
    with pytest.raises(rd.RegError):
        rd.so3_super_fibonacci(0)


def test_local_search_scores_match_oracle():
    """Global search, then 48 GeoBall-SF rotations (theta = 5 deg) around the
    best rotation scored on the same handle with the oracle's grids."""
    rd = _lib()
    p = synth.config_problem(1, 0)
    O, _, _ = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    m = S.lattice_edge(p.n)
    Sw = S.swept_occupancy(S.swept_lattice(p.poses, p.radius, p.length, m, p.h, p.center))
    h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius, p.length)
    try:
        rd.register_set_grids(h, O.astype(np.float32), Sw.astype(np.uint8))
        sc, _, _ = rd.score_rotations(h)
        best = int(np.argmax(sc.cpu().numpy()))
        q_star = p.so3[best].astype(np.float64)
        local = rd.so3_geoball_sf(48, q_star, math.radians(5.0))
        rd.register_set_rotations(h, local)
        assert h.n_rot == 48
        sc2, sh2, po2 = rd.score_rotations(h)
        sc2, sh2, po2 = sc2.cpu().numpy(), sh2.cpu().numpy(), po2.cpu().numpy()
        a = S.anchor(p.vertices)
        ql = local.cpu().numpy()
        fields = [S.correlate(O.astype(np.float32).astype(np.float64), S.resample(Sw, q, p.n, p.h, a, p.center))
                  for q in ql]
        ref = np.array([f.max() for f in fields])
        tol = 1e-4 * np.abs(ref).max()
        assert np.abs(sc2 - ref).max() <= tol
        n = p.n
        d = np.mod(sh2, n)
        flat = (d[:, 2] * n + d[:, 1]) * n + d[:, 0]
        for r in range(len(ql)):
            fr = int(np.argmax(fields[r].ravel()))
            if flat[r] != fr:
                assert fields[r].ravel()[flat[r]] >= fields[r].ravel()[fr] - tol
        # the poses are those of the local rotations
        qn = ql.astype(np.float64) / np.linalg.norm(ql.astype(np.float64), axis=1, keepdims=True)
        assert np.allclose(po2[:, :4], qn, atol=1e-12)
    finally:
        rd.register_free(h)


def test_set_rotations_grows_shrinks_and_validates():
    rd = _lib()
    p = synth.config_problem(1, 0, M=16)
    h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius, p.length)
    try:
        first = rd.score_rotations(h, shift=False, pose=False)[0].cpu().numpy()
        big = rd.so3_super_fibonacci(40)
        rd.register_set_rotations(h, big)
        s_big = rd.score_rotations(h, shift=False, pose=False)[0].cpu().numpy()
        assert s_big.shape == (40,)
        rd.register_set_rotations(h, p.so3)
        again = rd.score_rotations(h, shift=False, pose=False)[0].cpu().numpy()
        assert np.array_equal(first, again)
        bad = p.so3.copy()
        bad[3] *= 2.0
        with pytest.raises(rd.RegError):
            rd.register_set_rotations(h, bad)
        with pytest.raises(rd.RegError):
            rd.score_rotations(h, 0, 1)
        rd.register_set_rotations(h, big[:5])
        assert np.array_equal(rd.score_rotations(h, shift=False, pose=False)[0].cpu().numpy(), s_big[:5])
    finally:
        rd.register_free(h)
