"""Pins of the oracle's rotated-object variant of the global search (Sec. IV-D
as printed: the object grid O rotates and is resampled trilinearly onto the
canvas of the fixed swept occupancy S).  CPU only."""
import math

import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import search as S


def _lattice(m, g, deep=True):
    A = g.random((m, m, m))
    if deep:
        A[g.random((m, m, m)) < 0.25] = -50.0
    return A


def test_object_lattice_central_block_is_the_canvas_grid(cfg1):
    """O_w on the edge-m body lattice holds the canvas grid O (edge n) as its
    central block: the two grids sample the same points a + h (k - n/2)."""
    p = cfg1
    m = S.lattice_edge(p.n)
    Ow, fow, _ = S.object_lattice(p.vertices, p.faces, p.touchable, m, p.h)
    O, fo, _ = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    o = (m - p.n) // 2
    blk = (slice(o, o + p.n),) * 3
    assert np.array_equal(Ow[blk], O)
    assert np.array_equal(fow[blk], fo)
    assert (Ow == -50.0).any() and (Ow > 0).any()


def test_resample_object_at_identity_is_the_central_block():
    g = np.random.default_rng(21)
    n, h = 10, 0.3
    m = S.lattice_edge(n)
    Ow = _lattice(m, g)
    o = (m - n) // 2
    assert np.abs(S.resample_object(Ow, [1, 0, 0, 0], n, h) - Ow[o:o + n, o:o + n, o:o + n]).max() < 1e-12


def test_resample_object_quarter_turns_are_inverse_permutations():
    """Index maps written out by hand: a +90 deg turn about z rotates the
    object, so canvas voxel k reads the body lattice at R^T (k - n/2) + m/2,
    i.e. (x, y, z) -> (y, -x, z); about x, (x, y, z) -> (x, z, -y)."""
    g = np.random.default_rng(22)
    n, h = 12, 0.25
    m = S.lattice_edge(n)
    Ow = _lattice(m, g)
    c = math.sqrt(0.5)
    k = np.arange(n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    Oq = S.resample_object(Ow, [c, 0, 0, c], n, h)
    jx, jy, jz = (KY - n // 2) + m // 2, -(KX - n // 2) + m // 2, KZ - n // 2 + m // 2
    assert np.abs(Oq - Ow[jz, jy, jx]).max() < 1e-12
    Oq = S.resample_object(Ow, [c, c, 0, 0], n, h)
    jx, jy, jz = KX - n // 2 + m // 2, (KZ - n // 2) + m // 2, -(KY - n // 2) + m // 2
    assert np.abs(Oq - Ow[jz, jy, jx]).max() < 1e-12


def test_resample_object_matches_scipy_map_coordinates():
    """Trilinear values at the body points a + R^T h (k - n/2) equal scipy's
    order-1 map_coordinates on the lattice (an independent implementation)."""
    g = np.random.default_rng(23)
    n, h = 14, 0.3
    m = S.lattice_edge(n)
    Ow = _lattice(m, g)
    for _ in range(4):
        q = synth.haar_quaternion(g)
        R = synth.quat_to_mat(q)
        k = np.arange(n) - n / 2
        KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
        Kv = np.stack([KX, KY, KZ], -1).reshape(-1, 3)
        U = Kv @ R + m / 2            # rows: (R^T k)^T
        ref = ndimage.map_coordinates(Ow, [U[:, 2], U[:, 1], U[:, 0]], order=1, mode="constant", cval=0.0)
        assert np.abs(S.resample_object(Ow, q, n, h).ravel() - ref).max() < 1e-9


def test_resample_object_is_the_swept_resampler_at_the_inverse_rotation():
    """Rotating the object by R is rotating the lattice points by R^T: the
    variant's resampler equals the rotated-S resampler (pinned separately) at
    the conjugate quaternion, with a = wc."""
    g = np.random.default_rng(24)
    n, h = 12, 0.2
    m = S.lattice_edge(n)
    Ow = _lattice(m, g)
    for _ in range(3):
        q = synth.haar_quaternion(g)
        qc = np.array([q[0], -q[1], -q[2], -q[3]])
        a = g.normal(size=3)
        assert np.abs(S.resample_object(Ow, q, n, h) - S.resample(Ow, qc, n, h, a, a)).max() < 1e-12


def test_variant_at_identity_is_the_rotated_swept_field_reversed():
    """At R = I both searches correlate the same two grids (O's canvas block
    and S's canvas block), in opposite orders: C'[e] = C[-e], and the two pose
    formulas give the same pose."""
    g = np.random.default_rng(25)
    n, h = 12, 0.25
    m = S.lattice_edge(n)
    Ow = _lattice(m, g)
    Sw = (g.random((m, m, m)) < 0.4).astype(float)
    o = (m - n) // 2
    O = Ow[o:o + n, o:o + n, o:o + n]
    a, wc = np.array([0.3, -0.1, 0.2]), np.array([-0.2, 0.4, 0.05])
    Cs = S.correlate(O, S.resample(Sw, [1, 0, 0, 0], n, h, a, wc))
    Cv = S.correlate(S.swept_canvas(Sw, n), S.resample_object(Ow, [1, 0, 0, 0], n, h))
    idx = (-np.arange(n)) % n
    assert np.allclose(Cv, Cs[np.ix_(idx, idx, idx)], rtol=1e-12, atol=1e-9)
    e = np.array([2, -3, 1])
    R1, t1 = S.pose_from_object_shift([1, 0, 0, 0], e, a, wc, h)
    R2, t2 = S.pose_from_shift([1, 0, 0, 0], -e, a, wc, h)
    assert np.allclose(R1, R2) and np.allclose(t1, t2)


def test_variant_pose_formula_matches_world_frame_sum():
    """sum over the world canvas of S(z) O(R^T (z - t)) at the pose returned
    for (q, e), with O sampled by scipy at the body points, equals C'[e]."""
    g = np.random.default_rng(26)
    n, h = 16, 0.3
    m = S.lattice_edge(n)
    # the object's support within sqrt(3) n / 8 of the anchor, so that no
    # shift below n/4 carries it across the canvas edge (no wrap-around)
    Ow = np.zeros((m, m, m))
    c = slice(m // 2 - n // 8, m // 2 + n // 8)
    Ow[c, c, c] = np.where(g.random((2 * (n // 8),) * 3) < 0.3, -50.0, g.random((2 * (n // 8),) * 3))
    Sw = (g.random((m, m, m)) < 0.4).astype(float)
    Sc = S.swept_canvas(Sw, n)
    a, wc = np.array([0.31, -0.17, 0.05]), np.array([0.2, 0.1, -0.3])
    for _ in range(3):
        q = synth.haar_quaternion(g)
        Cv = S.correlate(Sc, S.resample_object(Ow, q, n, h))
        e = g.integers(-3, 4, size=3)
        R, t = S.pose_from_object_shift(q, e, a, wc, h)
        Z = S.canvas_points(n, h, wc)                  # world canvas points
        Y = (Z - t) @ R                                # body points R^T (z - t)
        U = (Y - (a - h * m / 2)) / h
        Oy = ndimage.map_coordinates(Ow, [U[:, 2], U[:, 1], U[:, 0]], order=1, mode="constant", cval=0.0)
        world = float(np.dot(Sc.ravel(), Oy))
        d = np.mod(e, n)
        assert world == pytest.approx(Cv[d[2], d[1], d[0]], rel=1e-9, abs=1e-9)


def test_variant_recovers_a_planted_pose_exactly():
    """S is the object's positive shell placed by a quarter turn about the
    anchor (an exact permutation of the lattice) and an integer shift: the
    variant's peak is that shift, and the pose formula returns the planted
    pose.  At the true shift S covers every positive value of O_q and no
    negative one, which no other shift can match."""
    g = np.random.default_rng(28)
    n, h = 16, 0.25
    m = S.lattice_edge(n)
    Ow = np.zeros((m, m, m))
    c = slice(m // 2 - 3, m // 2 + 3)
    Ow[c, c, c] = -50.0
    blob = g.random((8, 8, 8)) < 0.5
    shell = np.zeros((m, m, m), dtype=bool)
    shell[m // 2 - 4:m // 2 + 4, m // 2 - 4:m // 2 + 4, m // 2 - 4:m // 2 + 4] = blob
    shell[c, c, c] = False
    Ow[shell] = g.random(int(shell.sum())) + 0.1
    cq = math.sqrt(0.5)
    q = np.array([cq, 0.0, 0.0, cq])               # +90 deg about z
    Oq = S.resample_object(Ow, q, n, h)
    dk = np.array([3, -2, 1])
    Sc = np.roll(Oq > 0, shift=(dk[2], dk[1], dk[0]), axis=(0, 1, 2)).astype(float)
    s, flat, e = S.score_rotation_object(Sc, Ow, q, n, h)
    assert np.array_equal(-e, dk)
    assert s == pytest.approx(float(Oq[Oq > 0].sum()), rel=1e-12)
    a, wc = np.array([0.2, -0.3, 0.1]), np.array([1.0, 0.5, -0.5])
    R, t = S.pose_from_object_shift(q, e, a, wc, h)
    # the planted pose: body point a + u goes to wc + h dk + R u
    assert np.allclose(R @ a + t, wc + h * dk)
    assert np.allclose(R, synth.quat_to_mat(q))


def test_variant_recovers_the_known_pose_on_a_fine_canvas(cfg1):
    """The config-1 problem at h = 0.2 mm (64^3): the truth's rotation puts
    the peak within a voxel of the true pose, as the rotated-S search does.
    At its own 0.4 mm the interpolated -rho step (tau_in1 = 0.2 mm is half a
    voxel there) pulls the rotated-O peak about 1.6 voxels off."""
    p = cfg1
    n, h = 64, 0.2
    m = S.lattice_edge(n)
    Ow, _, _ = S.object_lattice(p.vertices, p.faces, p.touchable, m, h)
    Sc = S.swept_canvas(S.swept_occupancy(S.swept_lattice(p.poses, p.radius, p.length, m, h, p.center)), n)
    a = S.anchor(p.vertices)
    s, flat, e = S.score_rotation_object(Sc, Ow, p.q_gt, n, h)
    R, t = S.pose_from_object_shift(p.q_gt, e, a, p.center, h)
    Rg = synth.quat_to_mat(p.q_gt)
    err = np.linalg.norm((R @ a + t) - (Rg @ a + p.t_gt))
    assert err < h * math.sqrt(3) / 2 + 1e-9
    s_far, _, _ = S.score_rotation_object(Sc, Ow, [0.0, 1.0, 0.0, 0.0], n, h)
    assert s > s_far


def test_score_bounds_object_cover_every_flag_combination():
    """Brute force: every combination of moving three flagged lattice values
    of O (by up to |dO|, either sign) and flipping three flagged canvas voxels
    of S gives a field within the bound, by the direct definition."""
    n, h = 6, 0.3
    m = S.lattice_edge(n)
    g = np.random.default_rng(27)
    Ow = _lattice(m, g)
    Sc = (g.random((n, n, n)) < 0.5).astype(float)
    q = np.array([0.9, -0.2, 0.3, 0.25])
    q /= np.linalg.norm(q)
    # lattice points that are taps of canvas voxels (so the moves matter)
    R = S.quat_to_mat(q)
    ks = np.array([[1, 2, 3], [4, 4, 1], [2, 5, 5]], dtype=float)
    U = (ks - n / 2) @ R + m / 2
    flagO = [tuple(np.floor(u).astype(int)[::-1]) for u in U]
    dO = np.zeros_like(Ow)
    for j in flagO:
        dO[j] = 50.0 * g.random() + 1.0
    flagS = [tuple(g.integers(0, n, 3)) for _ in range(3)]
    Fc = np.zeros_like(Sc)
    for k in flagS:
        Fc[k] = 1.0
    C, B = S.score_bounds_object(Sc, Fc, Ow, dO, q, n, h)
    assert np.allclose(C, S.correlate_direct(Sc, S.resample_object(Ow, q, n, h)), atol=1e-9)
    assert B.max() > 0
    worst = 0.0
    for bits in range(1 << 6):
        O2 = Ow.copy()
        for i, j in enumerate(flagO):
            if bits >> i & 1:
                O2[j] += (1 if (bits + i) % 2 else -1) * dO[j]
        S2 = Sc.copy()
        for i, k in enumerate(flagS):
            if bits >> (3 + i) & 1:
                S2[k] = 1.0 - S2[k]
        C2 = S.correlate_direct(S2, S.resample_object(O2, q, n, h))
        assert np.all(np.abs(C2 - C) <= B + 1e-9)
        worst = max(worst, float(np.max(np.abs(C2 - C) / np.maximum(B, 1e-300) * (B > 0))))
    assert worst > 0.3
