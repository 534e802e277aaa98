"""Pins of the FP64 oracle's global-search functions (Sec. IV) against closed
forms, independent library routines, brute force and invariants."""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import search as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def box_mesh(b):
    """Axis-aligned box [-b, b], 12 outward CCW triangles."""
    bx, by, bz = b
    V = np.array([[x, y, z] for z in (-bz, bz) for y in (-by, by) for x in (-bx, bx)], dtype=np.float32)
    # vertex id = ix + 2 iy + 4 iz
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    F = []
    for a, b_, c, d in quads:
        F += [(a, b_, c), (a, c, d)]
    F = np.array(F, dtype=np.int32)
    # make every face outward
    T = V.astype(float)[F]
    nrm = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    flip = np.einsum("ij,ij->i", nrm, T.mean(axis=1)) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def box_sdf(P, b):
    q = np.abs(P) - np.asarray(b)
    return np.linalg.norm(np.maximum(q, 0), axis=1) + np.minimum(q.max(axis=1), 0)


def template(fo, d, tau_out1=0.5, tau_in1=0.2, deep=-50.0):
    ot = np.where((fo >= 0) & (fo < tau_out1), 1 - fo / tau_out1,
                  np.where((fo < 0) & (fo > -tau_in1), 1 + fo / tau_in1,
                           np.where(fo <= -tau_in1, deep, 0.0)))
    om = np.maximum(0.0, 1 - np.abs(d) / tau_out1)
    return np.minimum(ot, om)


# ------------------------------------------------------------ Table I

def test_table1_defaults():
    g = json.load(open(os.path.join(GOLD, "table1_parameters.json")))
    p = S.GridParams()
    assert p.tau_out1 == g["tau_out1_mm"] and p.tau_in1 == g["tau_in1_mm"]
    assert -p.rho == g["deep_value"]


# ------------------------------------------------------------ probe SDF

def test_probe_sdf_closed_forms():
    r, L = 0.5, 8.0
    f = lambda x, y, z: float(S.probe_sdf(x, y, z, r, L))
    # on the axis inside: nearest cap or side
    assert f(0, 0, 4) == pytest.approx(-0.5)
    assert f(0, 0, 0.1) == pytest.approx(-0.1)
    assert f(0.3, 0, 7.95) == pytest.approx(-0.05)
    # beyond the caps along the axis
    assert f(0, 0, -1.25) == pytest.approx(1.25)
    assert f(0.2, -0.1, 9.5) == pytest.approx(1.5)
    # beside the side wall
    assert f(0.3, 0.4, 3.0) == pytest.approx(0.0, abs=1e-15)
    assert f(2.0, 0, 3.0) == pytest.approx(1.5)
    # past the rim: distance to the rim circle
    assert f(1.0, 1.0, -2.0) == pytest.approx(math.hypot(math.sqrt(2) - 0.5, 2.0))
    assert f(0, 3.0, 10.0) == pytest.approx(math.hypot(2.5, 2.0))


def test_probe_sdf_c_matches_numpy():
    from oracle import _clib
    g = np.random.default_rng(1)
    P = g.uniform(-3, 11, size=(500, 3))
    a = S.probe_sdf(P[:, 0], P[:, 1], P[:, 2], 0.5, 8.0)
    b = np.array([_clib.lib().orc_probe_sdf(*p, 0.5, 8.0) for p in P])
    assert np.allclose(a, b, rtol=1e-14, atol=1e-15)


def test_probe_sdf_is_distance_outside():
    """Outside the cylinder f_p equals the distance to a dense sampling of its
    surface (up to the sampling resolution)."""
    r, L = 0.5, 8.0
    th = np.linspace(0, 2 * np.pi, 721)[:-1]
    zz = np.linspace(0, L, 801)
    side = np.stack([np.repeat(r * np.cos(th)[None], len(zz), 0).ravel(),
                     np.repeat(r * np.sin(th)[None], len(zz), 0).ravel(),
                     np.repeat(zz[:, None], len(th), 1).ravel()], 1)
    rr = np.linspace(0, r, 101)
    cap = np.stack([(rr[:, None] * np.cos(th)).ravel(), (rr[:, None] * np.sin(th)).ravel()], 1)
    caps = np.concatenate([np.c_[cap, np.zeros(len(cap))], np.c_[cap, np.full(len(cap), L)]])
    surf = np.concatenate([side, caps])
    g = np.random.default_rng(2)
    P = g.uniform([-2, -2, -2], [2, 2, 10], size=(60, 3))
    for p in P:
        f = float(S.probe_sdf(*p, r, L))
        if f <= 0:
            continue
        d = np.sqrt(((surf - p) ** 2).sum(1)).min()
        assert f <= d + 1e-12 and d - f < 0.01


# ---------------------------------------------------- mesh distances

def test_point_triangle_distance_vs_dense_sampling():
    from oracle import _clib
    g = np.random.default_rng(3)
    u = np.linspace(0, 1, 301)
    U, W = np.meshgrid(u, u)
    keep = U + W <= 1
    U, W = U[keep], W[keep]
    for _ in range(20):
        a, b, c = g.normal(size=(3, 3))
        p = g.normal(size=3) * 2
        pts = a + U[:, None] * (b - a) + W[:, None] * (c - a)
        dense = np.sqrt(((pts - p) ** 2).sum(1)).min()
        d = math.sqrt(_clib.lib().orc_point_tri_dist2(*(_clib.ptr(np.ascontiguousarray(x)) for x in (p, a, b, c))))
        assert d <= dense + 1e-12
        assert dense - d < 0.02


def test_winding_inside_icosphere():
    V, F = synth.icosphere(2)
    V = (3.0 * V).astype(np.float32)
    g = np.random.default_rng(4)
    P = g.uniform(-4, 4, size=(400, 3))
    rad = np.linalg.norm(P, axis=1)
    _, fo, _ = S.object_points(V, F, None, P)
    # the polyhedron lies between its inscribed radius and 3
    inr = 3.0 * np.cos(np.radians(12))
    sure_in, sure_out = rad < inr, rad > 3.0
    assert (fo[sure_in] < 0).all() and (fo[sure_out] > 0).all()


def test_object_grid_box_closed_form():
    """Box mesh: every canvas value equals the banded template of the textbook
    box SDF, both for the brute-force points path (winding number) and the
    banded grid path (ray parity), including rays through face diagonals."""
    b = (1.53125, 1.171875, 0.90625)   # exact in float32
    V, F = box_mesh(b)
    n, h = 40, 0.1
    O, fo, d = S.object_grid(V, F, None, n, h)
    a = S.anchor(V)
    assert np.allclose(a, 0, atol=1e-7)
    P = S.canvas_points(n, h, a)
    sdf = box_sdf(P, b)
    ref = template(sdf, np.abs(sdf))
    assert np.abs(O.ravel() - ref).max() < 1e-12
    band = np.abs(sdf) < 0.5
    assert np.abs(fo.ravel()[band] - sdf[band]).max() < 1e-12
    g = np.random.default_rng(5)
    sel = g.choice(len(P), 1500, replace=False)
    O2, fo2, _ = S.object_points(V, F, None, P[sel])
    assert np.abs(O2 - ref[sel]).max() < 1e-12
    assert np.abs(fo2 - sdf[sel]).max() < 1e-12


def test_object_grid_box_touchable_top():
    """Touchable subset = the two top triangles: O_m uses the distance to the
    top rectangle, a closed form."""
    b = (1.53125, 1.171875, 0.90625)   # exact in float32
    V, F = box_mesh(b)
    T = V.astype(float)[F]
    touch = (np.abs(T[:, :, 2] - b[2]) < 1e-6).all(axis=1).astype(np.uint8)
    assert touch.sum() == 2
    n, h = 40, 0.1
    O, _, d = S.object_grid(V, F, touch, n, h)
    P = S.canvas_points(n, h, S.anchor(V))
    dtop = np.sqrt(np.maximum(np.abs(P[:, 0]) - b[0], 0) ** 2 + np.maximum(np.abs(P[:, 1]) - b[1], 0) ** 2
                   + (P[:, 2] - b[2]) ** 2)
    ref = template(box_sdf(P, b), dtop)
    assert np.abs(O.ravel() - ref).max() < 1e-12


def test_object_grid_banded_equals_brute_force(cfg1):
    p = cfg1
    O, fo, d = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    P = S.canvas_points(p.n, p.h, S.anchor(p.vertices))
    g = np.random.default_rng(6)
    # half random, half in the band where the template varies
    band = np.flatnonzero(np.abs(fo.ravel()) < 0.6)
    sel = np.concatenate([g.choice(len(P), 700, replace=False), g.choice(band, 700, replace=False)])
    O2, fo2, d2 = S.object_points(p.vertices, p.faces, p.touchable, P[sel])
    assert np.abs(O.ravel()[sel] - O2).max() < 1e-12
    inb = np.abs(fo2) < 0.5
    assert np.abs(fo.ravel()[sel][inb] - fo2[inb]).max() < 1e-12
    assert (np.sign(fo.ravel()[sel]) == np.sign(fo2)).all()


# ------------------------------------------- threshold flags and bounds

def test_object_flags_box_closed_form():
    """Box whose top face lies 0.2 mm above a plane of canvas points: those
    voxels sit on the -tau_in1 jump.  The flagged set is the band of the
    textbook SDF, and the alternative value of each is the other branch of
    the template (closed form)."""
    b = (1.53125, 1.171875, 1.0)   # exact in float32; z = 0.8 is a canvas plane
    V, F = box_mesh(b)
    n, h = 40, 0.1
    O, fo, d = S.object_grid(V, F, None, n, h)
    P = S.canvas_points(n, h, S.anchor(V))
    sdf = box_sdf(P, b)
    delta = 1e-6
    dO = S.object_flags(O, fo, d, delta=delta).ravel()
    near = np.abs(sdf + 0.2) < delta
    assert near.sum() > 100 and (dO > 0).sum() == near.sum()
    assert ((dO > 0) == near).all()
    # other branch: deep voxels could take the shell value 1 + f/tau_in1 (about
    # 0, capped by the mask), shell voxels the penalty -50
    deep = sdf <= -0.2
    alt = np.where(deep, np.minimum(1 + sdf / 0.2, np.maximum(0, 1 - np.abs(sdf) / 0.5)), -50.0)
    ref = np.abs(alt - template(sdf, np.abs(sdf)))
    assert np.abs(dO[near] - ref[near]).max() < 1e-9
    assert np.all(dO[near] > 49.0)


def test_swept_flags_band():
    mf = np.array([-1.0, -1e-7, 0.0, 2e-7, 5e-5, np.inf])
    assert list(S.swept_flags(mf, 1e-6)) == [0, 1, 1, 1, 0, 0]


def test_score_bounds_cover_every_flag_combination():
    """Brute force: every combination of moving three flagged object voxels
    (by any amount up to |dO|, either sign) and flipping three flagged lattice
    points gives a field within the bound of its unperturbed one, computed
    by the direct O(n^6) definition of the correlation."""
    n, h = 6, 0.3
    m = S.lattice_edge(n)
    g = np.random.default_rng(41)
    O = g.normal(size=(n, n, n))
    O[g.random((n, n, n)) < 0.2] = -50.0
    Sw = (g.random((m, m, m)) < 0.5).astype(float)
    a, wc = np.array([0.1, -0.2, 0.05]), np.array([0.02, 0.0, -0.03])
    q = np.array([0.9, 0.2, -0.3, 0.25])
    q /= np.linalg.norm(q)
    flagO = [tuple(g.integers(0, n, 3)) for _ in range(3)]
    dO = np.zeros_like(O)
    for k in flagO:
        dO[k] = 50.0 * g.random() + 1.0
    # lattice points that are taps of canvas points (so the flips matter)
    R = S.quat_to_mat(q)
    ks = np.array([[1, 2, 3], [4, 4, 1], [2, 5, 5]], dtype=float)
    U = ((h * (ks - n / 2)) @ R.T + wc - (wc - h * m / 2)) / h
    flagS = [tuple(np.floor(u).astype(int)[::-1]) for u in U]
    Fs = np.zeros_like(Sw)
    for j in flagS:
        Fs[j] = 1.0
    C, B = S.score_bounds(O, dO, Sw, Fs, q, n, h, a, wc)
    assert np.allclose(C, S.correlate_direct(O, S.resample(Sw, q, n, h, a, wc)), atol=1e-9)
    assert B.max() > 0
    worst = 0.0
    for bits in range(1 << 6):
        O2 = O.copy()
        for i, k in enumerate(flagO):
            if bits >> i & 1:
                O2[k] += (1 if (bits + i) % 2 else -1) * dO[k]
        S2 = Sw.copy()
        for i, j in enumerate(flagS):
            if bits >> (3 + i) & 1:
                S2[j] = 1.0 - S2[j]
        C2 = S.correlate_direct(O2, S.resample(S2, q, n, h, a, wc))
        assert np.all(np.abs(C2 - C) <= B + 1e-9)
        worst = max(worst, float(np.max(np.abs(C2 - C) / np.maximum(B, 1e-300) * (B > 0))))
        lo, hi = S.score_interval(C, B)
        assert lo - 1e-9 <= C2.max() <= hi + 1e-9
        # the peak of every alternative is admissible
        assert int(np.argmax(C2.ravel())) in set(S.peak_admissible(C, B, lo, 1e-9).tolist())
    assert worst > 0.3   # the bound is not vacuous: some combination comes close


def test_peak_admissible_without_flags_is_the_tie_band():
    C = np.zeros((4, 4, 4))
    C.ravel()[[5, 17, 40]] = [3.0, 3.0 - 1e-6, 2.0]
    B = np.zeros_like(C)
    lo, hi = S.score_interval(C, B)
    assert lo == hi == 3.0
    assert list(S.peak_admissible(C, B, lo, 1e-5)) == [5, 17]
    assert list(S.peak_admissible(C, B, lo, 1e-7)) == [5]


def test_resample_of_a_list_equals_single_calls():
    n, h = 8, 0.25
    m = S.lattice_edge(n)
    g = np.random.default_rng(42)
    A, Bm = g.random((m, m, m)), g.random((m, m, m))
    q = np.array([0.3, -0.5, 0.7, 0.4])
    ra, rb = S.resample([A, Bm], q, n, h, np.zeros(3), np.zeros(3))
    assert np.array_equal(ra, S.resample(A, q, n, h, np.zeros(3), np.zeros(3)))
    assert np.array_equal(rb, S.resample(Bm, q, n, h, np.zeros(3), np.zeros(3)))


# ---------------------------------------------------- swept occupancy

def test_swept_single_axis_aligned_pose_count():
    """One pose with the identity rotation: the covered lattice points are the
    ones with (x-px)^2 + (y-py)^2 <= r^2 and 0 <= z-pz <= L."""
    r, L, h, m = 0.5, 8.0, 0.1, 120
    wc = np.array([0.0, 0.0, 0.0])
    p = np.array([0.013, -0.021, -3.963])
    pose = np.array([[1, 0, 0, 0, *p]], dtype=np.float32)
    mf = S.swept_lattice(pose, r, L, m, h, wc)
    Y = S.lattice_points(m, h, wc)
    pp = pose[0, 4:].astype(float)
    inside = (((Y[:, 0] - pp[0]) ** 2 + (Y[:, 1] - pp[1]) ** 2 <= r * r)
              & (Y[:, 2] - pp[2] >= 0) & (Y[:, 2] - pp[2] <= L))
    assert ((mf.ravel() <= 0) == inside).all()


def test_swept_volume_converges_to_cylinder_volume():
    r, L = 0.5, 8.0
    pose = np.array([[0.9, 0.3, -0.2, 0.25, 0.01, 0.02, -0.03]], dtype=np.float32)
    vols = []
    for h, m in ((0.1, 200), (0.05, 380)):
        mf = S.swept_lattice(pose, r, L, m, h, np.zeros(3))
        vols.append((mf <= 0).sum() * h ** 3)
    exact = math.pi * r * r * L
    assert abs(vols[1] - exact) / exact < 0.02
    assert abs(vols[1] - exact) < abs(vols[0] - exact) + 0.02 * exact


def test_swept_lattice_banded_equals_brute_force(cfg1):
    p = cfg1
    m = S.lattice_edge(p.n)
    mf = S.swept_lattice(p.poses, p.radius, p.length, m, p.h, p.center)
    Y = S.lattice_points(m, p.h, p.center)
    g = np.random.default_rng(7)
    near = np.flatnonzero(np.abs(mf.ravel()) < 0.3)
    sel = np.concatenate([g.choice(len(Y), 1500, replace=False), g.choice(near, 1500, replace=False)])
    bf = S.swept_points(p.poses, p.radius, p.length, Y[sel])
    cu = mf.ravel()[sel]
    ex = bf <= p.h
    assert np.abs(cu[ex] - bf[ex]).max() < 1e-12
    assert (cu[~ex] > p.h).all()
    assert ((cu <= 0) == (bf <= 0)).all()


# ------------------------------------------------- rotate and resample

def _rand_lattice(m, g, binary=True):
    A = g.random((m, m, m))
    return (A < 0.3).astype(float) if binary else A


def test_resample_identity_is_a_copy():
    g = np.random.default_rng(8)
    n, m, h = 12, S.lattice_edge(12), 0.3
    Sw = _rand_lattice(m, g)
    Sr = S.resample(Sw, [1, 0, 0, 0], n, h, np.array([0.2, -0.1, 0.4]), np.array([0.5, 0.0, -0.2]))
    o = (m - n) // 2
    assert np.abs(Sr - Sw[o:o + n, o:o + n, o:o + n]).max() < 1e-12


def test_resample_quarter_turns_are_permutations():
    g = np.random.default_rng(9)
    n, m, h = 12, S.lattice_edge(12), 0.25
    Sw = _rand_lattice(m, g)
    c = math.sqrt(0.5)
    o = (m - n) // 2
    k = np.arange(n)
    # +90 deg about z: (x, y, z) -> (-y, x, z);  lattice index j = R (k - n/2) + m/2
    Sr = S.resample(Sw, [c, 0, 0, c], n, h, np.zeros(3), np.zeros(3))
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    jx, jy, jz = -(KY - n // 2) + m // 2, (KX - n // 2) + m // 2, KZ - n // 2 + m // 2
    assert np.abs(Sr - Sw[jz, jy, jx]).max() < 1e-12
    # +90 deg about x: (x, y, z) -> (x, -z, y)
    Sr = S.resample(Sw, [c, c, 0, 0], n, h, np.zeros(3), np.zeros(3))
    jx, jy, jz = KX - n // 2 + m // 2, -(KZ - n // 2) + m // 2, (KY - n // 2) + m // 2
    assert np.abs(Sr - Sw[jz, jy, jx]).max() < 1e-12
    assert o >= 0


def test_resample_matches_scipy_map_coordinates():
    """Trilinear resampling equals scipy.ndimage.map_coordinates(order=1) at the
    rotated canvas points (an independent trilinear implementation)."""
    g = np.random.default_rng(10)
    n, h = 14, 0.3
    m = S.lattice_edge(n)
    Sw = _rand_lattice(m, g)
    a, wc = np.array([0.3, -0.2, 0.1]), np.array([-0.4, 0.25, 0.6])
    for _ in range(4):
        q = synth.haar_quaternion(g)
        Sr = S.resample(Sw, q, n, h, a, wc)
        R = synth.quat_to_mat(q)
        X = S.canvas_points(n, h, a)
        Y = (X - a) @ R.T + wc
        U = (Y - (wc - h * m / 2)) / h
        ref = ndimage.map_coordinates(Sw, [U[:, 2], U[:, 1], U[:, 0]], order=1, mode="constant", cval=0.0)
        assert np.abs(Sr.ravel() - ref).max() < 1e-9


def test_resample_reproduces_affine_fields():
    g = np.random.default_rng(11)
    n, h = 10, 0.2
    m = S.lattice_edge(n)
    al, be = np.array([0.7, -1.3, 0.4]), 2.5
    J = np.arange(m)
    JZ, JY, JX = np.meshgrid(J, J, J, indexing="ij")
    Sw = al[0] * JX + al[1] * JY + al[2] * JZ + be
    q = synth.haar_quaternion(g)
    Sr = S.resample(Sw, q, n, h, np.zeros(3), np.zeros(3))
    R = synth.quat_to_mat(q)
    k = np.arange(n) - n / 2
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    Kv = np.stack([KX, KY, KZ], -1).reshape(-1, 3)
    U = Kv @ R.T + m / 2
    assert np.abs(Sr.ravel() - (U @ al + be)).max() < 1e-9


# ------------------------------------------------------- correlation

@pytest.mark.parametrize("n", [4, 5, 6, 8])
def test_fft_correlation_equals_direct_definition(n):
    g = np.random.default_rng(100 + n)
    O = np.where(g.random((n, n, n)) < 0.3, -50.0, g.random((n, n, n)))
    Sg = g.random((n, n, n))
    C1 = S.correlate(O, Sg)
    # direct sum written out independently of the oracle's own direct form
    C2 = np.zeros_like(C1)
    idx = np.arange(n)
    for dz in range(n):
        for dy in range(n):
            for dx in range(n):
                tot = 0.0
                for kz in range(n):
                    for ky in range(n):
                        tot += np.dot(O[kz, ky], Sg[(kz + dz) % n, (ky + dy) % n, (idx + dx) % n])
                C2[dz, dy, dx] = tot
    assert np.abs(C1 - C2).max() < 1e-10 * np.abs(C2).max()
    assert np.abs(S.correlate_direct(O, Sg) - C2).max() < 1e-10 * np.abs(C2).max()


def test_correlation_sum_rule_and_zero_shift():
    g = np.random.default_rng(12)
    n = 16
    O = np.where(g.random((n, n, n)) < 0.2, -50.0, g.random((n, n, n)))
    Sg = g.random((n, n, n))
    C = S.correlate(O, Sg)
    assert C.sum() == pytest.approx(O.sum() * Sg.sum(), rel=1e-10)
    assert C[0, 0, 0] == pytest.approx(np.sum(O * Sg), rel=1e-12)


def test_correlation_of_deltas():
    n = 8
    O = np.zeros((n, n, n))
    Sg = np.zeros((n, n, n))
    O[1, 2, 3] = 1.0      # k0 = (x=3, y=2, z=1)
    Sg[6, 0, 5] = 1.0     # k1 = (x=5, y=0, z=6)
    C = S.correlate(O, Sg)
    # C[d] = 1 iff k0 + d = k1 (mod n):  d = (x=2, y=6, z=5)
    assert C[5, 6, 2] == pytest.approx(1.0)
    C[5, 6, 2] = 0
    assert np.abs(C).max() < 1e-12


# ----------------------------------------------------------- peak

def test_peak_lowest_index_on_ties():
    n = 8
    C = np.zeros((n, n, n))
    C[3, 1, 2] = 5.0
    C[1, 4, 6] = 5.0
    C[7, 7, 7] = 4.0
    s, flat, d = S.peak(C)
    assert s == 5.0 and flat == (1 * n + 4) * n + 6
    assert list(d) == [6 - n, 4 - n, 1]   # components >= n/2 wrap to negative


def test_peak_recovers_a_rolled_pattern():
    g = np.random.default_rng(13)
    n = 16
    m = S.lattice_edge(n)
    o = (m - n) // 2
    B = (g.random((n, n, n)) < 0.25).astype(float)
    for delta in ([3, -5, 7], [-8, 0, 2], [1, 1, -1]):
        Sw = np.zeros((m, m, m))
        # S_r[k + delta] = B[k] at R = I
        Sw[o:o + n, o:o + n, o:o + n] = np.roll(B, shift=(delta[2], delta[1], delta[0]), axis=(0, 1, 2))
        s, flat, d = S.score_rotation(B, Sw, [1, 0, 0, 0], n, 0.2, np.zeros(3), np.zeros(3))
        assert list(d) == delta
        assert s == pytest.approx(B.sum())


def test_pose_formula_matches_world_frame_sum():
    """sum_k O[k] S_w(R x_k + t) at the pose returned for (q, delta), evaluated
    in world coordinates with scipy's trilinear sampler, equals C[delta]."""
    g = np.random.default_rng(14)
    n, h = 16, 0.3
    m = S.lattice_edge(n)
    Sw = _rand_lattice(m, g)
    O = np.zeros((n, n, n))
    c = slice(n // 4, 3 * n // 4)
    O[c, c, c] = np.where(g.random((n // 2,) * 3) < 0.3, -50.0, g.random((n // 2,) * 3))
    a, wc = np.array([0.31, -0.17, 0.05]), np.array([0.2, 0.1, -0.3])
    for _ in range(3):
        q = synth.haar_quaternion(g)
        C = S.correlate(O, S.resample(Sw, q, n, h, a, wc))
        delta = g.integers(-n // 4 + 1, n // 4, size=3)
        R, t = S.pose_from_shift(q, delta, a, wc, h)
        X = S.canvas_points(n, h, a)
        Y = X @ R.T + t
        U = (Y - (wc - h * m / 2)) / h
        Sy = ndimage.map_coordinates(Sw, [U[:, 2], U[:, 1], U[:, 0]], order=1, mode="constant", cval=0.0)
        world = np.dot(O.ravel(), Sy)
        d = np.mod(delta, n)
        assert world == pytest.approx(C[d[2], d[1], d[0]], rel=1e-9, abs=1e-9)


def test_known_pose_recovered_within_a_voxel(cfg1):
    p = cfg1
    O, _, _ = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    m = S.lattice_edge(p.n)
    Sw = S.swept_occupancy(S.swept_lattice(p.poses, p.radius, p.length, m, p.h, p.center))
    a = S.anchor(p.vertices)
    s, flat, d = S.score_rotation(O, Sw, p.q_gt, p.n, p.h, a, p.center)
    R, t = S.pose_from_shift(p.q_gt, d, a, p.center, p.h)
    Rg = synth.quat_to_mat(p.q_gt)
    err = np.linalg.norm((R @ a + t) - (Rg @ a + p.t_gt))
    assert err < p.h * math.sqrt(3) / 2 + 1e-9


def test_top_k_order():
    s = np.array([1.0, 3.0, 2.0, 3.0, -1.0, 2.0])
    assert list(S.top_k(s, 4)) == [1, 3, 2, 5]


def test_sobol_hopf_rotation_angle_is_haar():
    """The SO(3) input set: rotation angles follow the Haar CDF (w - sin w)/pi."""
    q = synth.sobol_hopf_so3(4096, synth.rng(9, 0, 4))
    w = 2 * np.arccos(np.clip(np.abs(q[:, 0]), 0, 1))
    w.sort()
    emp = (np.arange(len(w)) + 0.5) / len(w)
    assert np.abs(emp - (w - np.sin(w)) / np.pi).max() < 0.01
