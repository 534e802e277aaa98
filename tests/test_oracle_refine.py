"""Pins of the FP64 refinement oracle (Sec. V) against closed forms, an
independent rotation library, quadrature, brute force, finite differences and
noise-free recovery of a known pose."""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from oracle import refine as Rf
from oracle import search as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PRM = Rf.RefineParams()


# ------------------------------------------------------------ proximity score

def test_proximity_defaults_follow_table1():
    g = json.load(open(os.path.join(GOLD, "table1_parameters.json")))
    assert PRM.tau_out2 == g["tau_out2_mm"] and PRM.tau_in2 == g["tau_in2_mm"]
    assert PRM.k == g["k_slope"] and PRM.lam == g["lambda"]
    assert PRM.tau_in2 / PRM.tau_out2 == pytest.approx(g["r_ratio"])


def test_proximity_values():
    tau, r, k = PRM.tau_out2, PRM.tau_in2 / PRM.tau_out2, PRM.k
    d = np.array([0.0, tau, -PRM.tau_in2, 2 * tau, -0.5, 0.5 * tau, -3 * PRM.tau_in2])
    s, ds, _ = Rf.proximity(d)
    assert s[0] == pytest.approx(1.0)
    assert s[1] == pytest.approx(0.0, abs=1e-15)
    assert s[2] == pytest.approx(0.0, abs=1e-12)
    assert s[3] == 0.0 and ds[3] == 0.0
    assert s[4] == pytest.approx(k * (-0.5 / tau + r))          # deep: linear penalty
    assert ds[4] == pytest.approx(k / tau)
    assert s[5] == pytest.approx(0.5)                            # cos^2(pi/4)
    assert s[6] == pytest.approx(k * (-3 * PRM.tau_in2 / tau + r))


@pytest.mark.parametrize("t0", [-0.15, 0.0, 1.0])
def test_proximity_is_c1_at_the_joints(t0):
    tau = PRM.tau_out2
    h = 1e-7
    d0 = t0 * tau
    sl, dl, _ = Rf.proximity(np.array([d0 - h, d0 - 2 * h]))
    sr, dr, _ = Rf.proximity(np.array([d0 + h, d0 + 2 * h]))
    assert abs(sl[0] - sr[0]) < 3 * h * max(1.0, abs(dl[0]))     # continuous
    left = (sl[0] - sl[1]) / h
    right = (sr[1] - sr[0]) / h
    assert abs(left - right) < 1e-3 * max(1.0, abs(left))        # derivative continuous
    assert abs(dl[0] - dr[0]) < 1e-3 * max(1.0, abs(dl[0]))


def test_proximity_derivative_matches_finite_differences():
    d = np.linspace(-0.2, 0.25, 901) + 1e-4
    s, ds, d2 = Rf.proximity(d)
    h = 1e-7
    sp, _, _ = Rf.proximity(d + h)
    sm, _, _ = Rf.proximity(d - h)
    fd = (sp - sm) / (2 * h)
    assert np.abs(fd - ds).max() < 1e-4 * np.abs(ds).max()


def test_printed_cubic_coefficients_break_continuity():
    """The coefficients as printed (A = k/r^2 + 2/r^3, B = -k/r - 3/r^2) give a
    jump at t = -r, so the C1-forced ones are used (a reading, not the print)."""
    r, k = PRM.tau_in2 / PRM.tau_out2, PRM.k
    A, B = k / r ** 2 + 2 / r ** 3, -k / r - 3 / r ** 2
    assert abs(A * (-r) ** 3 + B * r ** 2 + 1.0) > 1.0
    A2, B2 = k / r ** 2 - 2 / r ** 3, k / r - 3 / r ** 2
    assert A2 * (-r) ** 3 + B2 * r ** 2 + 1.0 == pytest.approx(0.0, abs=1e-12)
    assert 3 * A2 * r ** 2 - 2 * B2 * r == pytest.approx(k)


# ------------------------------------------------------------------ SO(3)

def test_so3_exp_matches_scipy():
    g = np.random.default_rng(1)
    for _ in range(20):
        w = g.normal(size=3) * g.uniform(1e-6, 2.0)
        assert np.abs(Rf.so3_exp(w) - Rotation.from_rotvec(w).as_matrix()).max() < 1e-13


def test_left_jacobian_is_the_integral_of_exp():
    """V(w) = int_0^1 exp(s w^) ds (the SO(3) left Jacobian), by quadrature."""
    g = np.random.default_rng(2)
    xs, ws = np.polynomial.legendre.leggauss(40)
    for _ in range(6):
        w = g.normal(size=3) * 0.7
        I = sum(wt * Rotation.from_rotvec(0.5 * (x + 1) * w).as_matrix() for x, wt in zip(xs, ws)) * 0.5
        assert np.abs(Rf.left_jacobian(w) - I).max() < 1e-12


def test_left_jacobian_series_joins_closed_form():
    g = np.random.default_rng(3)
    u = g.normal(size=3)
    u /= np.linalg.norm(u)
    a = Rf.left_jacobian(u * (1e-4 * (1 - 1e-9)))
    b = Rf.left_jacobian(u * (1e-4 * (1 + 1e-9)))
    assert np.abs(a - b).max() < 1e-11
    w = u * 0.3
    assert np.allclose(Rf.left_jacobian(w) @ w, w, atol=1e-15)


def test_pose_update_rotates_about_the_anchor():
    g = np.random.default_rng(4)
    R0 = Rotation.random(random_state=5).as_matrix()
    p0 = g.normal(size=3)
    a = g.normal(size=3)
    xi = np.concatenate([g.normal(size=3) * 0.3, g.normal(size=3) * 0.2])
    R, p = Rf.pose_of(xi, R0, p0, a)
    # the anchor moves by exactly V(w) v (Eq. left-update-p)
    assert np.allclose((R @ a + p) - (R0 @ a + p0), Rf.left_jacobian(xi[3:]) @ xi[:3], atol=1e-14)
    # with v = 0 the anchor is a fixed point
    R1, p1 = Rf.pose_of(np.concatenate([np.zeros(3), xi[3:]]), R0, p0, a)
    assert np.allclose(R1 @ a + p1, R0 @ a + p0, atol=1e-14)
    assert np.allclose(R1 @ R1.T, np.eye(3), atol=1e-14) and np.linalg.det(R1) == pytest.approx(1.0)


# ------------------------------------------------------------ distance query

def test_face_min_closed_forms():
    r, L = 0.5, 8.0
    # triangle parallel to the tip cap, below it, covering the axis: distance = gap
    tri = [np.array([-1.0, -1.0, -0.07]), np.array([2.0, -1.0, -0.07]), np.array([-1.0, 2.0, -0.07])]
    v, _, _ = Rf.face_min(*tri, r, L)
    assert v == pytest.approx(0.07, abs=1e-9)
    # the same plane just inside the cap: depth 0.04 (nearest boundary is the cap)
    tri = [np.array([-1.0, -1.0, 0.04]), np.array([2.0, -1.0, 0.04]), np.array([-1.0, 2.0, 0.04])]
    v, _, _ = Rf.face_min(*tri, r, L)
    assert v == pytest.approx(-0.04, abs=1e-9)
    # a vertical triangle beside the shaft: distance to the side wall
    tri = [np.array([0.8, -0.3, 2.0]), np.array([0.8, 0.3, 2.0]), np.array([0.8, 0.0, 3.0])]
    v, _, _ = Rf.face_min(*tri, r, L)
    assert v == pytest.approx(0.3, abs=1e-9)
    # a triangle beyond the rim: distance to the rim circle
    tri = [np.array([1.0, 0.0, -1.0]), np.array([1.0, 0.0, -1.0]) + 1e-3 * np.array([0, 1, 0]),
           np.array([1.0, 0.0, -1.0]) + 1e-3 * np.array([0, 0, -1])]
    v, _, _ = Rf.face_min(*tri, r, L)
    assert v == pytest.approx(math.hypot(0.5, 1.0), abs=1e-9)


def test_face_min_vs_dense_sampling():
    g = np.random.default_rng(6)
    u = np.linspace(0, 1, 161)
    U, W = np.meshgrid(u, u)
    keep = U + W <= 1
    U, W = U[keep], W[keep]
    for _ in range(40):
        c = g.uniform([-1, -1, -0.5], [1, 1, 1.0])
        tri = [c + g.normal(size=3) * 0.25 for _ in range(3)]
        v, s, t = Rf.face_min(*tri, 0.5, 8.0)
        P = tri[0] + U[:, None] * (tri[1] - tri[0]) + W[:, None] * (tri[2] - tri[0])
        dense = S.probe_sdf(P[:, 0], P[:, 1], P[:, 2], 0.5, 8.0).min()
        assert v <= dense + 1e-12
        assert dense - v < 0.01
        x = tri[0] + s * (tri[1] - tri[0]) + t * (tri[2] - tri[0])
        assert float(S.probe_sdf(*x, 0.5, 8.0)) == pytest.approx(v, abs=1e-12)


@pytest.fixture(scope="module")
def small_problem():
    p = synth.config_problem(1, 0)
    a = S.anchor(p.vertices)
    Rg = synth.quat_to_mat(p.q_gt)
    w0 = np.radians(1.0) * np.array([0.6, -0.5, 0.62])
    R0 = Rf.so3_exp(w0) @ Rg
    p0 = p.t_gt + np.array([0.05, -0.03, 0.04])
    return p, Rf.Problem(p.vertices, p.faces, p.poses, p.radius, p.length, R0, p0, a), Rg


def test_culling_keeps_every_distance_below_eps(small_problem):
    p, pb, _ = small_problem
    d, x, n, f = Rf.distance_query(p.vertices, p.faces, pb.table, pb.R0, pb.p0, p.poses, p.radius, p.length, 0.25)
    d2, _, _, f2 = Rf.distance_query(p.vertices, p.faces, pb.table, pb.R0, pb.p0, p.poses, p.radius, p.length, 50.0)
    m = d < 0.25
    assert m.sum() > 50
    assert np.abs(d[m] - d2[m]).max() < 1e-12
    assert (d2[~m] >= 0.25 - 1e-12).all()


def test_sensitivities_match_finite_differences(small_problem):
    p, pb, _ = small_problem
    g = np.random.default_rng(7)
    xi = np.concatenate([g.normal(size=3) * 0.02, g.normal(size=3) * 0.01])
    R, pp = Rf.pose_of(xi, pb.R0, pb.p0, pb.a)
    d, x, n, f = Rf.distance_query(p.vertices, p.faces, pb.table, R, pp, p.poses, p.radius, p.length, 0.25)
    G = Rf.sensitivities(xi, pb, x, n)
    sel = np.flatnonzero(np.abs(d) < 0.2)[:25]
    # the selection holds witnesses on the probe's inner side/cap ridge (the
    # min-max case) in the interior of a face and on a face edge
    ridge = []
    for i in sel:
        P = p.poses[i].astype(np.float64)
        u = synth.quat_to_mat(P[:4]).T @ (x[i] - P[4:])
        q1 = math.hypot(u[0], u[1]) - p.radius
        q2 = abs(u[2] - 0.5 * p.length) - 0.5 * p.length
        ridge.append(max(q1, q2) < 0 and abs(q1 - q2) < 1e-8)
    assert sum(ridge) >= 5
    h = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        Rp, ppp = Rf.pose_of(xi + e, pb.R0, pb.p0, pb.a)
        Rm, pm = Rf.pose_of(xi - e, pb.R0, pb.p0, pb.a)
        dp = Rf.distance_query(p.vertices, p.faces, pb.table, Rp, ppp, p.poses, p.radius, p.length, 0.25)[0]
        dm = Rf.distance_query(p.vertices, p.faces, pb.table, Rm, pm, p.poses, p.radius, p.length, 0.25)[0]
        fd = (dp - dm) / (2 * h)
        assert np.abs(fd[sel] - G[sel, j]).max() < 2e-4


def test_gradient_matches_finite_differences_of_J(small_problem):
    _, pb, _ = small_problem
    g = np.random.default_rng(8)
    xi = np.concatenate([g.normal(size=3) * 0.02, g.normal(size=3) * 0.01])
    J, grad, H = Rf.evaluate(xi, pb)
    h = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        fd = (Rf.evaluate(xi + e, pb, want_grad=False)[0] - Rf.evaluate(xi - e, pb, want_grad=False)[0]) / (2 * h)
        assert fd == pytest.approx(grad[j], rel=2e-4, abs=2e-3)
    assert np.all(np.linalg.eigvalsh(H) > 0)


def test_noise_free_recovery_of_a_known_pose(small_problem):
    """Contact poses touch the true surface (d = 0) and the lifted ones clear
    it, so the truth maximises sum s; from a start 1 deg / 0.07 mm off the
    refinement must return it (the lambda pull is ~1e-9 mm)."""
    p, pb, Rg = small_problem
    res = Rf.refine(pb)
    a = pb.a
    ce = np.linalg.norm((res.R @ a + res.p) - (Rg @ a + p.t_gt))
    re = np.degrees(Rotation.from_matrix(res.R.T @ Rg).magnitude())
    assert ce < 1e-5 and re < 1e-4
    assert res.J == pytest.approx(-float(p.contact.sum()), abs=1e-3)


def test_lm_step_free_set_matches_reduced_solve():
    """The active-set step equals the solve of the free coordinates' own block
    (written here as a sub-matrix solve, not by the row/column replacement the
    oracle uses), is zero on the active ones, and is the full solve with none."""
    g = np.random.default_rng(5)
    B = g.normal(size=(6, 6))
    H = B @ B.T + 0.1 * np.eye(6)
    grad = g.normal(size=6)
    mu = 0.3
    full = np.linalg.solve(H + mu * np.diag(np.diag(H)) + 1e-12 * np.eye(6), -grad)
    assert np.allclose(Rf.lm_step(H, grad, mu, np.zeros(6, bool)), full, rtol=1e-12, atol=1e-14)
    act = np.array([False, True, False, False, True, False])
    free = ~act
    Hf = H[np.ix_(free, free)]
    ref = np.linalg.solve(Hf + mu * np.diag(np.diag(Hf)) + 1e-12 * np.eye(free.sum()), -grad[free])
    st = Rf.lm_step(H, grad, mu, act)
    assert np.all(st[act] == 0.0)
    assert np.allclose(st[free], ref, rtol=1e-12, atol=1e-14)


def test_active_bounds_rule():
    prm = Rf.RefineParams()
    xi = np.array([prm.b_t, -prm.b_t, 0.1, prm.b_r, -prm.b_r, prm.b_r])
    g = np.array([-1.0, 1.0, -1.0, 1.0, -1.0, 0.0])
    # at +b with descent pushing up (g < 0), at -b pushing down (g > 0): held;
    # interior, or gradient pointing back inside, or zero: free
    assert Rf.active_bounds(xi, g, prm).tolist() == [True, True, False, False, False, False]


def test_lbfgsb_reaches_the_known_pose_and_the_gauss_newton_minimum(small_problem):
    """The paper's L-BFGS-B on the same objective: the noise-free truth is
    recovered (as by the Gauss-Newton iteration), the two solvers end at the
    same minimum, and the solution satisfies the box KKT conditions."""
    p, pb, Rg = small_problem
    lb = Rf.refine_lbfgsb(pb)
    gn = Rf.refine(pb)
    a = pb.a
    ce = np.linalg.norm((lb.R @ a + lb.p) - (Rg @ a + p.t_gt))
    re = np.degrees(Rotation.from_matrix(lb.R.T @ Rg).magnitude())
    assert ce < 1e-4 and re < 1e-3
    assert np.linalg.norm((lb.R @ a + lb.p) - (gn.R @ a + gn.p)) < 1e-4
    assert lb.J == pytest.approx(gn.J, abs=1e-6)
    prm = Rf.RefineParams()
    _, g, _ = Rf.evaluate(lb.xi, pb, prm)
    pg = lb.xi - Rf.project_box(lb.xi - g, prm)
    assert np.abs(pg).max() < 1e-5
