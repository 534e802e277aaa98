"""FP64 oracle of the continuous SE(3) refinement (Sec. V of the paper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module; the HIP path never does.

Pose model (Sec. V-A): the object pose T = (R, p) maps body to world.  A twist
xi = (v, w) (mm, rad) acts as a left perturbation about the anchor a:
    R(xi) = exp(w^) R0,   p(xi) = p0 + V(w) v + (I - exp(w^)) R0 a,
with V the SO(3) left Jacobian (Eq. se3-exp, left-update-R/p).

Objective (Eq. objective): J = -sum_i s(d_i) + lambda |xi|^2 with the proximity
score s of Sec. V-A and d_i the smallest signed probe-object distance at probe
pose i (Sec. V-B), subject to |v|_inf <= b_t, |w|_inf <= b_r (Eq. reg-problem).

Readings taken (listed in the design notes):
  * r = tau_in2 / tau_out2 = 0.15 (the printed ratio is inverted), and the cubic
    coefficients are the ones C1 continuity at t = -r and t = 0 forces:
    A = k/r^2 - 2/r^3, B = k/r - 3/r^2 (the printed ones break continuity);
  * lambda printed as "10e-4" is 1e-3;
  * b_t = 0.5 mm, b_r = 0.2 rad and eps = 0.25 mm are not given by the paper;
  * the rotation sensitivity of Eq. dd-domg is taken through the left Jacobian,
    dd/dw = V(w)^T ((x* - c) x n) + D^T n, which is the printed form at w = 0;
    D = d(V(w) v)/dw is taken by central differences as the paper does;
  * the solver is damped Gauss-Newton (Levenberg-Marquardt) on the box with an
    FP64 6x6 solve in place of L-BFGS-B; curvature sum_i max(0, -s'') g g^T.
    Like L-BFGS-B it keeps an active set: a coordinate at its bound whose
    gradient points out of the box is held there and the step solves for the
    others (a clamped full step stalls along the box faces);
  * refine_lbfgsb is the paper's L-BFGS-B on the same J and gradient (SciPy's
    implementation as the optimiser primitive), the reference of the device's
    L-BFGS-B solver.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np

from . import _clib


@dataclass
class RefineParams:
    tau_out2: float = 0.2
    tau_in2: float = 0.03
    k: float = 15.0
    lam: float = 1e-3
    b_t: float = 0.5
    b_r: float = 0.2
    eps: float = 0.25
    max_iters: int = 200
    tol_pg: float = 1e-10      # projected-gradient stop
    tol_step: float = 1e-12    # step-size stop
    mu0: float = 1e-3
    face_tol: float = 1e-10    # barycentric tolerance of the per-face minimisation


# ------------------------------------------------------------ proximity score

def proximity(d, prm: RefineParams = RefineParams()):
    """s(d), ds/dd and d2s/dd2 (one-sided at the C1 joints), vectorised."""
    d = np.asarray(d, dtype=np.float64)
    tau = prm.tau_out2
    r = prm.tau_in2 / prm.tau_out2
    k = prm.k
    A = k / r ** 2 - 2.0 / r ** 3
    B = k / r - 3.0 / r ** 2
    t = d / tau
    s = np.zeros_like(t)
    ds = np.zeros_like(t)
    d2 = np.zeros_like(t)
    m1 = (t > 0) & (t <= 1)
    s[m1] = np.cos(0.5 * np.pi * t[m1]) ** 2
    ds[m1] = -0.5 * np.pi * np.sin(np.pi * t[m1])
    d2[m1] = -0.5 * np.pi ** 2 * np.cos(np.pi * t[m1])
    m2 = (t > -r) & (t <= 0)
    s[m2] = A * t[m2] ** 3 + B * t[m2] ** 2 + 1.0
    ds[m2] = 3 * A * t[m2] ** 2 + 2 * B * t[m2]
    d2[m2] = 6 * A * t[m2] + 2 * B
    m3 = t <= -r
    s[m3] = k * (t[m3] + r)
    ds[m3] = k
    return s, ds / tau, d2 / tau ** 2


# ------------------------------------------------------------------ SO(3)

def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def so3_exp(w) -> np.ndarray:
    """Rodrigues: exp(w^)."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.linalg.norm(w))
    W = hat(w)
    if th < 1e-8:
        return np.eye(3) + W + 0.5 * W @ W
    return np.eye(3) + math.sin(th) / th * W + (1 - math.cos(th)) / th ** 2 * W @ W


def left_jacobian(w) -> np.ndarray:
    """V(w) = I + (1 - cos t)/t^2 w^ + (t - sin t)/t^3 (w^)^2, series below 1e-4."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.linalg.norm(w))
    W = hat(w)
    if th < 1e-4:
        return np.eye(3) + 0.5 * W + W @ W / 6.0 - (th ** 2) * W / 24.0 - (th ** 2) * (W @ W) / 120.0
    return np.eye(3) + (1 - math.cos(th)) / th ** 2 * W + (th - math.sin(th)) / th ** 3 * W @ W


def pose_of(xi, R0, p0, a):
    """(R(xi), p(xi)) of the left perturbation about the anchor."""
    v, w = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    dR = so3_exp(w)
    R = dR @ R0
    p = p0 + left_jacobian(w) @ v + (np.eye(3) - dR) @ (R0 @ a)
    return R, p


def coupling(w, v, h: float = 1e-7) -> np.ndarray:
    """D = d(V(w) v)/dw by central differences."""
    D = np.zeros((3, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        D[:, j] = (left_jacobian(w + e) @ v - left_jacobian(w - e) @ v) / (2 * h)
    return D


def project_box(xi, prm: RefineParams):
    out = np.array(xi, dtype=np.float64)
    out[:3] = np.clip(out[:3], -prm.b_t, prm.b_t)
    out[3:] = np.clip(out[3:], -prm.b_r, prm.b_r)
    return out


# ------------------------------------------------------------ distance query

def face_table(vertices, faces):
    """Body-frame face centroids and their bounding radii."""
    T = np.asarray(vertices, dtype=np.float32).astype(np.float64)[np.asarray(faces)]
    c = T.mean(axis=1)
    r = np.sqrt(((T - c[:, None, :]) ** 2).sum(-1)).max(axis=1)
    return np.ascontiguousarray(c), np.ascontiguousarray(r)


def face_min(p0, p1, p2, r: float, L: float, tol: float = 1e-10):
    """min of the probe SDF over a triangle given in the probe frame: (value, s, t)."""
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (p0, p1, p2)]
    s = ctypes.c_double()
    t = ctypes.c_double()
    v = _clib.lib().orc_face_min(*(_clib.ptr(x) for x in a), r, L, tol, ctypes.byref(s), ctypes.byref(t))
    return v, s.value, t.value


def distance_query(vertices, faces, table, R, p, poses, r: float, L: float, eps: float, tol: float = 1e-10):
    """d (N,), witness x* (N,3), probe normal n (N,3), face index (N,) (-1: none kept)."""
    V = np.ascontiguousarray(vertices, dtype=np.float32)
    F = np.ascontiguousarray(faces, dtype=np.int32)
    Pz = np.ascontiguousarray(poses, dtype=np.float32)
    fc, fr = table
    Rm = np.ascontiguousarray(R, dtype=np.float64)
    pv = np.ascontiguousarray(p, dtype=np.float64)
    n = len(Pz)
    d = np.empty(n)
    x = np.empty((n, 3))
    nn = np.empty((n, 3))
    fi = np.empty(n, dtype=np.int32)
    _clib.lib().orc_distance_query(_clib.ptr(V), _clib.ptr(F), len(F), _clib.ptr(fc), _clib.ptr(fr), _clib.ptr(Rm),
                                   _clib.ptr(pv), _clib.ptr(Pz), n, r, L, eps, tol, _clib.ptr(d), _clib.ptr(x),
                                   _clib.ptr(nn), _clib.ptr(fi))
    return d, x, nn, fi


# ------------------------------------------------------------------ objective

@dataclass
class Problem:
    vertices: np.ndarray
    faces: np.ndarray
    poses: np.ndarray
    radius: float
    length: float
    R0: np.ndarray
    p0: np.ndarray
    a: np.ndarray
    table: tuple = None

    def __post_init__(self):
        if self.table is None:
            self.table = face_table(self.vertices, self.faces)


def sensitivities(xi, pb: Problem, x, n):
    """g_i = [V^T n_i ; V^T ((x*_i - c) x n_i) + D^T n_i], c = p0 + V v + R0 a."""
    v, w = xi[:3], xi[3:]
    Vw = left_jacobian(w)
    D = coupling(w, v)
    c = pb.p0 + Vw @ v + pb.R0 @ pb.a
    gv = n @ Vw
    gw = np.cross(x - c, n) @ Vw + n @ D
    return np.concatenate([gv, gw], axis=1)


def evaluate(xi, pb: Problem, prm: RefineParams = RefineParams(), want_grad: bool = True):
    """J(xi) and, optionally, grad J and the Gauss-Newton curvature H."""
    R, p = pose_of(xi, pb.R0, pb.p0, pb.a)
    d, x, n, _ = distance_query(pb.vertices, pb.faces, pb.table, R, p, pb.poses, pb.radius, pb.length, prm.eps,
                                prm.face_tol)
    s, ds, d2s = proximity(d, prm)
    J = -s.sum() + prm.lam * float(np.dot(xi, xi))
    if not want_grad:
        return J, None, None
    g = sensitivities(xi, pb, x, n)
    grad = -(ds[:, None] * g).sum(axis=0) + 2 * prm.lam * xi
    w = np.maximum(0.0, -d2s)
    H = (g * w[:, None]).T @ g + 2 * prm.lam * np.eye(6)
    return J, grad, H


def solve6(A, b):
    """The 6x6 normal-equation solve (Cholesky-free reference)."""
    return np.linalg.solve(A, b)


def active_bounds(xi, g, prm: RefineParams):
    """Coordinates held at their bound: at the bound (within 1e-12 of it) with
    the gradient pointing out of the box, so that a descent step would leave it."""
    b = np.array([prm.b_t] * 3 + [prm.b_r] * 3)
    return ((xi >= b - 1e-12) & (g < 0)) | ((xi <= -b + 1e-12) & (g > 0))


def lm_step(H, g, mu, active):
    """Damped Gauss-Newton step on the free coordinates, zero on the active ones:
    (H + mu diag H + 1e-12 I) restricted to the free set, solved in FP64."""
    A = H + mu * np.diag(np.diag(H)) + 1e-12 * np.eye(6)
    rhs = -np.asarray(g, dtype=np.float64).copy()
    A = A.copy()
    A[active, :] = 0.0
    A[:, active] = 0.0
    A[active, active] = 1.0
    rhs[active] = 0.0
    return solve6(A, rhs)


@dataclass
class RefineResult:
    R: np.ndarray
    p: np.ndarray
    J: float
    iters: int
    xi: np.ndarray
    mu: float = 0.0   # damping when the iteration stopped (Gauss-Newton)


def refine(pb: Problem, prm: RefineParams = RefineParams()) -> RefineResult:
    """Damped Gauss-Newton on the box from xi = 0 (Sec. V-C; solver per the
    readings): each iteration solves for the free coordinates, projects onto the
    box, keeps the step if J decreases (mu / 3) and otherwise retries with 3 mu."""
    xi = np.zeros(6)
    mu = prm.mu0
    J, g, H = evaluate(xi, pb, prm)
    it = 0
    while it < prm.max_iters:
        pg = xi - project_box(xi - g, prm)
        if np.abs(pg).max() <= prm.tol_pg:
            break
        it += 1
        accepted = False
        step = np.zeros(6)
        active = active_bounds(xi, g, prm)
        while mu < 1e12:
            step = lm_step(H, g, mu, active)
            xn = project_box(xi + step, prm)
            Jn, _, _ = evaluate(xn, pb, prm, want_grad=False)
            if Jn < J:
                xi = xn
                mu = max(mu / 3.0, 1e-12)
                accepted = True
                break
            mu *= 3.0
        if not accepted or np.abs(step).max() <= prm.tol_step:
            break
        J, g, H = evaluate(xi, pb, prm)
    R, p = pose_of(xi, pb.R0, pb.p0, pb.a)
    return RefineResult(R=R, p=p, J=J, iters=it, xi=xi, mu=mu)


def refine_lbfgsb(pb: Problem, prm: RefineParams = RefineParams(), memory: int = 10, gtol: float = 1e-9,
                  ftol: float = 1e-15) -> RefineResult:
    """The paper's solver (Sec. V-C): L-BFGS-B on J(xi) over the box from
    xi = 0 with the analytic gradient, stopped when the projected gradient
    (gtol) or the relative reduction of J (ftol) falls below its threshold.
    SciPy's L-BFGS-B is the optimiser primitive; J and grad J are this
    module's."""
    from scipy.optimize import minimize

    bounds = [(-prm.b_t, prm.b_t)] * 3 + [(-prm.b_r, prm.b_r)] * 3

    def fun(xi):
        J, g, _ = evaluate(np.asarray(xi, dtype=np.float64), pb, prm)
        return J, g

    res = minimize(fun, np.zeros(6), jac=True, method="L-BFGS-B", bounds=bounds,
                   options=dict(maxcor=memory, gtol=gtol, ftol=ftol, maxiter=prm.max_iters, maxfun=20 * prm.max_iters))
    xi = np.asarray(res.x, dtype=np.float64)
    R, p = pose_of(xi, pb.R0, pb.p0, pb.a)
    return RefineResult(R=R, p=p, J=float(res.fun), iters=int(res.nit), xi=xi)

