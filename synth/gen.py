"""Seeded generators for meshes, probe trajectories, SO(3) sets and grid specs.

The paper evaluates on five scanned/CAD meshes scaled to 5-8 mm and on
OpenCAMLib contact trajectories of a cylindrical probe (Sec. VI-A).  Neither
ships with the paper, so these recipes stand in for them:

* mesh: an icosphere whose radius 5 mm is perturbed by real spherical
  harmonics of degree <= lmax with N(0, 0.1^2) coefficients, scaled so the
  perturbation stays within 10 % of the radius (star-shaped, watertight);
* touchable surface: the faces whose body-frame centroid has z > 0 (the swept
  hemisphere), standing in for the "touchable subset" of Sec. IV-A;
* trajectory: N probe poses with the probe axis along directions of a
  Fibonacci spiral over the upper hemisphere (polar angle 0..80 deg, pole to
  rim), the flat tip resting on the surface for a random 60 % of the poses and
  lifted along the axis by U[0.3, 1.0] mm for the rest; optional "hops" (the
  contact loss of Sec. VI-A) lift a fraction of the contact poses the same way,
  and optional Gaussian pose noise is applied after placement;
* SO(3) samples: scrambled Sobol points mapped through Hopf coordinates, the
  sampler the paper compares Super-Fibonacci against (Sec. IV-C);
* ground truth: a Haar-random rotation and a translation uniform in a 2 mm ball.

Quaternions are (w, x, y, z), scalar first, as in Alg. 1.  Poses are rows of
(qw, qx, qy, qz, tx, ty, tz) mapping probe-local coordinates to world.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import sph_harm_y
from scipy.stats import qmc

SEED = 260521398

# stream ids of the seeded generators
S_MESH, S_GT, S_TRAJ, S_CONTACT, S_SOBOL, S_ARRIVAL, S_SIZE, S_PICK = 0, 1, 2, 3, 4, 5, 6, 7


def rng(cfg: int, item: int, stream: int) -> np.random.Generator:
    """Independent generator for (config, item, stream)."""
    return np.random.default_rng(np.random.SeedSequence(SEED, spawn_key=(cfg, item, stream)))


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def icosphere(level: int):
    """Unit icosphere: 10*4^level + 2 vertices, 20*4^level CCW-outward faces."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(level):
        cache: dict = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts)
    F = np.array(faces, dtype=np.int32)
    # orient every face outward (the sphere is centred at the origin)
    nrm = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = np.einsum("ij,ij->i", nrm, V[F].mean(axis=1)) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def _real_sh(l: int, m: int, theta, phi):
    y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * y.real
    if m < 0:
        return math.sqrt(2.0) * (-1) ** m * y.imag
    return y.real


def perturbed_sphere(level: int, lmax: int, g: np.random.Generator, radius: float = 5.0):
    """Star-shaped watertight mesh: radius*(1 + s*P(u))*u with |s*P| <= 0.1."""
    U, F = icosphere(level)
    theta = np.arccos(np.clip(U[:, 2], -1.0, 1.0))
    phi = np.mod(np.arctan2(U[:, 1], U[:, 0]), 2 * np.pi)
    P = np.zeros(len(U))
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            P += g.normal(0.0, 0.1) * _real_sh(l, m, theta, phi)
    s = min(1.0, 0.1 / max(np.abs(P).max(), 1e-300))
    V = radius * (1.0 + s * P)[:, None] * U
    return V.astype(np.float32), F.astype(np.int32)


def touchable_mask(V: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Faces whose body-frame centroid lies above z = 0."""
    c = V.astype(np.float64)[F].mean(axis=1)
    return (c[:, 2] > 0).astype(np.uint8)


# ----------------------------------------------------------------------------
# rotations
# ----------------------------------------------------------------------------

def quat_to_mat(q) -> np.ndarray:
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = np.moveaxis(q, -1, 0)
    R = np.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], axis=-1)
    return R.reshape(q.shape[:-1] + (3, 3))


def mat_to_quat(R) -> np.ndarray:
    """Rotation matrix -> unit quaternion with w >= 0 (Shepperd's method)."""
    R = np.asarray(R, dtype=np.float64)
    tr = np.trace(R)
    cands = np.array([tr, R[0, 0], R[1, 1], R[2, 2]])
    i = int(np.argmax(cands))
    if i == 0:
        s = math.sqrt(1.0 + tr) * 2
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif i == 1:
        s = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif i == 2:
        s = math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    q /= np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def quat_mul(a, b) -> np.ndarray:
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def haar_quaternion(g: np.random.Generator) -> np.ndarray:
    q = g.normal(size=4)
    q /= np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def sobol_hopf_so3(M: int, g: np.random.Generator) -> np.ndarray:
    """M (a power of two) scrambled-Sobol samples mapped through Hopf coordinates."""
    if M <= 0 or M & (M - 1):
        raise ValueError("M must be a power of two")
    u = qmc.Sobol(d=3, scramble=True, rng=g).random_base2(int(round(math.log2(M))))
    th = np.arccos(1.0 - 2.0 * u[:, 0])
    ph = 2 * np.pi * u[:, 1]
    ps = 2 * np.pi * u[:, 2]
    q = np.stack([np.cos(th / 2) * np.cos(ps / 2), np.cos(th / 2) * np.sin(ps / 2),
                  np.sin(th / 2) * np.cos(ph + ps / 2), np.sin(th / 2) * np.sin(ph + ps / 2)], axis=1)
    return q


def _axis_angle_quat(w) -> np.ndarray:
    th = float(np.linalg.norm(w))
    if th < 1e-300:
        return np.array([1.0, 0.0, 0.0, 0.0])
    a = np.asarray(w) / th
    return np.concatenate([[math.cos(th / 2)], math.sin(th / 2) * a])


# ----------------------------------------------------------------------------
# trajectories
# ----------------------------------------------------------------------------

def hemisphere_directions(N: int, max_polar_deg: float = 80.0) -> np.ndarray:
    """Fibonacci spiral over the polar cap [0, max_polar], ordered pole to rim."""
    j = np.arange(N) + 0.5
    cmin = math.cos(math.radians(max_polar_deg))
    ct = 1.0 - (1.0 - cmin) * j / N
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = np.arange(N) * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)


def min_rotation_to(u) -> np.ndarray:
    """Quaternion of the minimal rotation taking e_z onto unit u (u_z > -1)."""
    u = np.asarray(u, dtype=np.float64)
    q = np.array([1.0 + u[2], -u[1], u[0], 0.0])
    return q / np.linalg.norm(q)


def _face_table(V: np.ndarray, F: np.ndarray):
    T = V.astype(np.float64)[F]                                # (F,3,3)
    cen = T.mean(axis=1)
    rad = np.sqrt(((T - cen[:, None, :]) ** 2).sum(-1)).max(axis=1)
    return T, cen, rad


def footprint_top(V: np.ndarray, F: np.ndarray, u: np.ndarray, r: float, table=None) -> float:
    """Highest point (along unit u) of the mesh inside the infinite cylinder of
    radius r about the line R*u.  A flat-ended probe with axis +u whose tip disk
    sits at this height rests on the surface without entering it."""
    u = np.asarray(u, dtype=np.float64)
    a = np.array([1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(u, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    T, cen, rad = _face_table(V, F) if table is None else table
    # keep only faces that can reach the column: centroid within r plus the
    # face's own circumradius (about its centroid) of the axis line
    cu = cen @ u
    perp2 = np.einsum("ij,ij->i", cen, cen) - cu * cu
    T = T[perp2 <= (r + rad) ** 2 * (1 + 1e-9)]
    P = np.stack([T @ e1, T @ e2], axis=-1)                    # (F,3,2)
    H = T @ u                                                  # (F,3)
    best = -np.inf
    # (1) vertices inside the disk
    inside = (P ** 2).sum(-1) <= r * r
    if inside.any():
        best = max(best, H[inside].max())
    # (2) edges crossing the circle
    for i0, i1 in ((0, 1), (1, 2), (2, 0)):
        A, B = P[:, i0], P[:, i1]
        D = B - A
        qa = (D ** 2).sum(-1)
        qb = 2 * (A * D).sum(-1)
        qc = (A ** 2).sum(-1) - r * r
        disc = qb * qb - 4 * qa * qc
        ok = (qa > 0) & (disc >= 0)
        sq = np.sqrt(np.where(ok, disc, 0.0))
        for sgn in (-1.0, 1.0):
            t = np.where(ok, (-qb + sgn * sq) / np.where(ok, 2 * qa, 1.0), -1.0)
            m = ok & (t >= 0) & (t <= 1)
            if m.any():
                best = max(best, (H[m, i0] + t[m] * (H[m, i1] - H[m, i0])).max())
    # (3) interior maximiser on the circle of the affine height over the face
    d1 = P[:, 1] - P[:, 0]
    d2 = P[:, 2] - P[:, 0]
    det = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]
    nd = np.abs(det) > 1e-12
    if nd.any():
        h1 = H[nd, 1] - H[nd, 0]
        h2 = H[nd, 2] - H[nd, 0]
        dt = det[nd]
        gx = (h1 * d2[nd, 1] - h2 * d1[nd, 1]) / dt
        gy = (h2 * d1[nd, 0] - h1 * d2[nd, 0]) / dt
        gn = np.hypot(gx, gy)
        safe = np.where(gn > 0, gn, 1.0)
        px = np.where(gn > 0, r * gx / safe, r)
        py = np.where(gn > 0, r * gy / safe, 0.0)
        # barycentric of (px,py) in the projected face
        rx = px - P[nd, 0, 0]
        ry = py - P[nd, 0, 1]
        b1 = (rx * d2[nd, 1] - ry * d2[nd, 0]) / dt
        b2 = (d1[nd, 0] * ry - d1[nd, 1] * rx) / dt
        m = (b1 >= 0) & (b2 >= 0) & (b1 + b2 <= 1)
        if m.any():
            hv = H[nd, 0] + gx * (px - P[nd, 0, 0]) + gy * (py - P[nd, 0, 1])
            best = max(best, hv[m].max())
    return float(best)


def make_trajectory(V, F, N, g, radius, contact_frac=0.6, hop_frac=0.0,
                    noise_t=0.0, noise_r_deg=0.0, q_gt=None, t_gt=None):
    """Probe poses (N,7) float64 in world, plus per-pose flags and lifts."""
    dirs = hemisphere_directions(N)
    n_contact = int(round(contact_frac * N))
    order = g.permutation(N)
    contact = np.zeros(N, dtype=bool)
    contact[order[:n_contact]] = True
    lift = np.where(contact, 0.0, g.uniform(0.3, 1.0, size=N))
    if hop_frac > 0:
        cidx = np.flatnonzero(contact)
        hop = g.permutation(cidx)[: int(round(hop_frac * len(cidx)))]
        contact[hop] = False
        lift[hop] = g.uniform(0.3, 1.0, size=len(hop))
    Rg = quat_to_mat(q_gt)
    table = _face_table(V, F)
    poses = np.zeros((N, 7))
    for j in range(N):
        u = dirs[j]
        s = footprint_top(V, F, u, radius, table) + lift[j]
        qb = min_rotation_to(u)
        q = quat_mul(q_gt, qb)
        p = Rg @ (s * u) + t_gt
        if noise_t > 0:
            p = p + g.normal(0.0, noise_t, size=3)
        if noise_r_deg > 0:
            w = g.normal(0.0, math.radians(noise_r_deg), size=3)
            q = quat_mul(_axis_angle_quat(w), q)
        q = q / np.linalg.norm(q)
        poses[j, :4] = q if q[0] >= 0 else -q
        poses[j, 4:] = p
    return poses, contact, lift


def grid_edge_m(n: int) -> int:
    """Edge of the swept-volume lattice: the smallest even m with m >= sqrt(3) n + 2."""
    return 2 * math.ceil((math.sqrt(3.0) * n + 2.0) / 2.0)


# ----------------------------------------------------------------------------
# problems
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    vertices: np.ndarray      # (V,3) float32, mm, body frame
    faces: np.ndarray         # (F,3) int32, CCW outward
    touchable: np.ndarray     # (F,) uint8
    poses: np.ndarray         # (N,7) float32, probe-local -> world
    so3: np.ndarray           # (M,4) float32 unit quaternions
    n: int
    h: float
    center: np.ndarray = field(default_factory=lambda: np.zeros(3))
    radius: float = 0.5       # probe radius (mm)
    length: float = 8.0       # probe length (mm)
    q_gt: np.ndarray = None   # (4,) float64 ground-truth rotation (body -> world)
    t_gt: np.ndarray = None   # (3,) float64 ground-truth translation
    contact: np.ndarray = None


CONFIGS = {
    1: dict(level=4, lmax=6, N=200, n=32, h=0.4, M=64, hop=0.0, noise_t=0.0, noise_r=0.0),
    2: dict(level=4, lmax=6, N=800, n=64, h=0.25, M=1024, hop=0.3, noise_t=0.0, noise_r=0.0),
    3: dict(level=5, lmax=12, N=2000, n=128, h=0.12, M=4096, hop=0.0, noise_t=0.05, noise_r=0.2),
}


def make_problem(cfg: int, item: int, level: int, lmax: int, N: int, n: int, h: float, M: int,
                 hop: float = 0.0, noise_t: float = 0.0, noise_r: float = 0.0,
                 radius: float = 0.5, length: float = 8.0, mesh=None) -> Problem:
    """A registration problem; `mesh` = (V, F) reuses a given object mesh (the
    serving workload draws its objects from a fixed pool)."""
    V, F = mesh if mesh is not None else perturbed_sphere(level, lmax, rng(cfg, item, S_MESH))
    touch = touchable_mask(V, F)
    gg = rng(cfg, item, S_GT)
    q_gt = haar_quaternion(gg)
    d = gg.normal(size=3)
    t_gt = d / np.linalg.norm(d) * 2.0 * gg.uniform() ** (1.0 / 3.0)
    poses, contact, _ = make_trajectory(V, F, N, rng(cfg, item, S_CONTACT), radius,
                                        hop_frac=hop, noise_t=noise_t, noise_r_deg=noise_r,
                                        q_gt=q_gt, t_gt=t_gt)
    so3 = sobol_hopf_so3(M, rng(cfg, item, S_SOBOL))
    return Problem(vertices=V, faces=F, touchable=touch, poses=poses.astype(np.float32),
                   so3=so3.astype(np.float32), n=n, h=h, radius=radius, length=length,
                   q_gt=q_gt, t_gt=t_gt, contact=contact)


def config_problem(cfg: int, item: int = 0, **over) -> Problem:
    p = dict(CONFIGS[cfg])
    p.update(over)
    return make_problem(cfg, item, p["level"], p["lmax"], p["N"], p["n"], p["h"], p["M"],
                        hop=p["hop"], noise_t=p["noise_t"], noise_r=p["noise_r"])


# ----------------------------------------------------------------------------
# uneven batches and serving
# ----------------------------------------------------------------------------

# canvas edges and SO(3) set sizes of the uneven batch (h = 15.36 mm / n keeps
# the 15.36 mm canvas of the 128^3 workload)
BATCH_N = (48, 60, 64, 80, 96, 120, 128)
BATCH_M = (512, 1024, 2048, 4096)
SERVE_MESHES = 20
SERVE_RATE = 200.0   # requests per second (Poisson)


def batch_spec(i: int, cfg: int = 4) -> dict:
    """Sizes of registration i of the uneven batch: n, h = 15.36/n, M, N in
    [300, 2000], SH degree in [6, 12], level-5 mesh, the pose noise of the
    128^3 workload."""
    g = rng(cfg, i, S_SIZE)
    n = int(g.choice(BATCH_N))
    return dict(level=5, lmax=int(g.integers(6, 13)), N=int(g.integers(300, 2001)), n=n, h=15.36 / n,
                M=int(g.choice(BATCH_M)), hop=0.0, noise_t=0.05, noise_r=0.2)


def batch_problem(i: int, cfg: int = 4, **over) -> Problem:
    spec = batch_spec(i, cfg)
    spec.update(over)
    return make_problem(cfg, i, **spec)


def serve_mesh(mesh_id: int, cfg: int = 5):
    """Object `mesh_id` of the serving pool: a level-5 perturbed sphere."""
    g = rng(cfg, 10_000 + mesh_id, S_MESH)
    lmax = int(g.integers(6, 13))
    return perturbed_sphere(5, lmax, rng(cfg, 10_000 + mesh_id, S_TRAJ))


def serve_spec(req: int, cfg: int = 5) -> dict:
    """Request `req` of the serving stream: one of SERVE_MESHES objects drawn
    uniformly; 10 % at n = 160 (h = 0.096 mm, 8192 rotations), the rest sized
    as the uneven batch."""
    g = rng(cfg, req, S_SIZE)
    mesh_id = int(g.integers(0, SERVE_MESHES))
    if g.uniform() < 0.1:
        spec = dict(level=5, lmax=0, N=int(g.integers(300, 2001)), n=160, h=0.096, M=8192)
    else:
        n = int(g.choice(BATCH_N))
        spec = dict(level=5, lmax=0, N=int(g.integers(300, 2001)), n=n, h=15.36 / n, M=int(g.choice(BATCH_M)))
    spec.update(hop=0.0, noise_t=0.05, noise_r=0.2)
    return dict(mesh_id=mesh_id, **spec)


def serve_problem(req: int, cfg: int = 5, mesh_cache: dict | None = None, **over) -> tuple[int, Problem]:
    """(mesh id, problem) of request `req`; trajectory, ground truth and SO(3)
    set are drawn fresh from the request id."""
    spec = serve_spec(req, cfg)
    spec.update(over)
    mid = spec.pop("mesh_id")
    if mesh_cache is not None and mid in mesh_cache:
        mesh = mesh_cache[mid]
    else:
        mesh = serve_mesh(mid, cfg)
        if mesh_cache is not None:
            mesh_cache[mid] = mesh
    return mid, make_problem(cfg, req, mesh=mesh, **spec)


def serve_picks(count: int, pool: int, cfg: int = 5) -> np.ndarray:
    """Which of `pool` pre-generated requests each of `count` arrivals carries."""
    return rng(cfg, 0, S_PICK).integers(0, pool, size=count)


def serve_arrivals(count: int, rate: float = SERVE_RATE, cfg: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of `count` requests."""
    return np.cumsum(rng(cfg, 0, S_ARRIVAL).exponential(1.0 / rate, size=count))
