"""FP64 oracle of the global grid-correlation search (Sec. IV of the paper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module; the HIP path never does.

Readings of the paper taken here (each listed in the design notes):
  * the deep-penetration value is -rho with rho = 50 (a penalty);
  * S(y) = 1 iff min_i f_p(T_i^{-1} y) <= 0 (inside-inclusive);
  * the score is the correlation C[d] = sum_k O[k] S[k + d] of Eq. (xcorr),
    whose FFT form is F^{-1}(conj(F(O)) * F(S));
  * the correlation is circular on the n^3 canvas; the padded (linear)
    variant of Sec. IV-B is the same search on an edge n >= n_o + n_s - 1
    (linear_edge), where no shift wraps (linear_correlate is its definition);
  * the swept grid is the one rotated: S_w is built once on a world lattice and
    trilinearly resampled per rotation, while O and its spectrum stay fixed;
    the paper's own variant, where O rotates and S stays on a world canvas,
    is at the end of this module;
  * anchor a = mean of the mesh vertices; canvas x_k = a + h (k - n/2);
  * ties: lowest flat index (kz*n + ky)*n + kx inside a rotation, lowest
    rotation index across rotations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import _clib


@dataclass
class GridParams:
    """Table I values: tau_out1 = 0.5 mm, tau_in1 = 0.2 mm, penalty 50."""
    tau_out1: float = 0.5
    tau_in1: float = 0.2
    rho: float = 50.0


# ---------------------------------------------------------------- probe

def probe_sdf(x, y, z, r: float, L: float):
    """Capped-cylinder SDF f_p in the probe frame (tip disk at the origin, axis
    +z, length L, radius r); negative inside.  Vectorised over numpy arrays."""
    x, y, z = np.asarray(x, float), np.asarray(y, float), np.asarray(z, float)
    q1 = np.hypot(x, y) - r
    q2 = np.abs(z - 0.5 * L) - 0.5 * L
    return np.minimum(np.maximum(q1, q2), 0.0) + np.hypot(np.maximum(q1, 0.0), np.maximum(q2, 0.0))


def quat_to_mat(q) -> np.ndarray:
    """R(q / |q|) for a quaternion (w, x, y, z)."""
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


# ---------------------------------------------------------------- grids

def anchor(vertices) -> np.ndarray:
    """Geometry centre a: the mean of the mesh vertices (FP64)."""
    return np.asarray(vertices, dtype=np.float64).mean(axis=0)


def canvas_points(n: int, h: float, a) -> np.ndarray:
    """x_k = a + h (k - n/2) for k in {0..n-1}^3, rows in flat order (kz, ky, kx)."""
    k = np.arange(n, dtype=np.float64) - n / 2
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    return np.stack([a[0] + h * kx, a[1] + h * ky, a[2] + h * kz], axis=-1).reshape(-1, 3)


def lattice_edge(n: int) -> int:
    """m = 2 ceil((sqrt(3) n + 2)/2): every rotated canvas point and its trilinear
    taps fall inside the m^3 lattice."""
    return 2 * math.ceil((math.sqrt(3.0) * n + 2.0) / 2.0)


def object_points(vertices, faces, touchable, pts, prm: GridParams = GridParams()):
    """O(x), f_o(x), d(x) at arbitrary points, brute force over every face;
    inside = generalised winding number >= 1/2 (Sec. IV-A)."""
    V = np.ascontiguousarray(vertices, dtype=np.float32)
    F = np.ascontiguousarray(faces, dtype=np.int32)
    T = None if touchable is None else np.ascontiguousarray(touchable, dtype=np.uint8)
    P = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    O = np.empty(len(P))
    fo = np.empty(len(P))
    d = np.empty(len(P))
    _clib.lib().orc_object_points(_clib.ptr(V), len(V), _clib.ptr(F), len(F), _clib.ptr(T),
                                  _clib.ptr(P), len(P), prm.tau_out1, prm.tau_in1, prm.rho,
                                  _clib.ptr(O), _clib.ptr(fo), _clib.ptr(d))
    return O, fo, d


def object_grid(vertices, faces, touchable, n: int, h: float, prm: GridParams = GridParams(),
                band: float | None = None):
    """O[k] on the canvas (shape (n,n,n), index [kz,ky,kx]) with f_o and d.
    Exact wherever the distances lie inside the band (default tau_out1 + h)."""
    V = np.ascontiguousarray(vertices, dtype=np.float32)
    F = np.ascontiguousarray(faces, dtype=np.int32)
    T = None if touchable is None else np.ascontiguousarray(touchable, dtype=np.uint8)
    a = np.ascontiguousarray(anchor(V))
    band = prm.tau_out1 + h if band is None else band
    O = np.empty(n ** 3)
    fo = np.empty(n ** 3)
    d = np.empty(n ** 3)
    _clib.lib().orc_object_grid(_clib.ptr(V), len(V), _clib.ptr(F), len(F), _clib.ptr(T), n, h,
                                _clib.ptr(a), prm.tau_out1, prm.tau_in1, prm.rho, band,
                                _clib.ptr(O), _clib.ptr(fo), _clib.ptr(d))
    sh = (n, n, n)
    return O.reshape(sh), fo.reshape(sh), d.reshape(sh)


def swept_points(poses, r: float, L: float, pts) -> np.ndarray:
    """min_i f_p(T_i^{-1} y) at arbitrary world points, brute force (Sec. IV-A)."""
    Pz = np.ascontiguousarray(poses, dtype=np.float32)
    P = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(P))
    _clib.lib().orc_swept_points(_clib.ptr(Pz), len(Pz), r, L, _clib.ptr(P), len(P), _clib.ptr(out))
    return out


def lattice_points(m: int, h: float, wc) -> np.ndarray:
    """y_j = wc + h (j - m/2), rows in flat order (jz, jy, jx)."""
    k = np.arange(m, dtype=np.float64) - m / 2
    jz, jy, jx = np.meshgrid(k, k, k, indexing="ij")
    return np.stack([wc[0] + h * jx, wc[1] + h * jy, wc[2] + h * jz], axis=-1).reshape(-1, 3)


def swept_lattice(poses, r: float, L: float, m: int, h: float, wc, margin: float | None = None):
    """min_i f_p on the m^3 world lattice (shape (m,m,m)); exact wherever it is
    below `margin` (default h), +inf marks points farther than that from every
    pose.  S_w = (result <= 0)."""
    Pz = np.ascontiguousarray(poses, dtype=np.float32)
    w = np.ascontiguousarray(wc, dtype=np.float64)
    out = np.empty(m ** 3)
    _clib.lib().orc_swept_lattice(_clib.ptr(Pz), len(Pz), r, L, m, h, _clib.ptr(w),
                                  h if margin is None else margin, _clib.ptr(out))
    return out.reshape(m, m, m)


def swept_occupancy(minf) -> np.ndarray:
    """S = 1 where the swept probe covers the point (f_p <= 0)."""
    return (np.asarray(minf) <= 0.0).astype(np.float64)


# ------------------------------------------------------ per-rotation score

def resample(S_w, q, n: int, h: float, a, wc):
    """S_r[k] = S_w at the world point R (x_k - a) + wc, trilinear on the
    lattice y_j = wc + h (j - m/2), taps outside the lattice count as 0
    (Sec. IV-D: rotate and resample by trilinear interpolation).  S_w may be a
    list of lattices of one edge m; each is resampled with the same weights and
    a list is returned."""
    grids = list(S_w) if isinstance(S_w, (list, tuple)) else [S_w]
    m = grids[0].shape[0]
    R = quat_to_mat(q)
    k = np.arange(n, dtype=np.float64) - n / 2
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    X = h * np.stack([kx, ky, kz], axis=-1).reshape(-1, 3)         # x_k - a
    Y = X @ R.T + np.asarray(wc, dtype=np.float64)                 # world points
    y0 = np.asarray(wc, dtype=np.float64) - h * (m / 2)
    U = (Y - y0) / h                                               # lattice coords (x,y,z)
    I = np.floor(U).astype(np.int64)
    Fr = U - I
    outs = [np.zeros(len(U)) for _ in grids]
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                ix, iy, iz = I[:, 0] + cx, I[:, 1] + cy, I[:, 2] + cz
                w = ((Fr[:, 0] if cx else 1 - Fr[:, 0]) * (Fr[:, 1] if cy else 1 - Fr[:, 1])
                     * (Fr[:, 2] if cz else 1 - Fr[:, 2]))
                ok = (ix >= 0) & (ix < m) & (iy >= 0) & (iy < m) & (iz >= 0) & (iz < m)
                for G, out in zip(grids, outs):
                    val = np.zeros(len(U))
                    val[ok] = G[iz[ok], iy[ok], ix[ok]]
                    out += w * val
    outs = [o.reshape(n, n, n) for o in outs]
    return outs if isinstance(S_w, (list, tuple)) else outs[0]


def correlate(O: np.ndarray, S: np.ndarray) -> np.ndarray:
    """C[d] = sum_k O[k] S[(k + d) mod n], circular, unnormalised, computed as
    F^{-1}(conj(F(O)) * F(S)) with numpy's FFT."""
    n = O.shape
    return np.fft.irfftn(np.conj(np.fft.rfftn(O)) * np.fft.rfftn(S), s=n, axes=(0, 1, 2))


def correlate_direct(O: np.ndarray, S: np.ndarray) -> np.ndarray:
    """The same correlation by its definition (Eq. xcorr), O(n^6): tiny grids only."""
    n = O.shape[0]
    C = np.zeros(O.shape)
    for dz in range(n):
        for dy in range(n):
            for dx in range(n):
                C[dz, dy, dx] = np.sum(O * np.roll(S, shift=(-dz, -dy, -dx), axis=(0, 1, 2)))
    return C


def linear_correlate(O: np.ndarray, S: np.ndarray) -> np.ndarray:
    """C_lin[d] = sum_k O[k] S[k + d] for every d in [-(n-1), n-1]^3 with S = 0
    off the grid: the correlation of the zero-padded grids (Sec. IV-B pads
    each axis to at least n_o + n_s - 1).  Axis order (dz, dy, dx), indexed by
    d + n - 1; computed as the circular correlation of the grids padded to 2n,
    where no shift in that range wraps onto the data."""
    n = O.shape[0]
    Op = np.zeros((2 * n,) * 3)
    Sp = np.zeros((2 * n,) * 3)
    Op[:n, :n, :n] = O
    Sp[:n, :n, :n] = S
    C = correlate(Op, Sp)
    idx = np.arange(-(n - 1), n) % (2 * n)
    return C[np.ix_(idx, idx, idx)]


def linear_peak(C_lin: np.ndarray):
    """(max, signed shift (dx, dy, dz)) of a linear correlation; the first
    maximum in (dz, dy, dx) order from the most negative shifts."""
    n = (C_lin.shape[0] + 1) // 2
    flat = int(np.argmax(C_lin.ravel()))
    kz, ky, kx = np.unravel_index(flat, C_lin.shape)
    return float(C_lin.ravel()[flat]), np.array([kx, ky, kz], dtype=np.int64) - (n - 1)


def probe_reach(poses, r: float, L: float, wc) -> float:
    """Largest distance from wc to a point of the probe (capped cylinder of
    radius r, tip disk at the pose origin, axis +z of length L) over the
    trajectory.  The farthest point of a disk with centre e, unit axis z and
    radius r from c lies on its rim: sqrt(((e-c).z)^2 + (|(e-c) x z| + r)^2)."""
    P = np.asarray(poses, dtype=np.float32).astype(np.float64)
    reach = 0.0
    for Pi in P:
        R = quat_to_mat(Pi[:4])
        z = R[:, 2]
        for end in (0.0, L):
            v = Pi[4:] + end * z - np.asarray(wc, dtype=np.float64)
            along = float(v @ z)
            across = float(np.linalg.norm(np.cross(v, z)))
            reach = max(reach, math.hypot(along, across + r))
    return reach


def linear_edge(vertices, poses, r: float, L: float, wc, h: float, tau_out1: float = 0.5):
    """(n_o, n_s, n_o + n_s - 1): grid extents of the object grid and of the
    rotated swept occupancy, and the edge from which the circular correlation
    is the linear one.  O vanishes beyond tau_out1 outside the mesh, so its
    support lies within the vertex radius about the anchor plus tau_out1; S_r
    lies within the probe reach about wc plus sqrt(3) h, the reach of the
    trilinear taps.  A ball of radius R about the canvas centre (a grid point)
    holds 2 floor(R/h) + 1 points along an axis."""
    V = np.asarray(vertices, dtype=np.float32).astype(np.float64)
    ro = float(np.max(np.linalg.norm(V - anchor(V), axis=1)))
    rs = probe_reach(poses, r, L, wc)
    n_o = 2 * math.floor((ro + tau_out1) / h) + 1
    n_s = 2 * math.floor(rs / h + math.sqrt(3.0)) + 1
    return n_o, n_s, n_o + n_s - 1


def support_extent(G: np.ndarray) -> int:
    """Largest per-axis extent (in grid points) of the nonzero entries of G."""
    nz = np.argwhere(G != 0)
    if len(nz) == 0:
        return 0
    return int((nz.max(axis=0) - nz.min(axis=0) + 1).max())


def peak(C: np.ndarray):
    """(max score, lowest flat index among the maxima, signed shift (dx,dy,dz))."""
    n = C.shape[0]
    flat = int(np.argmax(C.ravel()))      # numpy returns the first maximum
    kz, ky, kx = np.unravel_index(flat, C.shape)
    d = np.array([kx, ky, kz], dtype=np.int64)
    d = np.where(d >= n // 2, d - n, d)
    return float(C.ravel()[flat]), flat, d


def pose_from_shift(q, delta, a, wc, h: float):
    """Object pose x -> R x + t of a peak: R = R(q), t = wc - R a + h R delta.
    It turns sum_x O(x) S_w(R x + t) into sum_k O[k] S_r[k + delta] and reduces
    to the translation of Sec. IV-B at R = I."""
    R = quat_to_mat(q)
    t = np.asarray(wc, float) - R @ np.asarray(a, float) + h * (R @ np.asarray(delta, float))
    return R, t


def score_rotation(O, S_w, q, n, h, a, wc):
    """One rotation of the global search: resample, correlate, take the peak."""
    C = correlate(O, resample(S_w, q, n, h, a, wc))
    return peak(C)


def score_rotations(O, S_w, so3, n, h, a, wc, indices=None):
    """Scores, flat peak indices and signed shifts for the selected rotations."""
    idx = range(len(so3)) if indices is None else indices
    sc, fl, sh = [], [], []
    for r in idx:
        s, f, d = score_rotation(O, S_w, so3[r], n, h, a, wc)
        sc.append(s)
        fl.append(f)
        sh.append(d)
    return np.array(sc), np.array(fl, dtype=np.int64), np.array(sh, dtype=np.int64).reshape(-1, 3)


# ------------------------------------------- threshold decisions (flags)
#
# Two decisions of the grids are step functions of a distance: the object
# template jumps from 1 + f_o/tau_in1 (about 0) to -rho at f_o = -tau_in1, and
# the swept occupancy switches at f_p = 0.  An evaluation of the distance in
# another operation order (or precision) can take either side within its
# rounding error, so voxels within delta of a jump are flagged, and the score
# of a rotation is bounded over every combination of their two values.

def object_flags(O, fo, d, prm: GridParams = GridParams(), delta: float = 1e-4):
    """|O_alt - O| at the object voxels with |f_o + tau_in1| < delta (else 0):
    the change of O if the template takes the other side of its jump."""
    fo = np.asarray(fo, dtype=np.float64)
    near = np.abs(fo + prm.tau_in1) < delta
    shell = np.minimum(1.0 + fo / prm.tau_in1, np.maximum(0.0, 1.0 - np.asarray(d) / prm.tau_out1))
    alt = np.where(fo <= -prm.tau_in1, shell, -prm.rho)
    return np.where(near, np.abs(alt - np.asarray(O, dtype=np.float64)), 0.0)


def swept_flags(minf, delta: float = 1e-4):
    """1 at the lattice points with |min_i f_p| < delta, where the occupancy
    may take either value."""
    return (np.abs(np.asarray(minf)) < delta).astype(np.float64)


def score_bounds(O, dO, S_w, F_s, q, n: int, h: float, a, wc):
    """The correlation field C of one rotation and a bound B >= |C' - C| for
    every field C' obtained by moving flagged voxels to their other value.
    With D_r the resampled flag indicator (0 <= S_r' <= S_r + D_r, since
    resampling is linear with non-negative weights):
        C' - C = corr(O' - O, S_r') + corr(O, S_r' - S_r)
        |C' - C| <= corr(|dO|, S_r + D_r) + corr(|O|, D_r) = B."""
    S_r, D_r = resample([S_w, F_s], q, n, h, a, wc)
    C = correlate(O, S_r)
    B = np.zeros_like(C)
    if np.any(dO):
        B += correlate(dO, S_r + D_r)
    if np.any(D_r):
        B += correlate(np.abs(O), D_r)
    return C, np.maximum(B, 0.0)


def score_interval(C, B):
    """(lowest, highest) score of a rotation over the flagged alternatives:
    max (C - B) and max (C + B)."""
    return float(np.max(C - B)), float(np.max(C + B))


def peak_admissible(C, B, lo: float, tol: float) -> np.ndarray:
    """Flat indices that may be the peak of some alternative field within tol:
    C + B >= lo - tol (with no flags this is the tie band of the maximum)."""
    return np.flatnonzero((C + B).ravel() >= lo - tol)


def top_k(scores, K: int):
    """Rotation indices of the K best scores: score descending, index ascending."""
    s = np.asarray(scores, dtype=np.float64)
    order = np.lexsort((np.arange(len(s)), -s))
    return order[:K]


# ------------------------------- the paper's own variant: the object rotates
#
# Sec. IV-D as printed rotates the object grid O into each sampled orientation
# and resamples it trilinearly onto the common canvas, which holds the swept
# occupancy S unrotated; the correlation of Eq. (xcorr) then runs between the
# rotated O and the fixed S.  Here the canvas is z_k = wc + h (k - n/2) in the
# world frame, O_w is the object grid of Sec. IV-A on the body lattice
# a + h (j - m/2), and the rotated object has its anchor at the canvas centre.

def object_lattice(vertices, faces, touchable, m: int, h: float, prm: GridParams = GridParams()):
    """O_w[j] = O(a + h (j - m/2)) on the m^3 body lattice about the anchor,
    with f_o and d (shape (m,m,m), index [jz,jy,jx]): the object grid of
    Sec. IV-A on an edge-m lattice."""
    return object_grid(vertices, faces, touchable, m, h, prm)


def swept_canvas(S_w, n: int) -> np.ndarray:
    """S[k] = S_w at wc + h (k - n/2): the central n^3 block of the world
    lattice (its points coincide with the canvas points; m - n is even)."""
    m = S_w.shape[0]
    o = (m - n) // 2
    return np.asarray(S_w, dtype=np.float64)[o:o + n, o:o + n, o:o + n].copy()


def resample_object(O_w, q, n: int, h: float):
    """O_q[k] = O_w at the body point a + R^T h (k - n/2), trilinear on the
    body lattice, taps outside the lattice count as 0: the object rotated by
    R = R(q) about its anchor, the anchor at the canvas centre (Sec. IV-D).
    O_w may be a list of lattices of one edge m; each is resampled with the
    same weights and a list is returned."""
    grids = list(O_w) if isinstance(O_w, (list, tuple)) else [O_w]
    m = grids[0].shape[0]
    R = quat_to_mat(q)
    k = np.arange(n, dtype=np.float64) - n / 2
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    X = h * np.stack([kx, ky, kz], axis=-1).reshape(-1, 3)         # z_k - wc
    U = (X @ R) / h + m / 2                                        # R^T (z_k - wc) / h + m/2, as rows
    I = np.floor(U).astype(np.int64)
    Fr = U - I
    outs = [np.zeros(len(U)) for _ in grids]
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                ix, iy, iz = I[:, 0] + cx, I[:, 1] + cy, I[:, 2] + cz
                w = ((Fr[:, 0] if cx else 1 - Fr[:, 0]) * (Fr[:, 1] if cy else 1 - Fr[:, 1])
                     * (Fr[:, 2] if cz else 1 - Fr[:, 2]))
                ok = (ix >= 0) & (ix < m) & (iy >= 0) & (iy < m) & (iz >= 0) & (iz < m)
                for G, out in zip(grids, outs):
                    val = np.zeros(len(U))
                    val[ok] = G[iz[ok], iy[ok], ix[ok]]
                    out += w * val
    outs = [o.reshape(n, n, n) for o in outs]
    return outs if isinstance(O_w, (list, tuple)) else outs[0]


def score_rotation_object(S_c, O_w, q, n: int, h: float):
    """One rotation of the variant: (score, lowest flat index e among the
    maxima, signed e) of C'[e] = sum_j S[j] O_q[j + e] = F^{-1}(conj(F(S)) F(O_q)).
    The paper's C[dk] = sum_k O_q[k] S[k + dk] equals C'[-dk]: the shift of
    Eq. (xcorr) is dk = -e."""
    return peak(correlate(S_c, resample_object(O_w, q, n, h)))


def score_rotations_object(S_c, O_w, so3, n: int, h: float, indices=None):
    """Scores, flat indices e and signed e of the variant for the selected rotations."""
    idx = range(len(so3)) if indices is None else indices
    sc, fl, sh = [], [], []
    for r in idx:
        s, f, d = score_rotation_object(S_c, O_w, so3[r], n, h)
        sc.append(s)
        fl.append(f)
        sh.append(d)
    return np.array(sc), np.array(fl, dtype=np.int64), np.array(sh, dtype=np.int64).reshape(-1, 3)


def pose_from_object_shift(q, e, a, wc, h: float):
    """Object pose x -> R x + t of a peak at e: R = R(q), t = wc - R a + h dk
    with dk = -e.  The rotated object sits at x -> R (x - a) + wc on the
    canvas, and the shift dk of Eq. (xcorr) moves it by h dk (Sec. IV-B:
    t = h dk + o_s - o_o)."""
    R = quat_to_mat(q)
    t = np.asarray(wc, float) - R @ np.asarray(a, float) - h * np.asarray(e, float)
    return R, t


def score_bounds_object(S_c, F_c, O_w, dO_w, q, n: int, h: float):
    """The variant's field C' = corr(S, O_q) of one rotation and a bound
    B >= |C'' - C'| for every field C'' obtained by moving flagged voxels to
    their other value: S' differs from S only where F (the canvas block of
    the swept flags) is 1, and |O_q' - O_q| <= D_q = resample(|dO_w|)
    (resampling is linear with non-negative weights), so
        C'' - C' = corr(S' - S, O_q') + corr(S, O_q' - O_q)
        |C'' - C'| <= corr(F, |O_q| + D_q) + corr(S, D_q) = B."""
    O_q, D_q = resample_object([O_w, dO_w], q, n, h)
    C = correlate(S_c, O_q)
    B = np.zeros_like(C)
    if np.any(F_c):
        B += correlate(F_c, np.abs(O_q) + D_q)
    if np.any(D_q):
        B += correlate(S_c, D_q)
    return C, np.maximum(B, 0.0)
