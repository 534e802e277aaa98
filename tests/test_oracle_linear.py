"""Pins of the padded (linear) correlation variant of the search (Sec. IV-B:
each canvas axis padded to at least n_o + n_s - 1) in the oracle:

* linear_correlate against its definition, summed shift by shift;
* the circular correlation is the linear one folded modulo n (an identity of
  the two definitions, exact for any grids);
* with both supports inside boxes of n_o and n_s points and n >= n_o + n_s - 1
  every residue class holds one overlapping shift, so circular and linear
  maxima and peak shifts agree; with the canvas one point short they need not;
* linear_edge's extents hold the actual supports of the object grid and of
  resampled swept grids on the padded canvas of the smallest workload, and
  the probe reach is the farthest of densely sampled probe rims;
* the swept lattice's reach (the farthest occupied lattice point from the
  lattice centre) bounds the support of every resampled swept grid by that
  radius plus sqrt(3) voxels about the canvas centre, nearly tightly: the
  bound by which the split plane passes write rows and planes of S_r as
  zeros without sampling them.
"""
import math

import numpy as np
import pytest

import synth
from oracle import search as S


def _direct_linear(O, Sg):
    n = O.shape[0]
    C = np.zeros((2 * n - 1,) * 3)
    for dz in range(-(n - 1), n):
        for dy in range(-(n - 1), n):
            for dx in range(-(n - 1), n):
                acc = 0.0
                for kz in range(n):
                    for ky in range(n):
                        for kx in range(n):
                            jz, jy, jx = kz + dz, ky + dy, kx + dx
                            if 0 <= jz < n and 0 <= jy < n and 0 <= jx < n:
                                acc += O[kz, ky, kx] * Sg[jz, jy, jx]
                C[dz + n - 1, dy + n - 1, dx + n - 1] = acc
    return C


def test_linear_correlation_equals_its_definition():
    g = np.random.default_rng(0)
    O, Sg = g.normal(size=(4, 4, 4)), g.normal(size=(4, 4, 4))
    C = S.linear_correlate(O, Sg)
    D = _direct_linear(O, Sg)
    assert np.abs(C - D).max() < 1e-12 * np.abs(D).max()


def test_circular_is_the_linear_correlation_folded():
    g = np.random.default_rng(1)
    n = 6
    O, Sg = g.normal(size=(n, n, n)), g.normal(size=(n, n, n))
    C_lin = S.linear_correlate(O, Sg)
    fold = np.zeros((n, n, n))
    d = np.arange(-(n - 1), n)
    for iz, dz in enumerate(d):
        for iy, dy in enumerate(d):
            for ix, dx in enumerate(d):
                fold[dz % n, dy % n, dx % n] += C_lin[iz, iy, ix]
    C = S.correlate(O, Sg)
    assert np.abs(C - fold).max() < 1e-12 * np.abs(C).max()


def _boxed(g, n, w):
    """A grid of edge n whose support is a centred box of w points."""
    G = np.zeros((n, n, n))
    lo = n // 2 - w // 2
    G[lo:lo + w, lo:lo + w, lo:lo + w] = g.uniform(0.1, 1.0, size=(w, w, w))
    return G


@pytest.mark.parametrize("n_o,n_s", [(3, 5), (4, 4), (5, 6)])
def test_no_wrap_from_n_o_plus_n_s_minus_1(n_o, n_s):
    g = np.random.default_rng(n_o * 10 + n_s)
    n = n_o + n_s - 1
    O, Sg = _boxed(g, n, n_o), _boxed(g, n, n_s)
    C = S.correlate(O, Sg)
    C_lin = S.linear_correlate(O, Sg)
    assert _overlapping_per_residue(C_lin, n) == 1
    m_lin, sh_lin = S.linear_peak(C_lin)
    m, _, sh = S.peak(C)
    assert abs(m - m_lin) < 1e-12 * m_lin
    assert np.array_equal(np.mod(sh, n), np.mod(sh_lin, n))
    # one point short, some residue class holds two overlapping shifts
    Ow, Sw = _boxed(g, n - 1, n_o), _boxed(g, n - 1, n_s)
    assert _overlapping_per_residue(S.linear_correlate(Ow, Sw), n - 1) >= 2


def _overlapping_per_residue(C_lin, n):
    """Most shifts with a nonzero (overlapping, positive) linear correlation
    that fall into one residue class modulo n."""
    d = np.arange(-(n - 1), n)
    nz = np.argwhere(C_lin > 1e-9 * C_lin.max())
    counts = {}
    for z, y, x in nz:
        k = (d[z] % n, d[y] % n, d[x] % n)
        counts[k] = counts.get(k, 0) + 1
    return max(counts.values())


def test_probe_reach_is_the_farthest_rim_point():
    g = np.random.default_rng(4)
    q = g.normal(size=(5, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    poses = np.concatenate([q, g.normal(size=(5, 3)) * 3.0], axis=1).astype(np.float32)
    wc = np.array([0.3, -0.2, 0.1])
    r, L = 0.5, 8.0
    reach = S.probe_reach(poses, r, L, wc)
    best = 0.0
    phi = np.linspace(0.0, 2 * np.pi, 20001)
    for P in poses.astype(np.float64):
        R = S.quat_to_mat(P[:4])
        for end in (0.0, L):
            pts = (R @ np.stack([r * np.cos(phi), r * np.sin(phi), np.full_like(phi, end)])).T + P[4:]
            best = max(best, np.linalg.norm(pts - wc, axis=1).max())
    assert best <= reach + 1e-12 and reach - best < 1e-7


def test_linear_edge_holds_the_supports_of_the_smallest_workload():
    p = synth.config_problem(1, 0)
    n_o, n_s, need = S.linear_edge(p.vertices, p.poses, p.radius, p.length, p.center, p.h)
    assert need == n_o + n_s - 1
    n = 120                                   # the smallest supported edge >= need (107)
    O, _, _ = S.object_grid(p.vertices, p.faces, p.touchable, n, p.h)
    assert 0 < S.support_extent(O) <= n_o
    m = S.lattice_edge(n)
    Sw = S.swept_occupancy(S.swept_lattice(p.poses, p.radius, p.length, m, p.h, p.center))
    a = S.anchor(p.vertices)
    ext = [S.support_extent(S.resample(Sw, q, n, p.h, a, p.center)) for q in p.so3[:3]]
    print(f"\nn_o {n_o} (object support {S.support_extent(O)}), n_s {n_s} (swept supports {ext})")
    assert all(0 < e <= n_s for e in ext)
    # on the workload's own 32^3 canvas the swept grid is clipped: it wraps
    assert n_s > p.n


def test_lattice_reach_bounds_the_rotated_swept_support():
    p = synth.config_problem(1, 0)
    n = 120                                   # the padded canvas of the smallest workload
    m = S.lattice_edge(n)
    Sw = S.swept_occupancy(S.swept_lattice(p.poses, p.radius, p.length, m, p.h, p.center))
    occ = np.argwhere(Sw > 0)                 # (z, y, x) of occupied lattice points
    reach4 = int(((2 * occ - m) ** 2).sum(axis=1).max())
    bound = 0.5 * math.sqrt(reach4) + math.sqrt(3.0)
    a = S.anchor(p.vertices)
    k = np.arange(n) - n / 2
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    radius = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    far = []
    for q in p.so3[:4]:
        Sr = S.resample(Sw, q, n, p.h, a, p.center)
        far.append(float(radius[Sr != 0].max()))
    print(f"\nlattice reach {0.5 * math.sqrt(reach4):.2f} voxels, bound {bound:.2f}, farthest nonzero {far}")
    assert max(far) <= bound
    assert min(far) >= bound - 2.0 * math.sqrt(3.0)
    # the bound leaves a good part of the padded canvas's rows empty
    rows = (ky[:, :, 0] ** 2 + kz[:, :, 0] ** 2) > bound ** 2
    assert rows.mean() > 0.2
