"""The padded (linear) correlation variant of the search (Sec. IV-B), through
the C ABI:

* register_linear_edge gives the oracle's n_o + n_s - 1, bit for bit, and the
  smallest supported edge above it (120 for the 32^3 workload, 180 for the
  64^3 one, whose probe shafts need 173 points, 360 for the 128^3 one, which
  needs 359 and runs on the split plane passes, checked against the oracle in
  tests/test_gpu_split.py);
* on that edge the device's circular search is the linear correlation: for
  the 32^3 workload at 120^3 (h 0.4 mm) and the 64^3 workload at 180^3
  (h 0.25 mm), with the oracle's grids injected, scores meet the search's bar
  (1e-4 of the largest |score|) against the oracle's zero-padded correlation
  of the same grids, and the peak shifts agree modulo n or are tied within
  that bar.
"""
import math

import numpy as np
import pytest

import synth
from oracle import search as S

pytestmark = pytest.mark.gpu

TOL_REL = 1e-4


def _lib():
    import paper_2605_21398_amd as rd
    rd.load_library()
    return rd


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_linear_edge_matches_oracle(cfg):
    rd = _lib()
    p = synth.config_problem(cfg, 0)
    need, edge = rd.register_linear_edge(p.vertices, p.radius, p.length, p.poses, p.center, p.h)
    n_o, n_s, ref = S.linear_edge(p.vertices, p.poses, p.radius, p.length, p.center, p.h)
    print(f"\nconfig {cfg}: n_o {n_o}, n_s {n_s}, needed {need}, edge {edge}")
    assert need == ref
    # the fused plane passes' edges, then the split passes' edges above 180
    supported = [16, 32, 48, 60, 64, 80, 96, 120, 128, 160, 180, 192, 256, 360]
    assert edge == next((n for n in supported if n >= ref), 0)


def test_linear_edge_rejects_bad_input():
    rd = _lib()
    p = synth.config_problem(1, 0)
    with pytest.raises(rd.RegError):
        rd.register_linear_edge(p.vertices, p.radius, p.length, p.poses, p.center, 0.0)
    with pytest.raises(rd.RegError):
        rd.register_linear_edge(p.vertices, -1.0, p.length, p.poses, p.center, p.h)
    V = p.vertices.copy()
    V[3, 1] = np.nan
    with pytest.raises(rd.RegError):
        rd.register_linear_edge(V, p.radius, p.length, p.poses, p.center, p.h)


@pytest.mark.parametrize("cfg,edge", [(1, 120), (2, 180)])
def test_padded_search_is_the_linear_correlation(cfg, edge):
    rd = _lib()
    p = synth.config_problem(cfg, 0, M=16)
    _, n = rd.register_linear_edge(p.vertices, p.radius, p.length, p.poses, p.center, p.h)
    assert n == edge
    O, _, _ = S.object_grid(p.vertices, p.faces, p.touchable, n, p.h)
    m = S.lattice_edge(n)
    Sw = S.swept_occupancy(S.swept_lattice(p.poses, p.radius, p.length, m, p.h, p.center))
    h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, n, p.h, p.center, p.radius, p.length)
    try:
        rd.register_set_grids(h, O.astype(np.float32), Sw.astype(np.uint8))
        sc, sh = [t.cpu().numpy() for t in rd.score_rotations(h, pose=False)[:2]]
    finally:
        rd.register_free(h)
    a = S.anchor(p.vertices)
    O64 = O.astype(np.float32).astype(np.float64)
    sel = [0, 7, int(np.argmax(sc))]
    lin = []
    for r in sel:
        Sr = S.resample(Sw, p.so3[r], n, p.h, a, p.center)
        lin.append(S.linear_correlate(O64, Sr))
    ref = np.array([C.max() for C in lin])
    tol = TOL_REL * np.abs(ref).max()
    print(f"\n{n}^3: |score - linear max| {np.abs(sc[sel] - ref).max():.3e} (tol {tol:.3e})")
    assert np.abs(sc[sel] - ref).max() <= tol
    for j, r in enumerate(sel):
        m_lin, sh_lin = S.linear_peak(lin[j])
        if not np.array_equal(np.mod(sh[r], n), np.mod(sh_lin, n)):
            # the GPU's residue class must hold a tied linear value (its only
            # overlapping representative, as nothing wraps)
            d = np.mod(sh[r].astype(np.int64), n)
            reps = [[x for x in (dd - n, dd) if -(n - 1) <= x <= n - 1] for dd in d]
            v = max(lin[j][z + n - 1, y + n - 1, x + n - 1] for x in reps[0] for y in reps[1] for z in reps[2])
            assert v >= m_lin - tol
