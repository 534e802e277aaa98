"""GPU parity of the rotated-object search (the paper's own variant of Sec.
IV-D: the object grid O rotates about its anchor and is resampled onto the
canvas of the fixed swept occupancy S) against the oracle's variant, through
the C ABI, from the mesh.

Bars as for the rotated-S search: scores within 1e-4 of the largest |score|
of the problem, held to the oracle's interval over the voxels flagged at the
two threshold decisions (the -tau_in1 step of O on the body lattice, f_p = 0 of
S); peak indices admissible in the oracle's field (C + B reaches the interval's
low end less the tolerance); poses by the pose formula to 1e-9 mm.
"""
import math

import numpy as np
import pytest

import synth
from oracle import search as S

pytestmark = pytest.mark.gpu

TOL_REL = 1e-4
DELTA = 1e-9  # mm: flag band of the two threshold decisions (both sides evaluate them in double)


def _lib():
    import paper_2605_21398_amd as rd
    rd.load_library()
    return rd


def _handle(rd, p, so3=None, **prm):
    return rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3 if so3 is None else so3, p.n, p.h,
                            p.center, p.radius, p.length, params=dict(rotate_object=1, **prm))


def _oracle_fields(p, sel):
    """The variant's field C' and flag bound B of the selected rotations, with
    the counts of flagged lattice points of O and canvas voxels of S."""
    m = S.lattice_edge(p.n)
    Ow, fo, d = S.object_lattice(p.vertices, p.faces, p.touchable, m, p.h)
    dO = S.object_flags(Ow, fo, d, delta=DELTA)
    mf = S.swept_lattice(p.poses, p.radius, p.length, m, p.h, p.center)
    Sc = S.swept_canvas(S.swept_occupancy(mf), p.n)
    Fc = S.swept_canvas(S.swept_flags(mf, delta=DELTA), p.n)
    CB = [S.score_bounds_object(Sc, Fc, Ow, dO, p.so3[r], p.n, p.h) for r in sel]
    return CB, int((dO > 0).sum()), int(Fc.sum())


def _flat(e, n):
    d = np.mod(e, n)
    return (d[:, 2] * n + d[:, 1]) * n + d[:, 0]


def _check(p, sc, sh, po, sel, CB, tol, label):
    """Scores inside the oracle's intervals, peaks admissible, poses by the
    pose formula of the GPU's own shift.  Returns the number of rotations whose
    interval is wider than tol."""
    lo, hi = np.array([S.score_interval(C, B) for C, B in CB]).T
    s = sc[sel]
    e = -sh[sel]                      # the field index of the reported shift
    flat = _flat(e, p.n)
    err = np.maximum(lo - tol - s, s - hi - tol)
    wide = int(np.sum(hi - lo > tol))
    print(f"{label}: {len(sel)} rotations, tol {tol:.3e}, max |score - oracle| "
          f"{np.abs(s - 0.5 * (lo + hi)).max():.3e}, intervals wider than tol {wide}")
    assert err.max() <= 0.0, (int(np.argmax(err)), float(err.max()))
    for i, ((C, B), l) in enumerate(zip(CB, lo)):
        adm = set(S.peak_admissible(C, B, l, tol).tolist())
        assert int(flat[i]) in adm, (sel[i], int(flat[i]), sorted(adm)[:8])
    a = S.anchor(p.vertices)
    for i, r in enumerate(sel):
        R, t = S.pose_from_object_shift(p.so3[r], e[i], a, p.center, p.h)
        q = np.asarray(p.so3[r], dtype=np.float64)
        assert np.allclose(po[r, :4], q / np.linalg.norm(q), atol=1e-12)
        assert np.abs(po[r, 4:] - t).max() < 1e-9
        assert np.allclose(synth.quat_to_mat(po[r, :4]), R, atol=1e-12)
    return wide


@pytest.mark.parametrize("rescore", [0, 1])
def test_rotobj_config1_end_to_end(rescore):
    """Config 1 (32^3) from the mesh: every one of the 64 rotations against the
    oracle's variant; rescore = 1 re-scores every rotation's candidates exactly
    by sampling the rotated object lattice voxel by voxel."""
    rd = _lib()
    p = synth.config_problem(1, 0)
    h = _handle(rd, p, rescore=rescore)
    try:
        sc, sh, po = [t.cpu().numpy() for t in rd.score_rotations(h)]
        st = rd.register_search_stats(h)
    finally:
        rd.register_free(h)
    sel = list(range(len(p.so3)))
    CB, nO, nS = _oracle_fields(p, sel)
    print(f"flagged lattice points of O {nO}, flagged canvas voxels of S {nS}; search stats {st}")
    tol = TOL_REL * np.abs(np.array([C.max() for C, _ in CB])).max()
    wide = _check(p, sc, sh, po, sel, CB, tol, f"rotated object, config 1, rescore {rescore}")
    assert wide <= 2
    assert st["uncertain"] == 0
    if rescore:
        assert st["rescored"] == len(sel)


@pytest.mark.parametrize("cfg,n_samples", [(2, 8), (3, 4)])
def test_rotobj_full_size_sampled(cfg, n_samples):
    """Configs 2 (64^3, 1024 rotations) and 3 (128^3, 4096 rotations) from the
    mesh, in the launch configuration of a whole-set call: strided rotations
    and the GPU's best against the oracle's variant."""
    rd = _lib()
    p = synth.config_problem(cfg, 0)
    h = _handle(rd, p)
    try:
        sc, sh, po = [t.cpu().numpy() for t in rd.score_rotations(h)]
        st = rd.register_search_stats(h)
    finally:
        rd.register_free(h)
    M = len(p.so3)
    sel = sorted(set(np.linspace(0, M - 1, n_samples).astype(int).tolist()) | {int(np.argmax(sc))})
    CB, nO, nS = _oracle_fields(p, sel)
    print(f"config {cfg}: flagged O {nO}, flagged S {nS}; search stats {st}")
    tol = TOL_REL * max(np.abs(np.array([C.max() for C, _ in CB])).max(), np.abs(sc).max())
    _check(p, sc, sh, po, sel, CB, tol, f"rotated object, config {cfg}")
    assert st["uncertain"] == 0


def test_rotobj_identity_equals_the_rotated_swept_search():
    """At R = I both searches correlate O's canvas block with S's canvas block
    in opposite orders: C'[e] = C[-e] between the two handles' float32 fields
    within the tolerance, equal scores within it, and the same pose when the
    peaks coincide."""
    rd = _lib()
    p = synth.config_problem(1, 0)
    so3 = np.array([[1.0, 0.0, 0.0, 0.0], p.q_gt], dtype=np.float32)
    hv = _handle(rd, p, so3=so3)
    hs = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, so3, p.n, p.h, p.center, p.radius, p.length)
    try:
        Cv = rd.register_debug_correlation(hv, 0).cpu().numpy().astype(np.float64)
        Cs = rd.register_debug_correlation(hs, 0).cpu().numpy().astype(np.float64)
        sv, shv, pv = [t.cpu().numpy() for t in rd.score_rotations(hv)]
        ss, shs, ps = [t.cpu().numpy() for t in rd.score_rotations(hs)]
    finally:
        rd.register_free(hv)
        rd.register_free(hs)
    n = p.n
    idx = (-np.arange(n)) % n
    Csr = Cs[np.ix_(idx, idx, idx)]
    tol = TOL_REL * np.abs(Cs).max()
    print(f"identity: max |C'[e] - C[-e]| = {np.abs(Cv - Csr).max():.3e} (tol {tol:.3e}); "
          f"scores {sv[0]:.6f} / {ss[0]:.6f}")
    assert np.abs(Cv - Csr).max() <= tol
    assert abs(float(sv[0]) - float(ss[0])) <= tol
    if np.array_equal(shv[0], shs[0]):
        assert np.abs(pv[0] - ps[0]).max() < 1e-9


def test_rotobj_rejects_grid_injection():
    rd = _lib()
    p = synth.config_problem(1, 0, M=4)
    h = _handle(rd, p)
    try:
        m = S.lattice_edge(p.n)
        import torch
        Sw = torch.zeros(m ** 3, dtype=torch.uint8, device="cuda")
        with pytest.raises(rd.RegError, match="rotated-object"):
            rd.register_set_grids(h, None, Sw)
    finally:
        rd.register_free(h)


def test_rotobj_recovers_the_truth_on_a_fine_canvas():
    """The config-1 problem at 64^3, h = 0.2 mm, with the true rotation in the
    set: the variant's pose lies within a voxel of the truth (at the problem's
    own 0.4 mm the interpolated -rho step biases the rotated-O peak, as the
    oracle shows)."""
    rd = _lib()
    p = synth.config_problem(1, 0, M=8)
    so3 = np.concatenate([p.so3, p.q_gt[None, :]]).astype(np.float32)
    p.n, p.h = 64, 0.2
    h = _handle(rd, p, so3=so3)
    try:
        sc, sh, po = [t.cpu().numpy() for t in rd.score_rotations(h)]
    finally:
        rd.register_free(h)
    r = len(so3) - 1
    a = S.anchor(p.vertices)
    Rg = synth.quat_to_mat(p.q_gt)
    R = synth.quat_to_mat(po[r, :4])
    err = np.linalg.norm((R @ a + po[r, 4:]) - (Rg @ a + p.t_gt))
    print(f"truth rotation: anchor error {err:.3f} mm (h {p.h}); best rotation {int(np.argmax(sc))}")
    assert err < p.h * math.sqrt(3) / 2 + 1e-9


def _eager(rd, h):
    sc, _, po = rd.score_rotations(h, shift=False)
    top = rd.register_top_k(h, sc, 16)
    starts = po[top.long()]
    out, J, _ = rd.refine_se3(h, starts)
    return dict(scores=sc.cpu().numpy(), poses=po.cpu().numpy(), top=top.cpu().numpy(), refined=out.cpu().numpy(),
                J=J.cpu().numpy())


def test_rotobj_served_and_batched_equal_the_direct_path():
    """The rotated-object search through the server (params.rotate_object on
    the request) and captured in a batch graph gives the direct call's peaks,
    poses and refined poses bit for bit."""
    rd = _lib()
    ps = [synth.batch_problem(i, level=4, lmax=6, N=400, M=128) for i in range(2)]
    hs = [_handle(rd, p) for p in ps]
    try:
        ref = [_eager(rd, h) for h in hs]
        b = rd.Batch(hs, top_k=16, graph_rounds=8, branches=2)
        try:
            for rep in range(2):
                b.run()
                for i in range(len(hs)):
                    got = b.outputs(i)
                    for k in ("scores", "poses", "top", "refined", "J"):
                        assert np.array_equal(got[k], ref[i][k]), (rep, i, k)
        finally:
            b.close()
    finally:
        for h in hs:
            rd.register_free(h)
    srv = rd.Server(max_inflight=2)
    try:
        got = [srv.wait(srv.submit(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius,
                                   p.length, params=dict(rotate_object=1))) for p in ps]
    finally:
        srv.close()
    for r, e in zip(got, ref):
        assert r["status"] == 0
        assert np.array_equal(r["top_rot"], e["top"])
        assert np.array_equal(r["top_pose"], e["poses"][e["top"]])
        assert np.array_equal(r["refined_pose"], e["refined"])
        assert np.array_equal(r["refined_J"], e["J"])


@pytest.mark.parametrize("n,h", [(16, 0.8), (48, 0.3), (60, 0.25), (80, 0.2), (96, 0.16), (120, 0.128), (160, 0.096),
                                 (180, 0.0853)])
def test_rotobj_every_edge(n, h):
    """Every other compiled canvas edge (ragged batches, the composite-radix
    transforms, one plane workgroup per CU from 160 up): two rotations from
    the mesh against the oracle's variant."""
    rd = _lib()
    p = synth.config_problem(1, 1, n=n, h=h, M=16)
    p.so3 = p.so3[:2]
    hd = _handle(rd, p, batch=8)
    try:
        sc, sh, po = [t.cpu().numpy() for t in rd.score_rotations(hd)]
        st = rd.register_search_stats(hd)
    finally:
        rd.register_free(hd)
    sel = [0, 1]
    CB, nO, nS = _oracle_fields(p, sel)
    tol = TOL_REL * np.abs(np.array([C.max() for C, _ in CB])).max()
    _check(p, sc, sh, po, sel, CB, tol, f"rotated object, n = {n} (flagged O {nO}, S {nS})")
    assert st["uncertain"] == 0


def test_rotobj_rotation_set_swap_equals_a_fresh_handle():
    """register_set_rotations on a rotated-object handle (the local search's
    path) stores the new set transposed like register_init does: its scores
    and poses equal a fresh handle's on that set, bit for bit."""
    rd = _lib()
    p = synth.config_problem(1, 0, M=16)
    q2 = synth.config_problem(1, 2, M=16).so3
    h1 = _handle(rd, p)
    h2 = _handle(rd, p, so3=q2)
    try:
        rd.register_set_rotations(h1, q2)
        a = [t.cpu().numpy() for t in rd.score_rotations(h1)]
        b = [t.cpu().numpy() for t in rd.score_rotations(h2)]
    finally:
        rd.register_free(h1)
        rd.register_free(h2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
