"""GPU checks of the split plane passes (row and column passes through an HBM
plane buffer; edges above 180, or reg_params.split_plane), through the C ABI.

- At 64^3 and 128^3 the split passes compute what the fused plane passes
  compute: scores within 1e-4 of the largest |score|, the same peaks up to
  ties inside that band, and float32 fields within the candidate window's
  error bound of each other; also on a padded canvas (the 32^3 workload on
  128^3) whose rows and planes beyond the swept lattice's reach the split
  passes skip.
- At 192^3 and 256^3 from the mesh, and at 360^3 (the padded, linear canvas
  of the 128^3 workload), scores and peaks against the FP64 oracle's
  intervals.
- Served and captured in a batch graph, the split passes give the direct
  call's results bit for bit.
- The reach of the swept lattice (by which the split passes skip rows and
  planes of S_r) equals the host's maximum over the same lattice.
"""
import math

import numpy as np
import pytest

import synth
from oracle import search as S

pytestmark = pytest.mark.gpu

TOL_REL = 1e-4
DELTA = 1e-9


def _lib():
    import paper_2605_21398_amd as rd
    rd.load_library()
    return rd


def _handle(rd, p, so3=None, **prm):
    return rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3 if so3 is None else so3, p.n, p.h,
                            p.center, p.radius, p.length, params=prm)


def _flat(sh, n):
    d = np.mod(sh, n)
    return (d[:, 2] * n + d[:, 1]) * n + d[:, 0]


@pytest.mark.parametrize("cfg,n,h,M", [(2, 64, 0.25, 128), (3, 128, 0.12, 128), (1, 128, 0.4, 64)])
def test_split_passes_equal_the_fused_passes(cfg, n, h, M):
    """The last case pads the 32^3 workload to 128^3, where most rows and
    planes of S_r lie beyond the swept lattice's reach: the split passes write
    them as zeros unsampled, the fused passes sample and transform them."""
    rd = _lib()
    p = synth.config_problem(cfg, 0, n=n, h=h, M=M)
    hf = _handle(rd, p)
    hs = _handle(rd, p, split_plane=1)
    try:
        sf, shf, pf = [t.cpu().numpy() for t in rd.score_rotations(hf)]
        ss, shs, ps = [t.cpu().numpy() for t in rd.score_rotations(hs)]
        Cf = rd.register_debug_correlation(hf, 0).cpu().numpy().astype(np.float64)
        Cs = rd.register_debug_correlation(hs, 0).cpu().numpy().astype(np.float64)
        stf, sts = rd.register_search_stats(hf), rd.register_search_stats(hs)
    finally:
        rd.register_free(hf)
        rd.register_free(hs)
    tol = TOL_REL * np.abs(sf).max()
    d = np.abs(sf - ss)
    print(f"n={n}: max |split - fused| score {d.max():.3e} (tol {tol:.3e}); field {np.abs(Cf - Cs).max():.3e}; "
          f"stats fused {stf} split {sts}")
    assert d.max() <= tol
    ff, fs = _flat(shf, n), _flat(shs, n)
    for r in range(len(sf)):
        if ff[r] != fs[r]:
            # a tie within the tolerance: each side's peak scores on the other side's field within it
            assert abs(float(sf[r]) - float(ss[r])) <= tol, r
    same = ff == fs
    assert np.abs(pf[same] - ps[same]).max() < 1e-9
    # the two float32 fields agree within twice the candidate window's bound
    P = np.fft.rfftn(Cf)
    k = np.abs(np.fft.fftfreq(n) * n)
    kz, ky, kx = np.meshgrid(k, k, np.arange(n // 2 + 1), indexing="ij")
    P[np.maximum(np.maximum(kx, ky), kz) <= 3] = 0
    eps = 6.0 * 2.0 ** -24 * math.sqrt(float(np.mean(np.fft.irfftn(P, s=Cf.shape, axes=(0, 1, 2)) ** 2))) \
        * math.log2(n ** 3)
    assert np.abs(Cf - Cs).max() <= 2.0 * eps + 2.0 ** -22 * np.abs(Cf).max()
    assert sts["rotations"] == stf["rotations"]


def _oracle_check(p, sc, sh, sel, label):
    O, fo, d = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    m = S.lattice_edge(p.n)
    mf = S.swept_lattice(p.poses, p.radius, p.length, m, p.h, p.center)
    dO, Fs = S.object_flags(O, fo, d, delta=DELTA), S.swept_flags(mf, delta=DELTA)
    a = S.anchor(p.vertices)
    Sw = S.swept_occupancy(mf)
    lo, hi, adm, mx = [], [], [], []
    for r in sel:
        C, B = S.score_bounds(O, dO, Sw, Fs, p.so3[r], p.n, p.h, a, p.center)
        l, u = S.score_interval(C, B)
        lo.append(l)
        hi.append(u)
        mx.append(C.max())
        adm.append((C, B, l))
    tol = TOL_REL * max(np.abs(np.array(mx)).max(), np.abs(sc).max())
    s = sc[sel]
    err = np.maximum(np.array(lo) - tol - s, s - np.array(hi) - tol)
    print(f"{label}: {len(sel)} rotations, tol {tol:.3e}, max |score - oracle| "
          f"{np.abs(s - 0.5 * (np.array(lo) + np.array(hi))).max():.3e}, flagged O {int((dO > 0).sum())}, "
          f"S {int(Fs.sum())}")
    assert err.max() <= 0.0
    fl = _flat(sh[sel], p.n)
    for i, (C, B, l) in enumerate(adm):
        assert int(fl[i]) in set(S.peak_admissible(C, B, l, tol).tolist())


@pytest.mark.parametrize("n,h", [(192, 0.08), (256, 0.06)])
def test_split_edge_from_the_mesh(n, h):
    """Canvases above the fused passes' LDS limit (192^3 at h = 0.08 mm, 256^3
    at 0.06 mm; the 256-point transforms take radix-16 passes) from the mesh,
    two rotations against the oracle's intervals."""
    rd = _lib()
    p = synth.config_problem(1, 1, n=n, h=h, M=16)
    so3 = p.so3[:2]
    hd = _handle(rd, p, so3=so3, batch=8)
    try:
        sc, sh, _ = [t.cpu().numpy() for t in rd.score_rotations(hd)]
        st = rd.register_search_stats(hd)
    finally:
        rd.register_free(hd)
    p.so3 = so3
    _oracle_check(p, sc, sh, [0, 1], f"split {n}^3")
    assert st["uncertain"] == 0


def test_linear_canvas_of_the_128_workload():
    """The padded (linear) search of the 128^3 workload: register_linear_edge
    asks for 359 and gives 360, which the split passes serve; two rotations
    (the workload's first and the GPU's best of 16) against the oracle."""
    rd = _lib()
    p = synth.config_problem(3, 0)
    need, edge = rd.register_linear_edge(p.vertices, p.radius, p.length, p.poses, p.center, p.h)
    assert (need, edge) == (S.linear_edge(p.vertices, p.poses, p.radius, p.length, p.center, p.h)[2], 360)
    so3 = p.so3[::256][:16]
    p.n = edge
    hd = _handle(rd, p, so3=so3)
    try:
        sc, sh, _ = [t.cpu().numpy() for t in rd.score_rotations(hd)]
        st = rd.register_search_stats(hd)
    finally:
        rd.register_free(hd)
    p.so3 = so3
    sel = sorted({0, int(np.argmax(sc))})
    _oracle_check(p, sc, sh, sel, "linear 360^3 (128^3 workload)")
    assert st["uncertain"] == 0


def _eager(rd, h):
    sc, _, po = rd.score_rotations(h, shift=False)
    top = rd.register_top_k(h, sc, 16)
    out, J, _ = rd.refine_se3(h, po[top.long()])
    return dict(scores=sc.cpu().numpy(), poses=po.cpu().numpy(), top=top.cpu().numpy(), refined=out.cpu().numpy(),
                J=J.cpu().numpy())


def test_split_served_and_batched_equal_the_direct_path():
    """The split plane passes through the server (params.split_plane on the
    request) and captured in a batch graph give the direct call's peaks,
    poses and refined poses bit for bit (64^3, two registrations of 128
    rotations, two lanes)."""
    rd = _lib()
    ps = [synth.batch_problem(i, level=4, lmax=6, N=400, M=128, n=64, h=0.24) for i in range(2)]
    hs = [_handle(rd, p, split_plane=1, batch=32) for p in ps]
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
                                   p.length, params=dict(split_plane=1, batch=32))) for p in ps]
    finally:
        srv.close()
    for r, e in zip(got, ref):
        assert r["status"] == 0
        assert np.array_equal(r["top_rot"], e["top"])
        assert np.array_equal(r["top_pose"], e["poses"][e["top"]])
        assert np.array_equal(r["refined_pose"], e["refined"])
        assert np.array_equal(r["refined_J"], e["J"])


def test_swept_reach_equals_the_lattice_maximum():
    """The reach kernel's integer maximum over the occupied points of the
    handle's own S_w equals the host's, bit for bit (the 32^3 workload padded
    to 128^3, m = 224), on the split and the fused passes; the rotated-object
    search refuses the query."""
    rd = _lib()
    p = synth.config_problem(1, 0, n=128, h=0.4, M=16)
    hs = _handle(rd, p, split_plane=1)
    hf = _handle(rd, p)
    ho = _handle(rd, p, rotate_object=1)
    try:
        got = rd.register_debug_swept_reach(hs)
        got_f = rd.register_debug_swept_reach(hf)
        Sw = rd.register_debug_swept(hs).cpu().numpy()
        with pytest.raises(rd.RegError) as e:
            rd.register_debug_swept_reach(ho)
        assert e.value.code == rd.REG_ENOTSUP
    finally:
        rd.register_free(hs)
        rd.register_free(hf)
        rd.register_free(ho)
    m = Sw.shape[0]
    occ = np.argwhere(Sw != 0).astype(np.int64)
    want = int(((2 * occ - m) ** 2).sum(axis=1).max())
    print(f"m {m}, occupied {len(occ)}, reach {0.5 * math.sqrt(want):.3f} voxels")
    assert got == want and got_f == want
