"""GPU parity of the global search against the FP64 oracle, through the C ABI.

Tolerances (the method's stated bar): scores within 1e-4 of the largest
|score| of the problem; peak indices exact unless the oracle's own field at the
GPU's index is within that tolerance of its maximum; integer work (top-K,
shifts of a given peak) bit-exact.

End to end (mesh in, scores out) the grids are built on the device.  Their two
threshold decisions -- the -tau_in1 jump of the object template and the swept
surface f_p = 0 -- are evaluated in double on both sides, so they agree except
within rounding of the threshold: voxels within DELTA of it are flagged by the
oracle, the tests assert that the device grids agree with the oracle's
everywhere else, and each rotation's score is bounded over both values of
every flagged voxel (oracle.search.score_bounds).  The per-kernel tests
inject the oracle's own grids.
"""
import math

import numpy as np
import pytest

import synth
from oracle import search as S

pytestmark = pytest.mark.gpu

TOL_REL = 1e-4
DELTA = 1e-9  # mm: flag band of the two threshold decisions (both sides evaluate them in double)


KLOW = 3  # the library's KLOW: frequencies with max(|kx|,|ky|,|kz|) <= KLOW are carried in double


def eps_bound(C_ref, n):
    """The error bound the library's candidate window assumes for its float32
    field, 6 * 2^-24 * rms(C_high) * log2(n^3), where C_high is the field without
    its exact low-frequency block; plus the float32 rounding of the debug output."""
    P = np.fft.rfftn(C_ref)
    k = np.abs(np.fft.fftfreq(n) * n)
    kz, ky, kx = np.meshgrid(k, k, np.arange(n // 2 + 1), indexing="ij")
    P[np.maximum(np.maximum(kx, ky), kz) <= KLOW] = 0
    Ch = np.fft.irfftn(P, s=C_ref.shape, axes=(0, 1, 2))
    return 6.0 * 2.0 ** -24 * math.sqrt(float(np.mean(Ch ** 2))) * math.log2(n ** 3) + 2.0 ** -23 * np.abs(C_ref)


def _lib():
    import paper_2605_21398_amd as rd
    rd.load_library()
    return rd


def _oracle_grids(p):
    O, fo, _ = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    m = S.lattice_edge(p.n)
    mf = S.swept_lattice(p.poses, p.radius, p.length, m, p.h, p.center)
    return O, fo, mf


def _handle(rd, p, **kw):
    return rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center,
                            p.radius, p.length, **kw)


def _check_scores(sc_gpu, fl_gpu, sc_ref, fields_ref, tol):
    """scores within tol; flat index equal or inside the tolerance band of the
    oracle's own field at that rotation."""
    assert np.abs(sc_gpu - sc_ref).max() <= tol, np.abs(sc_gpu - sc_ref).max()
    for r in range(len(sc_gpu)):
        C = fields_ref[r]
        if C is None:
            continue
        flat_ref = int(np.argmax(C.ravel()))
        if fl_gpu[r] != flat_ref:
            assert C.ravel()[fl_gpu[r]] >= C.ravel()[flat_ref] - tol


def _flat_from_shift(sh, n):
    d = np.mod(sh, n)
    return (d[:, 2] * n + d[:, 1]) * n + d[:, 0]


def _problem(cfg, item, **over):
    return synth.config_problem(cfg, item, **over)


# ------------------------------------------------------------------ grids

def _grid_agreement(rd, handle, p, O, fo, d, mf):
    """Device grids against the oracle's: the binary decisions agree outside
    the flag band, the continuous values within float32 rounding.  Returns the
    oracle's flag grids (|dO|, swept flags)."""
    Og = rd.register_debug_object_grid(handle)[0].cpu().numpy()
    Swg = rd.register_debug_swept(handle).cpu().numpy()
    dO = S.object_flags(O, fo, d, delta=DELTA)
    Fs = S.swept_flags(mf, delta=DELTA)
    okO = dO == 0
    errO = np.abs(Og.astype(np.float64) - O)
    bad_sw = (Swg != (mf <= 0)) & (Fs == 0)
    near_jump = np.abs(fo + 0.2)[errO > 1.0]
    print(f"n={p.n}: flagged O {int((~okO).sum())}, flagged S_w {int(Fs.sum())}; "
          f"max |O_gpu - O| off the flags {errO[okO].max():.2e}; S_w disagreements off the flags {int(bad_sw.sum())}; "
          f"closest jump voxels that differ: {np.sort(near_jump)[:4]}; "
          f"|f_p| of S_w disagreements: {np.sort(np.abs(mf[Swg != (mf <= 0)]))[:4]}")
    assert errO[okO].max() < 1e-4
    assert not bad_sw.any()
    assert (~okO).sum() < 1e-3 * O.size and Fs.sum() < 1e-3 * Fs.size
    return dO, Fs


@pytest.mark.parametrize("cfg,over", [(1, {}), (1, dict(n=48, h=0.3, M=16)), (1, dict(n=60, h=0.25, M=16))])
def test_object_grid_and_swept_match_oracle(cfg, over):
    rd = _lib()
    p = _problem(cfg, 0, **over)
    h = _handle(rd, p)
    O, fo, d = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    mf = S.swept_lattice(p.poses, p.radius, p.length, S.lattice_edge(p.n), p.h, p.center)
    _grid_agreement(rd, h, p, O, fo, d, mf)


def _check_intervals(sc, flat, lo, hi, adm, tol, label):
    """Every rotation: score inside [lo - tol, hi + tol] of the oracle's
    interval over the flagged alternatives, peak index admissible (adm[r]: the
    flat indices whose C + B reaches lo - tol).  Reports how many rotations
    have an interval wider than tol."""
    wide = int(np.sum(hi - lo > tol))
    err = np.maximum(lo - tol - sc, sc - hi - tol)
    print(f"{label}: {len(sc)} rotations, tol {tol:.3e}, max |score - oracle| {np.abs(sc - 0.5 * (lo + hi)).max():.3e}, "
          f"intervals wider than tol: {wide}")
    assert err.max() <= 0.0, (int(np.argmax(err)), float(err.max()))
    for r in range(len(sc)):
        assert int(flat[r]) in adm[r], (r, int(flat[r]), adm[r][:8])
    return wide
# ------------------------------------------- per-rotation path, grids injected

@pytest.mark.parametrize("n,h,M,batch,rescore", [(32, 0.4, 64, 0, 0), (32, 0.4, 64, 0, 1), (48, 0.3, 13, 8, 1),
                                                 (60, 0.25, 11, 0, 0), (64, 0.25, 16, 8, 1), (80, 0.2, 9, 0, 0),
                                                 (16, 0.8, 10, 8, 1), (96, 0.16, 5, 0, 0), (120, 0.128, 3, 8, 1),
                                                 (160, 0.096, 2, 0, 0)])
def test_correlation_field_matches_oracle(n, h, M, batch, rescore):
    """Element-wise correlation field and peak of every rotation, with the
    oracle's O and S_w injected (several tiles, ragged batches); rescore=1
    re-scores every rotation's candidates exactly."""
    rd = _lib()
    p = _problem(1, 1, n=n, h=h, M=max(16, 1 << (M - 1).bit_length()))
    p.so3 = p.so3[:M]
    handle = _handle(rd, p, params=dict(batch=batch, rescore=rescore))
    O, fo, mf = _oracle_grids(p)
    Sw = S.swept_occupancy(mf)
    rd.register_set_grids(handle, O.astype(np.float32), Sw.astype(np.uint8))
    a = S.anchor(p.vertices)
    sc, sh, po = rd.score_rotations(handle)
    sc, sh, po = sc.cpu().numpy(), sh.cpu().numpy(), po.cpu().numpy()
    fields = [S.correlate(O.astype(np.float32).astype(np.float64), S.resample(Sw, q, n, h, a, p.center)) for q in p.so3]
    ref = np.array([f.max() for f in fields])
    tol = TOL_REL * np.abs(ref).max()
    _check_scores(sc, _flat_from_shift(sh, n), ref, fields, tol)
    if rescore:
        # exact sums over float32 trilinear samples: far inside the tolerance
        assert np.abs(sc - ref).max() <= 1e-6 * np.abs(ref).max() + 1e-6
    # the float32 field of two rotations, element by element, inside the error
    # bound that sizes the library's candidate window
    for r in (0, M - 1):
        Cg = rd.register_debug_correlation(handle, r).cpu().numpy()
        ratio = (np.abs(Cg - fields[r]) / eps_bound(fields[r], n)).max()
        print(f"n={n} rot={r}: max |C_gpu - C_oracle| / bound = {ratio:.3f}")
        assert ratio <= 1.0
    st = rd.register_search_stats(handle)
    assert st["uncertain"] == 0 and st["candidates"] >= st["rotations"]
    # poses follow from the shifts in FP64
    for r in range(M):
        R, t = S.pose_from_shift(p.so3[r], sh[r], a, p.center, h)
        qn = p.so3[r].astype(np.float64) / np.linalg.norm(p.so3[r].astype(np.float64))
        assert np.allclose(po[r, :4], qn, atol=1e-12)
        assert np.allclose(po[r, 4:], t, atol=1e-9)


def test_config1_end_to_end():
    """Config 1 from the mesh: device-built grids, all 64 rotations against the
    oracle's fields (intervals over the flagged voxels), top-16."""
    rd = _lib()
    p = _problem(1, 0)
    handle = _handle(rd, p)
    sc, sh, po = [t.cpu().numpy() for t in rd.score_rotations(handle)]
    O, fo, d = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    mf = S.swept_lattice(p.poses, p.radius, p.length, S.lattice_edge(p.n), p.h, p.center)
    dO, Fs = _grid_agreement(rd, handle, p, O, fo, d, mf)
    Sw = S.swept_occupancy(mf)
    a = S.anchor(p.vertices)
    CB = [S.score_bounds(O, dO, Sw, Fs, q, p.n, p.h, a, p.center) for q in p.so3]
    lo, hi = np.array([S.score_interval(C, B) for C, B in CB]).T
    tol = TOL_REL * np.abs(np.array([C.max() for C, _ in CB])).max()
    adm = [set(S.peak_admissible(C, B, l, tol).tolist()) for (C, B), l in zip(CB, lo)]
    wide = _check_intervals(sc, _flat_from_shift(sh, p.n), lo, hi, adm, tol, "config 1 end to end")
    assert wide <= 2
    top = rd.register_top_k(handle, rd._dev(sc, __import__("torch").float32), 16).cpu().numpy()
    assert list(top) == list(S.top_k(sc, 16))


def test_top_k_ties_and_ragged():
    rd = _lib()
    p = _problem(1, 0, M=16)
    handle = _handle(rd, p)
    s = np.array([1.0, 3.0, 2.0, 3.0, -1.0, 2.0, 3.0, -5.0, 0.5], dtype=np.float32)
    import torch
    out = rd.register_top_k(handle, torch.from_numpy(s).cuda(), 12).cpu().numpy()
    assert list(out[:9]) == list(S.top_k(s, 9)) and list(out[9:]) == [-1, -1, -1]
    # an empty call enqueues nothing and leaves the outputs untouched
    sc = torch.full((4,), 7.0, device="cuda")
    rd.score_rotations(handle, 3, 0, out=(sc, None, None))
    assert (sc.cpu().numpy() == 7.0).all()
    # a single-rotation call at the end of the set (a ragged last batch of one):
    # each call certifies against its own tolerance (1e-4 of its largest score),
    # so the value may come from the float32 field or an exact re-score, both
    # within the tolerance of the full call's
    one = rd.score_rotations(handle, 15, 1)[0].cpu().numpy()
    full = rd.score_rotations(handle)[0].cpu().numpy()
    assert abs(float(one[0]) - float(full[15])) <= TOL_REL * np.abs(full).max()


def test_abi_rejects_bad_inputs():
    rd = _lib()
    p = _problem(1, 0, M=16)
    bad = p.so3.copy()
    bad[3] *= 1.1
    with pytest.raises(rd.RegError) as e:
        rd.register_init(p.vertices, p.faces, p.touchable, p.poses, bad, p.n, p.h)
    assert e.value.code == rd.REG_EINVAL
    with pytest.raises(rd.RegError) as e:
        rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, 36, p.h)
    assert e.value.code == rd.REG_ENOTSUP
    F = p.faces.copy()
    F[5, 1] = len(p.vertices)
    with pytest.raises(rd.RegError) as e:
        rd.register_init(p.vertices, F, p.touchable, p.poses, p.so3, p.n, p.h)
    assert e.value.code == rd.REG_EINVAL
    h = _handle(rd, p)
    with pytest.raises(rd.RegError) as e:
        rd.score_rotations(h, first=10, count=10)
    assert e.value.code == rd.REG_EINVAL


def test_determinism_run_to_run():
    rd = _lib()
    p = _problem(1, 0)
    h = _handle(rd, p)
    a = [t.cpu().numpy() for t in rd.score_rotations(h)]
    b = [t.cpu().numpy() for t in rd.score_rotations(h)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ------------------------------------------------------------- full size

def _sampled_full_size(cfg, n_samples, rescore=0):
    rd = _lib()
    p = _problem(cfg, 0)
    handle = _handle(rd, p, params=dict(rescore=rescore))
    sc, sh, _ = [t.cpu().numpy() if t is not None else None for t in rd.score_rotations(handle)]
    O, fo, d = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    mf = S.swept_lattice(p.poses, p.radius, p.length, S.lattice_edge(p.n), p.h, p.center)
    Sw = S.swept_occupancy(mf)
    _grid_agreement(rd, handle, p, O, fo, d, mf)
    # per-rotation path on sampled rotations, oracle grids injected
    rd.register_set_grids(handle, O.astype(np.float32), Sw.astype(np.uint8))
    sc2, sh2, _ = [t.cpu().numpy() if t is not None else None for t in rd.score_rotations(handle, pose=False)]
    a = S.anchor(p.vertices)
    M = len(p.so3)
    sel = sorted(set(np.linspace(0, M - 1, n_samples).astype(int).tolist()) | {int(np.argmax(sc2))})
    fields = [S.correlate(O.astype(np.float32).astype(np.float64), S.resample(Sw, p.so3[r], p.n, p.h, a, p.center))
              for r in sel]
    ref = np.array([f.max() for f in fields])
    tol = TOL_REL * max(np.abs(ref).max(), np.abs(sc2).max())
    _check_scores(sc2[sel], _flat_from_shift(sh2[sel], p.n), ref, fields, tol)
    Cg = rd.register_debug_correlation(handle, sel[0]).cpu().numpy()
    ratio = (np.abs(Cg - fields[0]) / eps_bound(fields[0], p.n)).max()
    print(f"config {cfg}: max |C_gpu - C_oracle| / bound = {ratio:.3f}")
    assert ratio <= 1.0
    st = rd.register_search_stats(handle)
    print(f"config {cfg}: search stats {st}")
    assert st["uncertain"] == 0
    return p, sc, sh


def test_config2_full_size_sampled():
    _sampled_full_size(2, 6)


def test_config2_full_size_sampled_exact_rescore():
    _sampled_full_size(2, 4, rescore=1)


def test_config3_full_size_sampled():
    p, sc, sh = _sampled_full_size(3, 6)
    assert np.isfinite(sc).all()


def test_two_lanes_equal_one_lane():
    """A call over many batches alternates them between the handle's two
    streams (each with its own pass buffers); calls of one batch each stay on
    one lane.  With every rotation re-scored exactly (rescore = 1; otherwise the
    certification tolerance, 1e-4 of the call's largest score, depends on how
    the rotations are split into calls) scores, shifts and poses must be
    bit-identical."""
    rd = _lib()
    p = _problem(2, 0)
    h = _handle(rd, p, params=dict(rescore=1))
    try:
        B = rd.register_info(h)["batch"]
        M = len(p.so3)
        assert M > 2 * B
        full = [t.cpu().numpy() for t in rd.score_rotations(h)]
        parts = [[], [], []]
        for b0 in range(0, M, B):
            for k, t in enumerate(rd.score_rotations(h, b0, min(B, M - b0))):
                parts[k].append(t.cpu().numpy())
    finally:
        rd.register_free(h)
    for k in range(3):
        assert np.array_equal(full[k], np.concatenate(parts[k]))


# ------------------------------------- full size, every rotation, from the mesh

GOLD = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _golden_search(cfg, p):
    """The oracle's results of every rotation (tests/golden/make_search_golden.py)."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location("make_search_golden", os.path.join(GOLD, "make_search_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    g = np.load(os.path.join(GOLD, f"search_cfg{cfg}.npz"))
    assert str(g["digest"]) == mg.input_digest(p), "golden file written for other inputs: rerun make_search_golden.py"
    return g


@pytest.mark.parametrize("cfg", [2, 3])
def test_full_size_every_rotation_matches_oracle(cfg):
    """The 64^3 (1024 rotations) and 128^3 (4096 rotations) workloads from the
    mesh, in the default launch configuration: device-built grids against the
    oracle's, then every rotation's score and peak against the oracle's field
    (interval over flagged voxels), and the top-16 against the oracle's."""
    rd = _lib()
    p = _problem(cfg, 0)
    gold = _golden_search(cfg, p)
    handle = _handle(rd, p)
    try:
        sc, sh, _ = [t.cpu().numpy() for t in rd.score_rotations(handle)]
        top = rd.register_top_k(handle, rd._dev(sc, __import__("torch").float32), 16).cpu().numpy()
        st = rd.register_search_stats(handle)
        O, fo, d = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
        mf = S.swept_lattice(p.poses, p.radius, p.length, S.lattice_edge(p.n), p.h, p.center)
        _grid_agreement(rd, handle, p, O, fo, d, mf)
    finally:
        rd.register_free(handle)
    print(f"config {cfg}: search stats {st}")
    assert st["uncertain"] == 0
    lo, hi, cmax = gold["lo"], gold["hi"], gold["cmax"]
    tol = TOL_REL * np.abs(cmax).max()
    assert tol <= float(gold["window"])
    off, idx, val = gold["adm_off"], gold["adm_idx"], gold["adm_val"]
    adm = [set(idx[off[r]:off[r + 1]][val[off[r]:off[r + 1]] >= lo[r] - tol].tolist()) for r in range(len(sc))]
    wide = _check_intervals(sc, _flat_from_shift(sh, p.n), lo, hi, adm, tol, f"config {cfg} end to end")
    assert wide <= 0.01 * len(sc)
    # top-16: every device pick could be in the oracle's top-16, and every
    # rotation certainly in it is picked
    order = np.sort(lo)[::-1]
    lo16 = order[15]
    hi17 = np.sort(hi)[::-1][16]
    for r in top:
        assert hi[r] + 2 * tol >= lo16, r
    must = np.flatnonzero(lo - 2 * tol > hi17)
    assert set(must.tolist()) <= set(top.tolist())
    print(f"config {cfg}: top-16 {list(top)}; oracle top-16 {list(S.top_k(cmax, 16))}")
