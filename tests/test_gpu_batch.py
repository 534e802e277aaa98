"""Uneven batches as one captured hipGraph, and the rotation-batch autotuner.

Every replay of the graph (with eager work and synchronisations between the
replays) must reproduce, bitwise, what score_rotations, register_top_k and
refine_se3 give on each handle eagerly; the captured refinement budget is kept
small so that continuing refinements are covered too.  The rotation batch
does not change a rotation's arithmetic, so scores are bitwise equal under any
batch the autotuner picks.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2605_21398_amd as rd
    rd.load_library()
    return rd


def _handle(rd, p, **kw):
    return rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius,
                            p.length, **kw)


def _eager(rd, h):
    sc, _, po = rd.score_rotations(h, shift=False)
    top = rd.register_top_k(h, sc, 16)
    starts = po[top.long()]
    out, J, _ = rd.refine_se3(h, starts)
    return dict(scores=sc.cpu().numpy(), poses=po.cpu().numpy(), top=top.cpu().numpy(), refined=out.cpu().numpy(),
                J=J.cpu().numpy())


def test_batch_graph_replays_equal_eager_results():
    rd = _lib()
    ps = [synth.batch_problem(i, level=4, lmax=6, N=400, M=256) for i in range(4)]
    print("\ncanvases", [p.n for p in ps])
    hs = [_handle(rd, p) for p in ps]
    try:
        ref = [_eager(rd, h) for h in hs]
        b = rd.Batch(hs, top_k=16, graph_rounds=8, branches=3)
        try:
            for rep in range(3):
                b.run()
                for i in range(len(hs)):
                    got = b.outputs(i)
                    for k in ("scores", "poses", "top", "refined", "J"):
                        assert np.array_equal(got[k], ref[i][k]), (rep, i, k)
                # eager work between the replays
                rd.score_rotations(hs[rep % len(hs)], 0, 32)
                import torch
                torch.cuda.synchronize()
        finally:
            b.close()
    finally:
        for h in hs:
            rd.register_free(h)


def test_batch_graph_lbfgsb_equals_eager():
    """The same graph with the paper's solver (refine = "lbfgsb"): every replay
    equals refine_se3_lbfgsb on each handle, bit for bit."""
    rd = _lib()
    ps = [synth.batch_problem(i, level=4, lmax=6, N=400, M=256) for i in range(4, 6)]
    hs = [_handle(rd, p) for p in ps]
    try:
        ref = []
        for h in hs:
            sc, _, po = rd.score_rotations(h, shift=False)
            top = rd.register_top_k(h, sc, 16)
            out, J, _ = rd.refine_se3(h, po[top.long()], solver="lbfgsb")
            ref.append(dict(top=top.cpu().numpy(), refined=out.cpu().numpy(), J=J.cpu().numpy()))
        b = rd.Batch(hs, top_k=16, refine="lbfgsb", graph_rounds=6, branches=2)
        try:
            for rep in range(2):
                b.run()
                for i in range(len(hs)):
                    got = b.outputs(i)
                    for k in ("top", "refined", "J"):
                        assert np.array_equal(got[k], ref[i][k]), (rep, i, k)
        finally:
            b.close()
        with pytest.raises(ValueError):
            rd.Batch(hs, refine="newton")
    finally:
        for h in hs:
            rd.register_free(h)


def test_batch_abi_errors():
    rd = _lib()
    p = synth.batch_problem(0, level=4, lmax=6, N=300, M=64)
    h = _handle(rd, p)
    try:
        with pytest.raises(rd.RegError):
            rd.Batch([h], top_k=17)
        with pytest.raises(rd.RegError):
            rd.Batch([h, h])
        # a live batch captured the handle's rotation set: it cannot change
        b = rd.Batch([h], top_k=4, graph_rounds=2)
        try:
            with pytest.raises(rd.RegError) as e:
                rd.register_set_rotations(h, p.so3[:8])
            assert e.value.code == rd.REG_EBUSY
        finally:
            b.close()
        rd.register_set_rotations(h, p.so3[:8])
        assert h.n_rot == 8
    finally:
        rd.register_free(h)


def test_autotune_records_a_schedule_and_scores_do_not_depend_on_it(tmp_path):
    """The autotuner sweeps the plane and z workgroup variants, the rotation
    batch and the lanes; the recorded schedule is taken by later handles,
    survives a save/load round trip, and every schedule gives the same scores
    (bit for bit across batches and lanes; across workgroup shapes within the
    score tolerance, since the rounding order of the row and square sums
    changes)."""
    rd = _lib()
    p = synth.config_problem(2, 0, M=256)
    h = _handle(rd, p)
    try:
        B = rd.register_autotune(h, 256)
        assert B in (8, 16, 32, 64, 128, 256)
        sch = rd.register_tuned_schedule(p.n)
        print("\nschedule", sch)
        assert sch["tuned"] and sch["batch"] == B and sch["lanes"] in (1, 2)
        assert rd.register_tuned_batch(p.n) == B
        path = str(tmp_path / "schedule.json")
        rd.register_tune_save(path)
        rd.register_tune_load(path)
        assert rd.register_tuned_schedule(p.n)["batch"] == B
        ref = None
        for prm in ({}, {"batch": 8}, {"plane_variant": 1, "z_variant": 1}, {"plane_variant": 2, "z_variant": 3},
                    {"plane_variant": 3, "z_variant": 2, "lanes": 1}):
            h2 = _handle(rd, p, params=prm)
            try:
                if not prm:
                    assert h2.batch == min(B, 256)
                s2 = rd.score_rotations(h2, shift=False)[0].cpu().numpy()
            finally:
                rd.register_free(h2)
            if ref is None:
                ref = s2
            # batch and lanes change nothing in the arithmetic; the plane
            # variants split the low block's double-precision row sums and the
            # float32 sums of squares (the error windows) into other chunks,
            # so a rotation near the certification threshold may take its
            # field maximum or its exact re-score: both within the tolerance
            d = float(np.abs(s2 - ref).max())
            print(prm, "max |difference| / max |score| =", d / float(np.abs(ref).max()))
            if "plane_variant" in prm:
                assert d <= 1e-4 * np.abs(ref).max(), prm
            else:
                assert d == 0.0, prm
        with pytest.raises(rd.RegError):
            _handle(rd, p, params={"plane_variant": 4})   # (1024, 4) is not offered at 64^3
    finally:
        rd.register_free(h)
