"""Serving on the GPU: a registration's results are the same alone and in a
mix of uneven registrations running together (continuous batching), equal
those of the direct C-ABI path, and do not depend on whether its object came
from the resident object cache.  The kernels are deterministic (order-free
reductions and atomics), so the comparison is bitwise."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2605_21398_amd as rd
    rd.load_library()
    return rd


def _problems(count=5):
    # uneven canvases from the batch draw, smaller sets to keep the test short
    return [synth.batch_problem(i, level=4, lmax=6, N=400, M=256) for i in range(count)]


def _submit(srv, p, **kw):
    return srv.submit(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius, p.length,
                      **kw)


def _same(a, b):
    for k in ("top_rot", "top_score", "top_pose", "refined_pose", "refined_J"):
        assert np.array_equal(a[k], b[k]), k
    assert a["best_score"] == b["best_score"] and np.array_equal(a["best_pose"], b["best_pose"])


def test_results_alone_equal_results_in_the_mix():
    rd = _lib()
    ps = _problems()
    print("\ncanvases", [p.n for p in ps])
    alone = rd.Server(mode="serial")
    try:
        ref = [alone.wait(_submit(alone, p)) for p in ps]
    finally:
        alone.close()
    mix = rd.Server(max_inflight=4)
    try:
        tickets = [_submit(mix, p) for p in ps]
        got = [mix.wait(t) for t in tickets]
    finally:
        mix.close()
    overlap = 0
    for i, a in enumerate(got):
        for b in got[i + 1:]:
            overlap += a["t_start_ns"] < b["t_end_ns"] and b["t_start_ns"] < a["t_end_ns"]
    print("overlapping pairs in the mix:", overlap)
    assert overlap > 0
    for a, b in zip(ref, got):
        assert a["status"] == 0 and b["status"] == 0
        _same(a, b)


def test_server_matches_the_direct_path():
    rd = _lib()
    p = _problems(1)[0]
    srv = rd.Server(max_inflight=2)
    try:
        r = srv.wait(_submit(srv, p))
    finally:
        srv.close()
    h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius, p.length)
    try:
        sc, _, po = rd.score_rotations(h, shift=False)
        top = rd.register_top_k(h, sc, 16).cpu().numpy()
        starts = po.cpu().numpy()[top]
        out, J, _ = rd.refine_se3(h, starts)
    finally:
        rd.register_free(h)
    assert np.array_equal(r["top_rot"], top)
    assert np.array_equal(r["top_pose"], starts)
    assert np.array_equal(r["refined_pose"], out.cpu().numpy())
    assert np.array_equal(r["refined_J"], J.cpu().numpy())


def test_server_lbfgsb_refinement_matches_the_direct_path():
    """A request may ask for the paper's solver (refine = 2): the served
    result equals refine_se3_lbfgsb on a handle of its own, bit for bit."""
    rd = _lib()
    p = _problems(1)[0]
    srv = rd.Server(max_inflight=2)
    try:
        r = srv.wait(_submit(srv, p, refine="lbfgsb"))
        with pytest.raises(ValueError):
            _submit(srv, p, refine="newton")
    finally:
        srv.close()
    h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius, p.length)
    try:
        sc, _, po = rd.score_rotations(h, shift=False)
        top = rd.register_top_k(h, sc, 16).cpu().numpy()
        starts = po.cpu().numpy()[top]
        out, J, _ = rd.refine_se3(h, starts, solver="lbfgsb")
    finally:
        rd.register_free(h)
    assert np.array_equal(r["refined_pose"], out.cpu().numpy())
    assert np.array_equal(r["refined_J"], J.cpu().numpy())


def test_object_cache_hit_gives_the_same_result():
    rd = _lib()
    p = _problems(1)[0]
    q = synth.batch_problem(0, level=4, lmax=6, N=300, M=128)  # same mesh and canvas, other request
    srv = rd.Server(max_inflight=2)
    try:
        first = srv.wait(_submit(srv, p, object_id=7))
        hit = srv.wait(_submit(srv, q, object_id=7))
        st = srv.stats()
        cold = srv.wait(_submit(srv, q, object_id=-1))
    finally:
        srv.close()
    assert first["status"] == 0
    assert st["cache_hits"] >= 1 and st["cached_objects"] == 1
    _same(hit, cold)
