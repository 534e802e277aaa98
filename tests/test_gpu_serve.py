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


def test_concurrent_requests_for_one_object_equal_cold_runs():
    """Two requests for the same object submitted back to back into a 2-slot
    server: the second may take the object from the cache while the first's
    build is still queued on the device.  Both must equal cold runs (object
    built afresh) bit for bit."""
    rd = _lib()
    p = synth.batch_problem(1, level=5, lmax=8, N=600, M=512)
    q = synth.batch_problem(1, level=5, lmax=8, N=300, M=256)
    assert np.array_equal(p.vertices, q.vertices) and p.n == q.n
    import time
    srv = rd.Server(max_inflight=2)
    try:
        # the second and third requests arrive while the first registration
        # (which builds the object) is still running
        t1 = _submit(srv, p, object_id=3)
        time.sleep(0.02)
        t2 = _submit(srv, q, object_id=3)
        t3 = _submit(srv, q, object_id=3)
        r1, r2, r3 = srv.wait(t1), srv.wait(t2), srv.wait(t3)
        st = srv.stats()
        c1 = srv.wait(_submit(srv, p, object_id=-1))
        c2 = srv.wait(_submit(srv, q, object_id=-1))
    finally:
        srv.close()
    print("cache hits", st["cache_hits"], "misses", st["cache_misses"])
    assert st["cache_hits"] + st["cache_misses"] == 3 and st["cache_hits"] >= 1
    for a, b in ((r1, c1), (r2, c2), (r3, c2)):
        assert a["status"] == 0 and b["status"] == 0
        _same(a, b)


def test_object_cache_is_keyed_by_the_mesh_contents():
    """The same caller id for two different meshes does not share an object:
    the second request builds its own and equals its cold run."""
    rd = _lib()
    p = synth.batch_problem(0, level=4, lmax=6, N=300, M=128)
    q = synth.batch_problem(0, level=4, lmax=6, N=300, M=128)
    q.vertices = (q.vertices * np.float32(1.01)).astype(np.float32)
    srv = rd.Server(max_inflight=1)
    try:
        srv.wait(_submit(srv, p, object_id=9))
        r = srv.wait(_submit(srv, q, object_id=9))
        st = srv.stats()
        cold = srv.wait(_submit(srv, q, object_id=-1))
    finally:
        srv.close()
    assert st["cache_hits"] == 0 and st["cached_objects"] == 2
    _same(r, cold)
