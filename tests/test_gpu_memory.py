"""The device memory cache: a freed handle's blocks are kept, the next handle
of the same sizes takes them without new allocations and computes the same
scores (the kernels overwrite every buffer they read), and releasing the cache
returns every block."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2605_21398_amd as rd
    rd.load_library()
    return rd


def _handle(rd, p):
    return rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius, p.length)


def test_freed_blocks_are_reused_with_identical_results():
    rd = _lib()
    rd.register_release_cached()
    assert rd.register_cached_bytes() == 0
    p = synth.config_problem(1, 0, M=64)
    h = _handle(rd, p)
    first = rd.score_rotations(h, shift=False)[0].cpu().numpy()
    rd.register_free(h)
    held = rd.register_cached_bytes()
    assert held > 0
    h = _handle(rd, p)
    try:
        # the second handle's buffers all came from the cache
        assert rd.register_cached_bytes() < held
        again = rd.score_rotations(h, shift=False)[0].cpu().numpy()
    finally:
        rd.register_free(h)
    assert np.array_equal(first, again)
    rd.register_release_cached()
    assert rd.register_cached_bytes() == 0
