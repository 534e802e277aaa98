"""The allocation-free GeoBall-SF entry point (so3_geoball_sf_noalloc) against
so3_geoball_sf, through the C ABI: two calls in a row, the second smaller and
with another ball, each within the samplers' float32 bar (3e-7) of the
allocating entry point, and every sample inside its ball."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2605_21398_amd as rd
    rd.load_library()
    return rd


def test_noalloc_sampler_equals_the_allocating_one():
    import torch

    from oracle import sampling as SA
    rd = _lib()
    out = torch.full((5000, 4), float("nan"), dtype=torch.float32, device="cuda")
    for n, q0, theta_deg, gamma in ((5000, [0.3, -0.2, 0.9, 0.1], 5.0, 0.0), (777, [1.0, 0.0, 0.0, 0.0], 40.0, 1.3247)):
        theta = math.radians(theta_deg)
        ref = rd.so3_geoball_sf(n, q0, theta, gamma).cpu().numpy()
        rd.so3_geoball_sf_noalloc(n, q0, theta, gamma, out=out)
        torch.cuda.synchronize()
        got = out[:n].cpu().numpy()
        err = float(np.abs(got.astype(np.float64) - ref).max())
        same = int(np.sum(np.all(got == ref, axis=1)))
        print(f"n={n} theta={theta_deg} deg: max |noalloc - alloc| = {err:.2e}, bitwise equal samples {same}/{n}")
        assert err <= 3e-7
        q = np.asarray(q0, dtype=np.float64)
        assert SA.quat_distance(got.astype(np.float64), q / np.linalg.norm(q)).max() <= theta + 1e-6
    # the rows past the second call's n still hold the first call's samples
    assert np.isfinite(out[777:].cpu().numpy()).all()


def test_noalloc_sampler_rejects_bad_arguments():
    rd = _lib()
    for args in [(0, [1, 0, 0, 0], 0.1), (10, [0, 0, 0, 0], 0.1), (10, [1, 0, 0, 0], 0.0), (10, [1, 0, 0, 0], 2.0)]:
        with pytest.raises(rd.RegError):
            rd.so3_geoball_sf_noalloc(*args)
