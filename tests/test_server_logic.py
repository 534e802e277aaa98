"""Serving-loop logic on the CPU: the server's test executor (cfg.fake) runs
no device work and takes a fixed time per rotation, so admission by slots and
device footprint, arrival order, serial mode, poll/wait and cancellation are
checked without a GPU."""
import time

import numpy as np
import pytest

import paper_2605_21398_amd as rd

TET_V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float32)
TET_F = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], dtype=np.int32)


def _submit(srv, M, n=32, **kw):
    P = np.zeros((3, 7), dtype=np.float32)
    P[:, 0] = 1.0
    Q = np.zeros((M, 4), dtype=np.float32)
    Q[:, 0] = 1.0
    return srv.submit(TET_V, TET_F, None, P, Q, n, 0.4, **kw)


def _max_overlap(results):
    ev = sorted([(r["t_start_ns"], 1) for r in results] + [(r["t_end_ns"], -1) for r in results],
                key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_slots_bound_concurrency_and_admission_keeps_arrival_order():
    srv = rd.Server(max_inflight=2, fake_us_per_rotation=200.0)
    try:
        tickets = [_submit(srv, 100) for _ in range(6)]
        res = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    assert all(r["status"] == 0 for r in res)
    assert _max_overlap(res) == 2
    admits = [r["t_admit_ns"] for r in res]
    assert admits == sorted(admits)
    for r in res:
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_start_ns"] <= r["t_end_ns"]
        assert r["t_end_ns"] - r["t_start_ns"] >= 19e6  # 100 rotations x 200 us


def test_footprint_budget_limits_what_runs_together():
    probe = rd.Server(max_inflight=1, fake_us_per_rotation=1.0)
    try:
        fp = probe.wait(_submit(probe, 512, n=128))["footprint_bytes"]
    finally:
        probe.close()
    assert fp > 64 << 20  # a 128^3 registration needs tens of MB at least
    srv = rd.Server(max_inflight=4, fake_us_per_rotation=100.0, hbm_budget_bytes=int(1.5 * fp))
    try:
        tickets = [_submit(srv, 200, n=128) for _ in range(4)]
        res = [srv.wait(t) for t in tickets]
        assert srv.stats()["in_use_bytes"] == 0
    finally:
        srv.close()
    assert _max_overlap(res) == 1
    # the same requests with room for all of them overlap
    srv = rd.Server(max_inflight=4, fake_us_per_rotation=100.0, hbm_budget_bytes=8 * fp)
    try:
        res = [srv.wait(t) for t in [_submit(srv, 200, n=128) for _ in range(4)]]
    finally:
        srv.close()
    assert _max_overlap(res) >= 3


def test_serial_mode_runs_one_at_a_time():
    srv = rd.Server(max_inflight=4, mode="serial", fake_us_per_rotation=100.0)
    try:
        res = [srv.wait(t) for t in [_submit(srv, 100) for _ in range(4)]]
    finally:
        srv.close()
    assert _max_overlap(res) == 1


def test_poll_wait_and_ticket_release():
    srv = rd.Server(max_inflight=1, fake_us_per_rotation=500.0)
    try:
        t = _submit(srv, 200)  # 100 ms
        assert srv.poll(t) is None
        assert srv.wait(t, timeout_ms=1) is None
        r = srv.wait(t)
        assert r["status"] == 0 and r["n_top"] == 16
        with pytest.raises(rd.RegError) as e:
            srv.poll(t)
        assert e.value.code == rd.REG_EINVAL
    finally:
        srv.close()


def test_submit_validation_and_budget_refusal():
    srv = rd.Server(max_inflight=1, fake_us_per_rotation=1.0, hbm_budget_bytes=1 << 20)
    try:
        with pytest.raises(rd.RegError) as e:
            _submit(srv, 64)
        assert e.value.code == rd.REG_EBUSY
        with pytest.raises(rd.RegError) as e:
            _submit(srv, 64, top_k=17)
        assert e.value.code == rd.REG_EINVAL
    finally:
        srv.close()


def test_destroy_cancels_queued_and_waits_for_running():
    srv = rd.Server(max_inflight=1, fake_us_per_rotation=1000.0)
    for _ in range(5):
        _submit(srv, 100)  # 100 ms each
    time.sleep(0.02)
    t0 = time.perf_counter()
    srv.close()
    # the running registration finishes, the four queued ones are cancelled
    assert time.perf_counter() - t0 < 0.5
