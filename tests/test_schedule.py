"""CPU checks of the schedule records (host-only calls, no device): the tuned
MI355X schedules shipped with the package load, every supported edge has a
valid record, and save -> load reproduces them."""
import json
import os

import paper_2605_21398_amd as rd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCHEDULES = os.path.join(ROOT, "paper_2605_21398_amd", "schedules", "mi355x.json")
EDGES = (32, 48, 60, 64, 80, 96, 120, 128, 160, 180)


def test_shipped_schedules_cover_every_edge():
    recs = {r["n"]: r for r in json.load(open(SCHEDULES))}
    assert sorted(recs) == list(EDGES)
    rd.register_tune_load(SCHEDULES)
    for n in EDGES:
        s = rd.register_tuned_schedule(n)
        r = recs[n]
        assert s["tuned"], n
        assert s["batch"] == r["batch"] and s["batch"] % 8 == 0
        assert s["lanes"] == r["lanes"] in (1, 2)
        assert s["pass1_workgroup"] == rd.PLANE_VARIANTS[r["pv1"]]
        assert s["pass3_workgroup"] == rd.PLANE_VARIANTS[r["pv3"]]
        assert s["z_threads"] == rd.Z_THREADS[r["zv"]]
        # above 128 only the widest plane workgroup fits one plane per CU
        if n > 128:
            assert s["pass1_workgroup"] == s["pass3_workgroup"] == (1024, 4)


def test_save_then_load_round_trip(tmp_path):
    rd.register_tune_load(SCHEDULES)
    out = tmp_path / "again.json"
    rd.register_tune_save(str(out))
    a = {r["n"]: r for r in json.load(open(SCHEDULES))}
    b = {r["n"]: r for r in json.load(open(out))}
    assert sorted(a) == sorted(b)
    for n in a:
        for k in ("batch", "lanes", "pv1", "pv3", "zv"):
            assert a[n][k] == b[n][k], (n, k)


def test_malformed_schedule_file_is_rejected(tmp_path):
    bad = tmp_path / "bad.json"
    bad.write_text('[ {"n": 64, "batch": 64} ]')
    try:
        rd.register_tune_load(str(bad))
    except rd.RegError:
        return
    raise AssertionError("a schedule entry without its variants was accepted")
