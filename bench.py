#!/usr/bin/env python3
"""Throughput of the global SO(3) search on one MI355X.

A step is one registration request through the whole hot path with its inputs
already in HBM: object grid and spectrum, swept occupancy, every SO(3) sample
scored (rotate + voxelise, forward FFT, spectral product, inverse FFT, argmax),
poses, top-16, and the SE(3) refinement of those 16 starts.  Default workload:
128^3 canvas at 0.12 mm, 4096 SO(3) samples, 2000 noisy probe poses,
10242-vertex perturbed-sphere mesh (synthetic).

Prints one JSON line: value = rotations scored per second over the timed steps;
roofline = the dominant per-rotation kernel's algorithmic HBM bytes per launch
over its mean launch time (HIP events on the library's stream); cpu_baseline =
the FP64 oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the oracle's processes run one BLAS thread each (set before numpy loads)
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

HBM_PEAK_GBPS = 8000.0
METRIC = "SO(3) rotations scored/sec at 128^3 (GB/s vs HBM peak); p50/p99 request latency"
KERNELS = {0: "k_rotvox_fwd_xy", 1: "k_zpass", 2: "k_inv_xy_argmax"}
# search schedules tuned on an MI355X (paper_2605_21398_amd/schedules/make_schedule.py)
SCHEDULE_FILE = os.path.join(ROOT, "paper_2605_21398_amd", "schedules", "mi355x.json")


def workload_name(p, cfg):
    return (f"config {cfg}: {p.n}^3 canvas, h {p.h} mm, {len(p.so3)} SO(3) samples, {len(p.poses)} probe poses, "
            f"{len(p.vertices)}-vertex mesh")


_ORC = {}


def _oracle_rotation(r):
    """One rotation of the oracle's search (grids from the pool's parent)."""
    from oracle import search as S
    g = _ORC
    t = time.perf_counter()
    S.score_rotation(g["O"], g["Sw"], g["so3"][r], g["n"], g["h"], g["a"], g["wc"])
    return time.perf_counter() - t


def host_cores() -> int:
    """Host cores the oracle's process pool uses: the CPU share of the process
    (at most 16, the share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_search_rate(p, n_sample: int, cores: int):
    """The oracle's search on `n_sample` strided rotations of p: (setup s,
    rotations/s on `cores` processes (numpy FFTs, one thread each), rotations)."""
    import multiprocessing as mp

    from oracle import search as S
    t0 = time.perf_counter()
    O, _, _ = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    Sw = S.swept_occupancy(S.swept_lattice(p.poses, p.radius, p.length, S.lattice_edge(p.n), p.h, p.center))
    setup = time.perf_counter() - t0
    _ORC.update(O=O, Sw=Sw, so3=p.so3, n=p.n, h=p.h, a=S.anchor(p.vertices), wc=p.center)
    M = len(p.so3)
    idx = list(range(0, M, max(1, M // n_sample)))[:n_sample]
    t1 = time.perf_counter()
    if cores == 1:
        for r in idx:
            _oracle_rotation(r)
    else:
        with mp.get_context("fork").Pool(cores) as pool:
            pool.map(_oracle_rotation, idx, chunksize=1)
    return setup, len(idx) / (time.perf_counter() - t1), len(idx)


def cpu_baseline(p, args, starts, evals: int, small):
    """The FP64 oracle as it stands, on the host cores.  The headline workload:
    setup grids, a strided sample of rotations on a pool over all cores
    (extrapolated linearly to the full set) and one refinement objective
    evaluation times the number the refinement of all starts made; the same
    search on one core; the two smaller workloads' searches over all their
    rotations."""
    import numpy as np

    from oracle import refine as Rf
    from oracle import search as S
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    cores = host_cores()
    setup, rate, n_all = oracle_search_rate(p, args.cpu_sample, cores)
    _, rate1, n_one = oracle_search_rate(p, max(2, args.cpu_sample // 32), 1)
    M = len(p.so3)
    a = S.anchor(p.vertices)
    q = starts[0]
    pb = Rf.Problem(p.vertices, p.faces, p.poses, p.radius, p.length, S.quat_to_mat(q[:4]), q[4:], a)
    t3 = time.perf_counter()
    Rf.evaluate(np.zeros(6), pb)
    per_eval = time.perf_counter() - t3
    full = setup + M / rate + evals * per_eval
    omp = int(os.environ.get("OMP_NUM_THREADS", "1"))
    out = {"value": M / full, "unit": "rotations/s", "cores": cores, "kind": "oracle",
           "sample": (f"object grid + swept lattice ({setup:.2f} s), {n_all} strided rotations of {M} on a pool of "
                      f"{cores} processes (numpy FFTs in FP64, one thread each: {rate:.2f} rotations/s) extrapolated "
                      f"to all {M}, and one refinement objective evaluation ({per_eval:.2f} s, distance queries on "
                      f"{omp} OpenMP thread(s)) times the {evals} evaluations of the {len(starts)} starts"),
           "search_rotations_per_s": {"all_cores": rate, "one_core": rate1, "cores": cores,
                                      "rotations_timed": {"all_cores": n_all, "one_core": n_one}}}
    for cfg, q_small in small.items():
        _, r, n = oracle_search_rate(q_small, len(q_small.so3), cores)   # every rotation
        out[f"config{cfg}_search_rotations_per_s"] = {"value": r, "rotations_timed": n, "cores": cores,
                                                      "n": q_small.n}
    return out


SEARCH_SOURCES = ("search_kernels.hip", "search_kernels.h", "fft_device.h")


def search_code_digest() -> str:
    """SHA-256 of the search kernels' code: their sources with comments and
    blank lines removed, so that an edit of comments alone keeps counters
    taken on the same code valid."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2605_21398_amd", "csrc")
    sha = hashlib.sha256()
    for f in SEARCH_SOURCES:
        text = open(os.path.join(csrc, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", l).rstrip() for l in text.splitlines()]
        sha.update("\n".join(l for l in lines if l.strip()).encode())
    return sha.hexdigest()


def counter_traffic(kernel: str, n: int, rotations_per_launch: float):
    """HBM bytes per launch of `kernel` at edge n from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's counters), or
    None when there is none, its launches held another number of rotations, or
    the kernels' code has changed since."""
    import re
    path = os.path.join(ROOT, "profiles", "traffic_search_128.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    data = json.loads(m.group(1))
    if search_code_digest() != data.get("search_code_sha256"):
        return None
    k = data["kernels"].get(f"{kernel}<{n}>")
    if k is None or k.get("rotations_per_launch") != rotations_per_launch:
        return None
    return k["traffic_bytes"]


def _gen_batch(i):
    import synth
    return synth.batch_problem(i)


def _gen_serve(req):
    import synth
    return synth.serve_problem(req)


def generate(args):
    """All synthetic workloads, made in a process pool before the GPU is touched."""
    import multiprocessing as mp

    import synth
    jobs = {}
    workers = max(1, min(16, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(workers) as pool:
        if args.batch > 0:
            jobs["batch"] = pool.map_async(_gen_batch, range(args.batch))
        if args.serve > 0:
            jobs["serve"] = pool.map_async(_gen_serve, range(args.serve_pool))
        small = {c: pool.apply_async(synth.config_problem, (c,)) for c in (1, 2) if c != args.config}
        main_p = synth.config_problem(args.config)
        out = {k: v.get() for k, v in jobs.items()}
        out["small"] = {c: v.get() for c, v in small.items()}
    out["main"] = main_p
    return out


def batch_bench(rd, torch, probs, args):
    """The uneven batch: the recorded schedule per canvas edge (autotuned here
    where none is recorded), all registrations (search + top-16 + refinement)
    captured in one graph and replayed, against the same work issued eagerly
    handle after handle."""
    import numpy as np
    mk = lambda p, **kw: rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center,
                                          p.radius, p.length, **kw)
    tuned = {}
    for p in probs:
        if p.n not in tuned:
            rec = rd.register_tuned_schedule(p.n)
            if rec["tuned"]:
                tuned[p.n] = rec["batch"]
                continue
            h = mk(p)
            tuned[p.n] = rd.register_autotune(h, 256)
            rd.register_free(h)
    hs = [mk(p) for p in probs]
    try:
        t0 = time.perf_counter()
        for h in hs:
            sc, _, po = rd.score_rotations(h, shift=False)
            top = rd.register_top_k(h, sc, 16)
            rd.refine_se3(h, po[top.long()])
        torch.cuda.synchronize()
        eager = time.perf_counter() - t0
        b = rd.Batch(hs, top_k=16, graph_rounds=64)
        try:
            b.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.batch_reps):
                b.run()
            torch.cuda.synchronize()
            graph = (time.perf_counter() - t0) / args.batch_reps
        finally:
            b.close()
    finally:
        for h in hs:
            rd.register_free(h)
    rot = sum(len(p.so3) for p in probs)
    return {"registrations": len(probs), "rotations": rot, "canvases": sorted({p.n for p in probs}),
            "tuned_batch": {str(k): v for k, v in sorted(tuned.items())},
            "graph_ms": graph * 1e3, "graph_rotations_per_s": rot / graph,
            "eager_ms": eager * 1e3, "eager_rotations_per_s": rot / eager,
            "work": "per registration: every rotation scored, top-16, refinement of the 16 starts"}


def _serve_run(rd, pool, arrivals, pick, mode, slots, window=None):
    """Feed Poisson arrivals (times in s; request i takes pool[pick[i]]) to a
    server and collect the results.  With a window (s), submission stops at
    its end, the server is closed once the requests running then finish (the
    queue is cancelled), and only requests completed inside the window count.
    Returns (results, wall s, queue-depth samples (t, queued, running),
    offered rotations)."""
    import threading

    srv = rd.Server(max_inflight=slots, mode=mode)
    tickets, depth = [], []
    t0 = time.perf_counter()
    stop = threading.Event()

    def feed():
        for i, t in enumerate(arrivals):
            if window is not None and t > window:
                break
            d = t - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            mid, p = pool[pick[i]]
            tickets.append((pick[i], srv.submit(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center,
                                                p.radius, p.length, object_id=mid)))

    def watch():
        while not stop.is_set():
            st = srv.stats()
            depth.append((time.perf_counter() - t0, st["queued"], st["running"]))
            stop.wait(0.25)

    th, tw = threading.Thread(target=feed), threading.Thread(target=watch)
    th.start()
    tw.start()
    th.join()
    res = []
    if window is None:
        res = [(k, srv.wait(t)) for k, t in tickets]
        wall = time.perf_counter() - t0
    else:
        end_ns = None
        while time.perf_counter() - t0 < window:
            time.sleep(0.01)
        for k, t in tickets:
            r = srv.poll(t)
            if r is not None:
                res.append((k, r))
        wall = window
    stop.set()
    tw.join()
    st = srv.stats()
    srv.close()
    offered = sum(len(pool[pick[i]][1].so3) for i in range(len(tickets)))
    return res, wall, depth, offered, st


def serve_bench(rd, pool, args):
    """Poisson streams of registrations (config 5's size mix: requests drawn
    from a pool of pre-generated ones, 20 objects) through the server, serial
    (one at a time, the plain path) against continuous (shared search streams,
    least remaining work first): at a rate the serial path sustains, every
    request timed from submission to completion; and at the workload's 200/s
    over a fixed window, offered against served rotations/s and the queue
    depth."""
    import numpy as np

    import synth
    # serial service time of the pool (each request once, after a warm pass)
    srv = rd.Server(mode="serial")
    try:
        for mid, p in pool[:4]:
            srv.wait(srv.submit(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius,
                                p.length, object_id=mid))
        svc = []
        for mid, p in pool:
            r = srv.wait(srv.submit(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius,
                                    p.length, object_id=mid))
            svc.append((r["t_end_ns"] - r["t_start_ns"]) / 1e9)
    finally:
        srv.close()
    mean_svc = float(np.mean(svc))
    capacity = 1.0 / mean_svc
    out = {"pool": len(pool), "pool_rotations": sum(len(p.so3) for _, p in pool),
           "serial_service_ms": {"mean": mean_svc * 1e3, "p50": float(np.percentile(svc, 50)) * 1e3,
                                 "max": float(np.max(svc)) * 1e3},
           "serial_capacity_per_s": capacity, "runs": []}
    rate = args.serve_load * capacity
    for label, r, count, window in (("sustained", rate, args.serve, None),
                                    ("overloaded", args.serve_rate, int(args.serve_rate * args.serve_window) + 1,
                                     args.serve_window)):
        arr = synth.serve_arrivals(count, r)
        pick = synth.serve_picks(count, len(pool))
        run = {"label": label, "offered_per_s": r, "arrivals": int(np.sum(arr <= window)) if window else count}
        if window:
            run["window_s"] = window
        for mode, slots in (("serial", 1), ("continuous", args.serve_slots)):
            res, wall, depth, offered, st = _serve_run(rd, pool, arr, pick, mode, slots, window)
            lat = np.array([(x["t_end_ns"] - x["t_submit_ns"]) / 1e6 for _, x in res]) if res else np.zeros(1)
            served_rot = sum(len(pool[k][1].so3) for k, _ in res)
            d = np.array([q for _, q, _ in depth]) if depth else np.zeros(1)
            run[mode] = {"completed": len(res), "p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)), "served_per_s": len(res) / wall,
                         "offered_rotations_per_s": offered / wall, "served_rotations_per_s": served_rot / wall,
                         "queue_depth": {"mean": float(d.mean()), "max": int(d.max()), "last": int(d[-1])},
                         "slots": slots, "cache_hits": st["cache_hits"], "cache_misses": st["cache_misses"]}
            print(f"bench: serving {label} {mode} done", file=sys.stderr, flush=True)
        out["runs"].append(run)
    out["workload"] = ("Poisson arrivals; requests drawn from a pool of pre-generated ones with config 5's mix: "
                       "20 objects; 90 % canvases 48..128 with 512..4096 rotations, 10 % 160^3 with 8192; "
                       "300..2000 probe poses; search + top-16 + refinement per request; the sustained rate is "
                       f"{args.serve_load:.2f} x the serial capacity measured on the pool")
    return out


def local_search_bench(rd, torch, p, args):
    """Local search in the orientation subspace (Sec. IV-C, IV-D): GeoBall-SF
    samples in the geodesic ball of radius theta around the global maximum,
    scored on the same handle (same object grid and swept lattice)."""
    import numpy as np

    def sync():
        torch.cuda.synchronize()
        return time.perf_counter()

    def angle_deg(q):
        q = np.asarray(q, dtype=np.float64)
        q = q / np.linalg.norm(q)
        return float(np.degrees(2.0 * np.arccos(min(1.0, abs(float(np.dot(q, p.q_gt)))))))

    h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius, p.length)
    try:
        sc, _, po = rd.score_rotations(h)
        sc, po = sc.cpu().numpy(), po.cpu().numpy()
        g = int(np.argmax(sc))
        q_star = po[g, :4]
        theta = np.radians(args.local_theta)
        t0 = sync()
        local = rd.so3_geoball_sf(args.local, q_star, theta)
        t1 = sync()
        rd.register_set_rotations(h, local)
        rd.score_rotations(h)  # warm
        times = []
        for _ in range(2):
            t2 = sync()
            sc2, _, po2 = rd.score_rotations(h)
            times.append(sync() - t2)
        sc2, po2 = sc2.cpu().numpy(), po2.cpu().numpy()
        b = int(np.argmax(sc2))
        score_s = min(times)
        return {"samples": args.local, "theta_deg": args.local_theta, "sampler": "GeoBall-SF (gamma = n)",
                "sampler_ms": (t1 - t0) * 1e3, "score_ms": score_s * 1e3, "rotations_per_s": args.local / score_s,
                "best_score_global": float(sc[g]), "best_score_local": float(sc2[b]),
                "rotation_error_deg": {"global": angle_deg(q_star), "local": angle_deg(po2[b, :4])}}
    finally:
        rd.register_free(h)


def small_config_bench(rd, torch, probs, reps: int = 5):
    """The smaller workloads' searches (32^3 with 64 rotations, 64^3 with 1024):
    rotations/s of score_rotations over all rotations with the tuned schedule,
    and the model HBM traffic rate (4 half-spectra per rotation plus the object
    spectrum once per batch); at these sizes the intermediates stay in the
    L2/MALL caches, so the HBM roofline does not bind."""
    out = {}
    for cfg, p in sorted(probs.items()):
        h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius,
                             p.length)
        try:
            if not rd.register_tuned_schedule(p.n)["tuned"]:
                rd.register_autotune(h, len(p.so3))
        finally:
            rd.register_free(h)
        h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius,
                             p.length)
        try:
            rd.score_rotations(h, shift=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                rd.score_rotations(h, shift=False)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            info = rd.register_info(h)
            st = rd.register_search_stats(h)
        finally:
            rd.register_free(h)
        M = len(p.so3)
        H8 = info["spectrum_elems"] * 8
        model = (4 * H8 + H8 / info["batch"]) * M
        out[f"config{cfg}"] = {"workload": workload_name(p, cfg), "rotations_per_s": M / dt, "ms_per_call": dt * 1e3,
                               "model_GBps": model / dt / 1e9, "model_frac": model / dt / 1e9 / HBM_PEAK_GBPS,
                               "schedule": rd.register_tuned_schedule(p.n),
                               "search_stats_per_call": {k: v / (reps + 1) for k, v in st.items()}}
    return out


def _pose_errors(p, po):
    """Rotation angle (deg) and anchor displacement (mm) of FP64 poses
    (quaternion, translation) against the problem's ground truth."""
    import numpy as np
    from scipy.spatial.transform import Rotation

    a = p.vertices.astype(np.float64).mean(axis=0)
    Rg = Rotation.from_quat(np.roll(p.q_gt, -1)).as_matrix()
    R = Rotation.from_quat(np.roll(po[:4], -1)).as_matrix()
    ang = float(np.degrees(Rotation.from_matrix(R.T @ Rg).magnitude()))
    return ang, float(np.linalg.norm(R @ a + po[4:] - (Rg @ a + p.t_gt)))


def sampler_bench(rd, torch, p, M: int):
    """Global search with the workload's Sobol->Hopf set against a
    Super-Fibonacci set of the same size (Sec. IV-C) on one handle: the best
    peak's pose error and the best of the top-16."""
    import numpy as np

    h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3[:M], p.n, p.h, p.center, p.radius,
                         p.length)
    try:
        out = {}
        for name, so3 in (("sobol_hopf", None), ("super_fibonacci", rd.so3_super_fibonacci(M))):
            if so3 is not None:
                rd.register_set_rotations(h, so3)
            sc, _, po = rd.score_rotations(h)
            top = rd.register_top_k(h, sc, 16).cpu().numpy()
            po = po.cpu().numpy()
            errs = [_pose_errors(p, po[t]) for t in top]
            q = (p.so3[:M] if so3 is None else so3.cpu().numpy()).astype(np.float64)
            q /= np.linalg.norm(q, axis=1, keepdims=True)
            nearest = float(np.degrees(2.0 * np.arccos(min(1.0, np.abs(q @ p.q_gt).max()))))
            out[name] = {"best": {"deg": errs[0][0], "mm": errs[0][1]}, "nearest_sample_deg": nearest,
                         "top16_min_deg": min(e[0] for e in errs), "best_score": float(sc.max())}
        out["rotations"] = M
        return out
    finally:
        rd.register_free(h)


def linear_bench(rd, torch, M: int = 4096, M3: int = 1024):
    """The padded variant of the search (Sec. IV-B) on the 32^3 (h 0.4 mm),
    64^3 (h 0.25 mm) and 128^3 (h 0.12 mm) workloads: the circular search on
    the workload's canvas against the same search on the edge
    register_linear_edge gives (n_o + n_s - 1 = 107 -> 120, 173 -> 180 and
    359 -> 360, the last on the split plane passes), where the correlation is
    linear.  Same Super-Fibonacci set (M3 rotations at 128^3); rotations/s of
    the scoring, model HBM bytes per rotation and the best peak's pose
    error."""
    out = {}
    for cfg in (1, 2):
        out[f"config{cfg}"] = _linear_one(rd, torch, cfg, M)
    out["config3"] = _linear_one(rd, torch, 3, M3)
    return out


def _linear_one(rd, torch, cfg: int, M: int):
    import numpy as np
    import synth

    p = synth.config_problem(cfg, 0)
    need, edge = rd.register_linear_edge(p.vertices, p.radius, p.length, p.poses, p.center, p.h)
    so3 = rd.so3_super_fibonacci(M)
    res = {"needed_edge": need, "rotations": M}
    for name, n in (("circular", p.n), ("linear", edge)):
        h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, so3, n, p.h, p.center, p.radius, p.length)
        try:
            rd.score_rotations(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sc, _, po = rd.score_rotations(h)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            info = rd.register_info(h)
            sc, po = sc.cpu().numpy(), po.cpu().numpy()
            b = int(np.argmax(sc))
            ang, mm = _pose_errors(p, po[b])
            H8 = info["spectrum_elems"] * 8
            # spectrum round trips per rotation: 4 on the fused plane passes;
            # the split passes write and read the plane buffer in both plane passes
            passes = 4 if n <= 180 else 8
            res[name] = {"n": n, "rotations_per_s": M / dt, "model_bytes_per_rotation": passes * H8 + H8 / info["batch"],
                         "plane_passes": "fused" if n <= 180 else "split",
                         "best": {"deg": ang, "mm": mm, "score": float(sc[b])}}
        finally:
            rd.register_free(h)
    res["cost_ratio"] = res["circular"]["rotations_per_s"] / res["linear"]["rotations_per_s"]
    return res


def rotate_object_bench(rd, torch, p, reps: int = 3):
    """The paper's own form of the search (Sec. IV-D: the object grid rotates
    onto the canvas of the fixed swept grid) against the default (the swept
    grid rotates) on the workload's rotation set: rotations/s of the scoring
    (best of reps whole-set calls), the best peak's pose error and score."""
    import numpy as np

    out = {"rotations": len(p.so3)}
    for name, rot_obj in (("rotate_swept", 0), ("rotate_object", 1)):
        h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius,
                             p.length, params=dict(rotate_object=rot_obj))
        try:
            rd.score_rotations(h)
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(reps):
                t0 = time.perf_counter()
                sc, _, po = rd.score_rotations(h)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            sc, po = sc.cpu().numpy(), po.cpu().numpy()
            b = int(np.argmax(sc))
            ang, mm = _pose_errors(p, po[b])
            out[name] = {"rotations_per_s": len(p.so3) / best, "ms_per_call": best * 1e3,
                         "best": {"deg": ang, "mm": mm, "score": float(sc[b])}}
        finally:
            rd.register_free(h)
    out["cost_ratio"] = out["rotate_swept"]["rotations_per_s"] / out["rotate_object"]["rotations_per_s"]
    return out


def isolated_launches(rd, torch, p, dev_args, reps: int = 8):
    """Mean event-timed launch of each search pass when it runs alone: calls of
    one batch each stay on one lane, so no other pass shares the GPU."""
    h = rd.register_init(*dev_args, p.n, p.h, p.center, p.radius, p.length)
    try:
        B = rd.register_info(h)["batch"]
        rd.score_rotations(h, 0, B)
        rd.register_set_timing(h, True)
        for r in range(reps):
            rd.score_rotations(h, (r * B) % max(1, len(p.so3) - B + 1), B)
        return {KERNELS[k]: ms / la for k, (ms, la, ro) in rd.register_get_timing(h).items() if la}
    finally:
        rd.register_free(h)


def solver_bench(rd, torch, p, dev_args, starts, reps: int = 3):
    """The refinement of the step's 16 starts by both solvers on one handle:
    time per call (after one untimed call each) and how far apart the refined
    poses are (anchor displacement, rotation angle)."""
    import numpy as np
    from scipy.spatial.transform import Rotation

    h = rd.register_init(*dev_args, p.n, p.h, p.center, p.radius, p.length)
    try:
        res, ms, stats = {}, {}, {}
        for solver in ("gn", "lbfgsb"):
            rd.refine_se3(h, starts, solver=solver)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = rd.refine_se3(h, starts, solver=solver)
            torch.cuda.synchronize()
            ms[solver] = (time.perf_counter() - t0) / reps * 1e3
            res[solver] = [x.cpu().numpy() for x in r]
            stats[solver] = rd.register_refine_stats(h)
    finally:
        rd.register_free(h)
    a = p.vertices.astype(np.float64).mean(axis=0)
    dpos, dang = [], []
    for k in range(len(starts)):
        Ra = Rotation.from_quat(res["gn"][0][k, [1, 2, 3, 0]]).as_matrix()
        Rb = Rotation.from_quat(res["lbfgsb"][0][k, [1, 2, 3, 0]]).as_matrix()
        dpos.append(float(np.linalg.norm(Ra @ a + res["gn"][0][k, 4:] - Rb @ a - res["lbfgsb"][0][k, 4:])))
        dang.append(float(np.degrees(Rotation.from_matrix(Ra.T @ Rb).magnitude())))
    same = [i for i in range(len(starts)) if dpos[i] <= 1e-3 and dang[i] <= 1e-3]
    return {"starts": len(starts), "ms_per_call": ms,
            "rounds": {k: v["rounds"] for k, v in stats.items()},
            "accepted_steps": {k: [int(x) for x in v[2]] for k, v in res.items()},
            "best_J": {k: float(np.min(v[1])) for k, v in res.items()},
            "same_minimum_within_1e-3": len(same),
            "pose_gap_max": {"mm": max(dpos), "deg": max(dang)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=256,
                    help="strided oracle rotations of the headline workload in the CPU baseline (0: skip)")
    ap.add_argument("--tune", type=int, default=0,
                    help="1: autotune the search schedule of the workload's edge before timing (else the --schedule file)")
    ap.add_argument("--schedule", default=SCHEDULE_FILE,
                    help="tuned schedules to load (register_tune_load; '' for the library defaults)")
    ap.add_argument("--small", type=int, default=1, help="time the 32^3 and 64^3 workloads too (0: skip)")
    ap.add_argument("--batch", type=int, default=32, help="registrations of the uneven batch (0: skip)")
    ap.add_argument("--batch-reps", type=int, default=2)
    ap.add_argument("--serve", type=int, default=600, help="requests of the sustained serving run (0: skip serving)")
    ap.add_argument("--serve-pool", type=int, default=64, help="pre-generated requests the arrivals draw from")
    ap.add_argument("--serve-load", type=float, default=0.7, help="sustained rate as a share of the serial capacity")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="overloaded Poisson arrival rate (requests/s)")
    ap.add_argument("--serve-window", type=float, default=8.0, help="seconds of arrivals at the overloaded rate")
    ap.add_argument("--serve-slots", type=int, default=6)
    ap.add_argument("--variants", type=int, default=1,
                    help="Super-Fibonacci vs Sobol->Hopf and padded linear correlation (0: skip)")
    ap.add_argument("--solvers", type=int, default=1, help="compare Gauss-Newton and L-BFGS-B refinement (0: skip)")
    ap.add_argument("--local", type=int, default=5000, help="GeoBall-SF samples of the local search (0: skip)")
    ap.add_argument("--local-theta", type=float, default=5.0, help="geodesic ball radius (deg)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="issue one plain 512 MiB device copy first (the counter calibration of the traffic figure)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}); the search shards by rotation "
              "range across GPUs, which this benchmark does not launch.", file=sys.stderr)
        sys.exit(2)

    work = generate(args)
    print("bench: workloads generated", file=sys.stderr, flush=True)

    import numpy as np
    import torch

    import paper_2605_21398_amd as rd

    rd.load_library()
    torch.cuda.set_device(0)
    p = work["main"]
    if args.traffic_probe:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    dev = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dt)
    V, F, T = dev(p.vertices, torch.float32), dev(p.faces, torch.int32), dev(p.touchable, torch.uint8)
    P, Q = dev(p.poses, torch.float32), dev(p.so3, torch.float32)
    M = len(p.so3)
    K_TOP = 16
    stats = {k: [0.0, 0, 0] for k in KERNELS}
    info = {}
    sched_source = "library defaults"
    if args.schedule and not args.tune and (args.schedule != SCHEDULE_FILE or os.path.exists(args.schedule)):
        rd.register_tune_load(args.schedule)
        sched_source = os.path.relpath(args.schedule, ROOT)
    if args.tune:
        h = rd.register_init(V, F, T, P, Q, p.n, p.h, p.center, p.radius, p.length)
        try:
            rd.register_autotune(h, 512)
        finally:
            rd.register_free(h)
        print("bench: schedule tuned", file=sys.stderr, flush=True)
        sched_source = "autotuned in this run"

    refine_s = []
    score_wall = []

    def step(timing: bool):
        h = rd.register_init(V, F, T, P, Q, p.n, p.h, p.center, p.radius, p.length)
        if timing:
            rd.register_set_timing(h, True)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
        sc, sh, po = rd.score_rotations(h)
        if timing:
            torch.cuda.synchronize()
            score_wall.append(time.perf_counter() - s0)
        top = rd.register_top_k(h, sc, K_TOP)
        starts = po[top.long()]
        if timing:
            torch.cuda.synchronize()
            r0 = time.perf_counter()
        res = rd.refine_se3(h, starts)
        if timing:
            refine_s.append(time.perf_counter() - r0)
            for k, (ms, la, ro) in rd.register_get_timing(h).items():
                stats[k][0] += ms
                stats[k][1] += la
                stats[k][2] += ro
        info.update(rd.register_info(h))
        info["starts"] = starts.cpu().numpy()
        info["iters"] = res[2].cpu().numpy()
        info["J"] = res[1].cpu().numpy()
        info["refined"] = res[0].cpu().numpy()
        info.update(rd.register_refine_stats(h))
        info["search_stats"] = rd.register_search_stats(h)
        rd.register_free(h)
        return sc, top

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        step(True)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    value = args.steps * M / wall

    H8 = info["spectrum_elems"] * 8
    B = info["batch"]
    per_rot = {0: H8, 1: 2 * H8, 2: H8}       # algorithmic HBM bytes per rotation
    per_launch_extra = {0: 0, 1: H8, 2: 0}     # W read once per launch
    kern = {}
    for k, (ms, la, ro) in stats.items():
        if la == 0:
            continue
        bytes_per_launch = (per_rot[k] * ro + per_launch_extra[k] * la) / la
        avg_s = ms / la / 1e3
        kern[KERNELS[k]] = {"avg_launch_ms": ms / la, "launches": la, "rotations_per_launch": ro / la,
                            "algorithmic_bytes_per_launch": bytes_per_launch,
                            "achieved_GBps": bytes_per_launch / avg_s / 1e9, "share_of_kernel_time": ms}
    tot = sum(v["share_of_kernel_time"] for v in kern.values())
    for v in kern.values():
        v["share_of_kernel_time"] = v["share_of_kernel_time"] / tot
    dom = max(kern, key=lambda k: kern[k]["share_of_kernel_time"])
    d = kern[dom]
    # the two lanes of the search overlap batches, so the kernels' event times
    # add up to more than the phase's wall time
    score_s = float(np.mean(score_wall))
    sched = rd.register_tuned_schedule(p.n)
    model_bytes = (4 * H8 + H8 / B) * M
    out = {
        "metric": METRIC, "value": value, "unit": "rotations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload_name(p, args.config), "n": p.n, "h_mm": p.h, "rotations": M,
                   "poses": len(p.poses), "faces": len(p.faces), "batch": B, "top_k": K_TOP},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": d["achieved_GBps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": d["achieved_GBps"] / HBM_PEAK_GBPS,
                     "traffic": counter_traffic(dom, p.n, d["rotations_per_launch"]),
                     "algorithmic_bytes_per_launch": d["algorithmic_bytes_per_launch"],
                     "note": ("per-launch time in the timed region" +
                              (", where the two lanes' passes share the GPU; 'isolated' times the same launch alone"
                               if sched["lanes"] > 1 else "; one lane, so each launch has the GPU to itself"))},
        "latency_ms": {"p50": float(np.percentile(lat, 50)) * 1e3, "p99": float(np.percentile(lat, 99)) * 1e3,
                       "mode": "serial, one request at a time"},
        "score_phase": {"ms_per_step": score_s * 1e3, "rotations_per_s": M / score_s,
                        "model_GBps": model_bytes / score_s / 1e9, "model_frac": model_bytes / score_s / 1e9 / HBM_PEAK_GBPS,
                        "kernel_ms_per_step": tot / args.steps,
                        "lanes": sched["lanes"]},
        "schedule": dict(sched, source=sched_source),
        "search_stats": info["search_stats"],
        "kernels": kern,
        "refine": {"ms_per_step": float(np.mean(refine_s)) * 1e3, "starts": K_TOP, "rounds": info["rounds"],
                   "evaluations": info["evaluations"], "accepted_steps": [int(x) for x in info["iters"]],
                   "best_J": float(np.min(info["J"]))},
    }
    # pose error against the synthetic ground truth: the best search peak and
    # the refined start of least J (the paper's Table II stages)
    g_ang, g_mm = _pose_errors(p, info["starts"][0])
    r_ang, r_mm = _pose_errors(p, info["refined"][int(np.argmin(info["J"]))])
    out["accuracy"] = {"search_best": {"deg": g_ang, "mm": g_mm}, "refined_best_J": {"deg": r_ang, "mm": r_mm},
                       "note": "anchor displacement (mm) and rotation angle (deg) from the ground-truth pose; "
                               "the probe poses carry 0.05 mm / 0.2 deg noise"}
    print("bench: timed steps done", file=sys.stderr, flush=True)
    iso = isolated_launches(rd, torch, p, (V, F, T, P, Q))
    if dom in iso:
        a_iso = d["algorithmic_bytes_per_launch"] / (iso[dom] / 1e3) / 1e9
        out["roofline"]["isolated"] = {"avg_launch_ms": iso[dom], "achieved": a_iso, "frac": a_iso / HBM_PEAK_GBPS,
                                       "all_passes_ms": iso}
    if args.local > 0:
        out["local_search"] = local_search_bench(rd, torch, p, args)
        print("bench: local search done", file=sys.stderr, flush=True)
    if args.solvers:
        out["refine_solvers"] = solver_bench(rd, torch, p, (V, F, T, P, Q),
                                             torch.from_numpy(info["starts"]).to("cuda"))
        print("bench: solver comparison done", file=sys.stderr, flush=True)
    if args.variants:
        out["samplers"] = sampler_bench(rd, torch, p, len(p.so3))
        out["linear_correlation"] = linear_bench(rd, torch)
        out["rotate_object"] = rotate_object_bench(rd, torch, p)
        print("bench: sampler, linear-correlation and rotated-object variants done", file=sys.stderr, flush=True)
    if args.batch > 0:
        out["batch"] = batch_bench(rd, torch, work["batch"], args)
        print("bench: uneven batch done", file=sys.stderr, flush=True)
    if args.serve > 0:
        out["serving"] = serve_bench(rd, work["serve"], args)
        print("bench: serving done", file=sys.stderr, flush=True)
    if args.small and work.get("small"):
        out["configs"] = small_config_bench(rd, torch, work["small"])
        print("bench: smaller workloads done", file=sys.stderr, flush=True)
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(p, args, info["starts"], int(info["evaluations"]), work.get("small", {}))
        print("bench: cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
