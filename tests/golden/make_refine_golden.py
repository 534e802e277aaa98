"""Writes the oracle's Gauss-Newton refinement of the 16 best search peaks of
the 128^3 workload to tests/golden/refine_cfg3.npz.

Only the FP64 oracle (oracle/) and the seeded input generators (synth/) are
called.  The starts are the oracle's own top-16 (score descending, rotation
index ascending) from tests/golden/search_cfg3.npz, which
make_search_golden.py writes: each start is the pose of its rotation's peak
(oracle.search.pose_from_shift).  Each is refined by oracle.refine.refine; the
file also holds the final twist, the projected gradient there and the damping
mu when the iteration stopped (small where it converged, large where the
Gauss-Newton model kept failing, as at a kink of the objective).

    python tests/golden/make_refine_golden.py --workers 4
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import refine as Rf  # noqa: E402
from oracle import search as S  # noqa: E402

sys.path.insert(0, HERE)
from make_search_golden import input_digest  # noqa: E402

K = 16
_G = {}


def starts_from_search(p, gold, K=K):
    """(rotation indices, K x 7 start poses (unit quaternion w >= 0, t)) of the
    oracle's top-K peaks."""
    top = S.top_k(gold["cmax"], K)
    a = S.anchor(p.vertices)
    out = []
    for r in top:
        flat = int(gold["flat"][r])
        n = p.n
        d = np.array([flat % n, (flat // n) % n, flat // (n * n)], dtype=np.int64)
        d = np.where(d >= n // 2, d - n, d)
        _, t = S.pose_from_shift(p.so3[r], d, a, p.center, p.h)
        q = np.asarray(p.so3[r], dtype=np.float64)
        q = q / np.linalg.norm(q)
        if q[0] < 0:
            q = -q
        out.append(np.concatenate([q, t]))
    return np.asarray(top), np.stack(out)


def _one(k: int):
    g = _G
    st = g["starts"][k]
    pb = Rf.Problem(g["p"].vertices, g["p"].faces, g["p"].poses, g["p"].radius, g["p"].length,
                    S.quat_to_mat(st[:4]), st[4:], g["a"], g["table"])
    t0 = time.time()
    o = Rf.refine(pb)
    # projected gradient where the iteration stopped: small at a stationary
    # point, not at a kink of J where the damped steps stall
    _, gr, _ = Rf.evaluate(o.xi, pb)
    pg = float(np.abs(o.xi - Rf.project_box(o.xi - gr, Rf.RefineParams())).max())
    print(f"start {k}: J {o.J:.8f} iters {o.iters} pg {pg:.3e} mu {o.mu:.1e} in {time.time() - t0:.0f} s", flush=True)
    return k, o.R, o.p, o.J, o.iters, o.xi, pg, o.mu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=4)
    a = ap.parse_args()
    p = synth.config_problem(3, 0)
    gold = np.load(os.path.join(HERE, "search_cfg3.npz"))
    assert str(gold["digest"]) == input_digest(p), "the search golden belongs to other inputs"
    top, starts = starts_from_search(p, gold)
    _G.update(p=p, starts=starts, a=S.anchor(p.vertices), table=Rf.face_table(p.vertices, p.faces))
    t0 = time.time()
    with mp.get_context("fork").Pool(a.workers) as pool:
        res = sorted(pool.imap_unordered(_one, range(len(starts))), key=lambda x: x[0])
    out = os.path.join(HERE, "refine_cfg3.npz")
    np.savez_compressed(out, digest=np.array(input_digest(p)), rotations=top, starts=starts,
                        R=np.stack([x[1] for x in res]), p=np.stack([x[2] for x in res]),
                        J=np.array([x[3] for x in res]), iters=np.array([x[4] for x in res]),
                        xi=np.stack([x[5] for x in res]), pg=np.array([x[6] for x in res]),
                        mu=np.array([x[7] for x in res]))
    print(f"{len(res)} starts refined in {time.time() - t0:.0f} s -> {out}")


if __name__ == "__main__":
    main()
