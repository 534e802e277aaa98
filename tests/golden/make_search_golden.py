"""Writes the oracle's global-search results for the 64^3 and 128^3 workloads
(every rotation of each) to tests/golden/search_cfg<k>.npz.

Only the FP64 oracle (oracle/) and the seeded input generators (synth/) are
called.  Per rotation r the file holds the oracle's field maximum and its
lowest flat index, the interval [lo, hi] of the score over both values of
every flagged threshold voxel (oracle.search.score_bounds, flag band DELTA),
and the flat indices whose C + B comes within WINDOW of lo with their C + B
(the admissible peaks for any tolerance up to WINDOW).  A digest of the
generated inputs is stored so that a test can tell if the generator changed.

    python tests/golden/make_search_golden.py            # configs 2 and 3
    python tests/golden/make_search_golden.py --cfg 2 --workers 8
"""
from __future__ import annotations

import argparse
import hashlib
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
from oracle import search as S  # noqa: E402

DELTA = 1e-9       # mm, flag band of the two threshold decisions
TOL_REL = 1e-4     # score tolerance relative to the largest |score|
WINDOW_REL = 1e-3  # stored admissible window, relative to a pre-pass estimate of the largest |score|

_G = {}


def input_digest(p) -> str:
    """sha256 over the inputs the search sees."""
    h = hashlib.sha256()
    for a in (p.vertices, p.faces, p.touchable, p.poses, p.so3):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(np.array([p.n, p.h, *np.asarray(p.center, dtype=np.float64), p.radius, p.length]).tobytes())
    return h.hexdigest()


def _one(r: int):
    g = _G
    C, B = S.score_bounds(g["O"], g["dO"], g["Sw"], g["Fs"], g["so3"][r], g["n"], g["h"], g["a"], g["wc"])
    lo, hi = S.score_interval(C, B)
    flat = int(np.argmax(C.ravel()))
    adm = S.peak_admissible(C, B, lo, g["window"])
    val = (C + B).ravel()[adm]
    return r, float(C.ravel()[flat]), flat, lo, hi, adm.astype(np.int32), val


def run(cfg: int, workers: int) -> str:
    t0 = time.time()
    p = synth.config_problem(cfg, 0)
    O, fo, d = S.object_grid(p.vertices, p.faces, p.touchable, p.n, p.h)
    mf = S.swept_lattice(p.poses, p.radius, p.length, S.lattice_edge(p.n), p.h, p.center)
    _G.update(O=O, dO=S.object_flags(O, fo, d, delta=DELTA), Sw=S.swept_occupancy(mf),
              Fs=S.swept_flags(mf, delta=DELTA), so3=p.so3, n=p.n, h=p.h, a=S.anchor(p.vertices), wc=p.center)
    M = len(p.so3)
    # pre-pass: the largest |score| over a strided subset sizes the stored window
    _G["window"] = 0.0
    pre = [_one(r) for r in range(0, M, max(1, M // 32))]
    g0 = max(abs(x[1]) for x in pre)
    _G["window"] = WINDOW_REL * g0
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        res = sorted(pool.imap_unordered(_one, range(M), chunksize=4))
    cmax = np.array([x[1] for x in res])
    tol = TOL_REL * np.abs(cmax).max()
    assert tol <= _G["window"], (tol, _G["window"])
    off = np.zeros(M + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(x[5]) for x in res])
    out = os.path.join(HERE, f"search_cfg{cfg}.npz")
    np.savez_compressed(out, digest=np.array(input_digest(p)), delta=DELTA, window=_G["window"],
                        cmax=cmax, flat=np.array([x[2] for x in res], dtype=np.int64),
                        lo=np.array([x[3] for x in res]), hi=np.array([x[4] for x in res]),
                        adm_off=off, adm_idx=np.concatenate([x[5] for x in res]),
                        adm_val=np.concatenate([x[6] for x in res]),
                        n_flag_O=int((_G["dO"] > 0).sum()), n_flag_S=int(_G["Fs"].sum()))
    print(f"config {cfg}: {M} rotations in {time.time() - t0:.0f} s, tol {tol:.4e}, window {_G['window']:.4e}, "
          f"flags O {int((_G['dO'] > 0).sum())} S {int(_G['Fs'].sum())}, "
          f"intervals wider than tol {int(np.sum(np.array([x[4] - x[3] for x in res]) > tol))}"
          f" -> {out}", flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cfg", type=int, nargs="*", default=[2, 3])
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for c in a.cfg:
        run(c, a.workers)


if __name__ == "__main__":
    main()
