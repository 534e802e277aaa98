"""Autotunes the search schedule of every supported canvas edge on this GPU and
saves it as JSON (register_tune_save), for register_tune_load or
`bench.py --schedule`.

Each edge is tuned on a synthetic registration of its size: the 32^3, 64^3
and 128^3 workloads for those edges, otherwise a registration of the uneven
batch's draw at that edge (h = 15.36 mm / n), 512 rotations.

    python -m paper_2605_21398_amd.schedules.make_schedule            # -> mi355x.json
    python -m paper_2605_21398_amd.schedules.make_schedule --out my.json --edges 64 128

Records of edges not tuned in the run are kept from the output file when it
exists.
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

EDGES = (32, 48, 60, 64, 80, 96, 120, 128, 160, 180)
WORKLOAD_OF_EDGE = {32: 1, 64: 2, 128: 3}


def problem_for(n: int):
    import synth
    if n in WORKLOAD_OF_EDGE:
        return synth.config_problem(WORKLOAD_OF_EDGE[n], 0)
    return synth.batch_problem(0, n=n, h=15.36 / n, M=512)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "mi355x.json"))
    ap.add_argument("--edges", type=int, nargs="*", default=list(EDGES))
    ap.add_argument("--max-rotations", type=int, default=1024)
    a = ap.parse_args()
    import paper_2605_21398_amd as rd
    rd.load_library()
    if os.path.exists(a.out):
        rd.register_tune_load(a.out)
    for n in a.edges:
        p = problem_for(n)
        h = rd.register_init(p.vertices, p.faces, p.touchable, p.poses, p.so3, p.n, p.h, p.center, p.radius,
                             p.length)
        try:
            rd.register_autotune(h, min(len(p.so3), a.max_rotations))
        finally:
            rd.register_free(h)
        print(n, rd.register_tuned_schedule(n), flush=True)
    rd.register_tune_save(a.out)
    print("saved", a.out)


if __name__ == "__main__":
    main()
