"""Host logic of the padded (linear) variant's edge on the CPU, through the C
ABI (register_linear_edge computes on the host): the needed edge n_o + n_s - 1
equals the oracle's bit for bit on the three workloads, the returned canvas is
the smallest edge at least that large among those the header lists (the fused
plane passes' edges up to 180, the split passes' 192, 256 and 360), and a need
above 360 returns edge 0 with the need still set."""
import os
import re

import pytest

import paper_2605_21398_amd as rd
import synth
from oracle import search as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_edges():
    txt = open(os.path.join(ROOT, "include", "regdock.h")).read()
    m = re.search(r"n must be one of ([0-9, ]+)\(plane\s*\n\s*\*\s*passes in one workgroup per plane\) or ([0-9, ]+)\(split", txt)
    assert m, "edge list not found in the header"
    fused = [int(v) for v in m.group(1).replace(" ", "").split(",") if v]
    split = [int(v) for v in m.group(2).replace(" ", "").split(",") if v]
    return fused, split


def test_header_lists_the_edges():
    fused, split = header_edges()
    assert fused == [16, 32, 48, 60, 64, 80, 96, 120, 128, 160, 180]
    assert split == [192, 256, 360]


@pytest.mark.parametrize("cfg,h", [(1, None), (2, None), (3, None), (3, 0.1)])
def test_linear_edge_matches_the_oracle(cfg, h):
    rd.load_library()
    p = synth.config_problem(cfg, 0)
    hh = p.h if h is None else h
    need, edge = rd.register_linear_edge(p.vertices, p.radius, p.length, p.poses, p.center, hh)
    n_o, n_s, ref = S.linear_edge(p.vertices, p.poses, p.radius, p.length, p.center, hh)
    fused, split = header_edges()
    want = next((n for n in fused + split if n >= ref), 0)
    print(f"config {cfg}, h {hh}: n_o {n_o}, n_s {n_s}, needed {need} (oracle {ref}), edge {edge}")
    assert need == ref
    assert edge == want
    if ref > 360:
        assert edge == 0
