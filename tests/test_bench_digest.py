"""The counter traffic that bench.py reports is tied to the search kernels'
code: a comment edit keeps the recorded digest valid, a code edit does not.
Host logic only."""
import importlib.util
import os
import shutil

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_digest_ignores_comments_but_not_code(tmp_path):
    b = _bench()
    src = os.path.join(ROOT, "paper_2605_21398_amd", "csrc")
    dst = tmp_path / "paper_2605_21398_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in b.SEARCH_SOURCES:
        shutil.copy(os.path.join(src, f), dst / f)
    b.ROOT = str(tmp_path)
    d0 = b.search_code_digest()
    assert d0 == _bench().search_code_digest()          # the copies hash like the tree
    k = dst / "search_kernels.hip"
    text = k.read_text()
    k.write_text("// a new comment line\n" + text.replace("namespace regdock {", "namespace regdock {  /* note */", 1))
    assert b.search_code_digest() == d0
    hdr = dst / "search_kernels.h"
    htext = hdr.read_text()
    assert "constexpr int KLOW = 3;" in htext
    k.write_text(text)
    hdr.write_text(htext.replace("constexpr int KLOW = 3;", "constexpr int KLOW = 2;", 1))
    assert b.search_code_digest() != d0
    hdr.write_text(htext)
    h = dst / "fft_device.h"
    k.write_text(text)
    h.write_text(h.read_text().replace("r == 15 ||", "r == 14 ||", 1))
    assert b.search_code_digest() != d0


def test_committed_traffic_summary_matches_the_tree():
    """profiles/traffic_search_128.md was measured on the kernels' current
    code, so the bench line carries its traffic figure."""
    b = _bench()
    assert b.counter_traffic("k_rotvox_fwd_xy", 128, 64.0) is not None
