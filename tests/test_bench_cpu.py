"""The measurement script's host-side logic, on the CPU: the one-GPU contract
of its command line, the algorithmic byte model and the lookup of counter
traffic, which must report nothing when the counters were taken from other
kernel source."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _per_unit(fn, unit, slots, edge):
    zero = dict(n_hits=0, n_md=0, n_seg=0, n_t3=0, n_t5=0)
    assert fn(zero, 0, 0) == {"md": 0, "seg": 0, "t3": 0, "t5": 0}
    # one unit of each quantity at a time
    for k, want in unit.items():
        got = fn(dict(zero, **{k: 1}), 0, 0)
        assert (got["md"], got["seg"], got["t3"], got["t5"]) == want, k
    one = fn(zero, 1, 0)
    assert (one["md"], one["seg"]) == slots
    assert fn(zero, 0, 1)["seg"] == edge
    # linear in every count
    c = dict(n_hits=3, n_md=5, n_seg=7, n_t3=11, n_t5=13)
    a, b = fn(c, 17, 19), fn({k: 2 * v for k, v in c.items()}, 34, 38)
    assert all(b[k] == 2 * a[k] for k in a)


def test_algorithmic_bytes_follow_the_per_unit_model():
    """md: 12 B/hit + 48 B/slot + 40 B/MD; seg: 28 B/MD + 12 B/edge + 8 B/segment;
    t3: 8 B/segment + 16 B/triplet; t5: 16 B/triplet + 12 B/quintuplet"""
    _per_unit(bench.algorithmic_bytes,
              {"n_hits": (12, 0, 0, 0), "n_md": (40, 28, 0, 0), "n_seg": (0, 8, 8, 0),
               "n_t3": (0, 0, 16, 16), "n_t5": (0, 0, 0, 12)}, (48, 0), 12)
    # the headline event's segment stage (20,767 MDs, 202,772 map edges read,
    # 43,162 segments): 3,360,036 B
    c = dict(n_hits=54937, n_md=20767, n_seg=43162, n_t3=16445, n_t5=7110)
    assert bench.algorithmic_bytes(c, 12700, 202772)["seg"] == 3360036


def test_layout_bytes_follow_the_library_layouts():
    _per_unit(bench.layout_bytes,
              {"n_hits": (28, 0, 0, 0), "n_md": (85, 77, 65, 57), "n_seg": (0, 8, 4, 0),
               "n_t3": (0, 0, 17, 17), "n_t5": (0, 0, 0, 25)}, (68, 8), 4)


def test_code_digest_ignores_comments_only():
    src = "int f(int x)\n{\n    return x + 1;   // one more\n}\n"
    d = bench.code_digest([src])
    assert bench.code_digest(["/* a note */\nint f(int x)\n{\n\n    return x + 1;\n}\n"]) == d
    assert bench.code_digest([src.replace("x + 1", "x + 2")]) != d
    assert bench.code_digest([src, ""]) != d                  # file boundaries count


def test_traffic_is_read_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    assert len(digest) == 16
    f = tmp_path / "chain_pu200_traffic.txt"
    f.write_text(f"# header: not a value\nsource_digest: {digest}\n"
                 "hbm_bytes_per_launch[k_seg<32>]: 123456\n")
    monkeypatch.setattr(bench, "TRAFFIC_DIR", str(tmp_path))
    assert bench.measured_traffic("k_seg<32>") == 123456.0
    assert bench.measured_traffic("k_seg<8>") is None          # variant not counted
    f.write_text("source_digest: 0000000000000000\n"
                 "hbm_bytes_per_launch[k_seg<32>]: 123456\n")
    assert bench.measured_traffic("k_seg<32>") is None          # other kernel source
    f.unlink()
    assert bench.measured_traffic("k_seg<32>") is None          # no summary

