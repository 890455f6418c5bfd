"""bench.py's contract, checked on the host: more than one GPU is refused with a message, the headline
workload and its flop count (8 N^3 per chain product, Algorithm 1 over the packed steps of Section 5.3),
and the HBM traffic figure it takes from a committed profiler summary only while that summary's kernel
source is unchanged."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2305_14398_amd import binding as B  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_headline_workload_and_its_flop_count():
    circuits = bench.workload(11)
    assert [c.family for c in circuits] == ["qft", "dj", "dj", "dj"]
    assert all(c.n == 11 for c in circuits)
    steps = [len(B.qsim_pack_steps(c.n, c.gates)) - 1 for c in circuits]
    assert steps[0] == 71  # 11 Hadamard steps, 55 controlled phases, 5 swaps: one gate per step
    # k steps cost k - 1 products of 8 N^3 flops (the first step is expanded straight into U)
    N = 2048
    assert sum(bench.flops_of(B, c) for c in circuits) == 8.0 * N ** 3 * sum(k - 1 for k in steps)
    assert bench.flops_of(B, circuits[0]) == 8.0 * N ** 3 * 70


def test_traffic_only_while_the_profiled_source_is_unchanged():
    profile = "cgemm_fp32_3m_qft11_dj11.md"
    assert bench.counted_traffic(profile, "README.md") is None  # a different source: stale
    assert bench.counted_traffic("no_such_summary.md", "paper_2305_14398_amd/csrc/tile_f32.h") is None
    t = bench.counted_traffic(profile, "paper_2305_14398_amd/csrc/tile_f32.h")
    if t is None:
        pytest.skip("the product tile changed since its counters were taken")
    algorithmic = 3 * 8 * 2048 * 2048  # read A and B, write C (complex64, N = 2048)
    assert algorithmic <= t <= 4 * algorithmic
