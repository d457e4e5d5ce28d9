"""bench.py's command-line contract that holds without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_flop_count_matches_the_block_structure():
    sys.path.insert(0, ROOT)
    import bench
    # per interval: a forward and a transposed product of 196 + 2 * 60 MACs, 2 flops each
    assert bench.pipg_flops_per_iter(20) == 19 * (4 * 316 + 428) + 171 * 20
    assert bench.pipg_flops_per_iter(2) == 1 * (4 * 316 + 428) + 171 * 2
    # with the torque: B^-_k and B^+_k have 15 x 7 entries, a node 22 entries
    assert bench.pipg_flops_per_iter(30, 7) == 29 * (4 * (196 + 2 * 105) + 428) + 9 * 22 * 30
