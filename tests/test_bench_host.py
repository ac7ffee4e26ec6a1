"""Host-side pieces of the benchmark (CPU): the one-GPU guard and the
algorithmic byte count of a half-sweep launch that prices the roofline."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    rec = json.loads(res.stdout.strip().splitlines()[-1])
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]


@pytest.mark.parametrize("n,N", [(3, 1), (5, 3), (7, 8), (15, 2)])
def test_halfsweep_bytes_counts_every_access_once(n, N):
    # brute force over the red nodes ((x + k) even) of an n x n grid: each reads
    # its four faces and right-hand sides f_Y, f_P per sample and f_U, and writes
    # y, p per sample and u; every black node's y and p are read once
    import bench
    faces, reads_nb, rhs, writes = set(), set(), 0, 0
    for k in range(n):
        for x in range(n):
            if (x + k) % 2:
                continue
            faces |= {("x", k, x), ("x", k, x + 1), ("y", k, x), ("y", k + 1, x)}
            for dx, dk in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                if 0 <= x + dx < n and 0 <= k + dk < n:
                    reads_nb.add((x + dx, k + dk))
            rhs += 2 * N + 1
            writes += 2 * N + 1
    black = sum(1 for k in range(n) for x in range(n) if (x + k) % 2)
    assert len(reads_nb) == black           # every black node is some red node's neighbour
    words = len(faces) * N + len(reads_nb) * 2 * N + rhs + writes
    assert bench.halfsweep_bytes(n, N, 8) == 8.0 * words
