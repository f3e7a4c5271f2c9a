"""Host-side logic that needs no GPU: the benchmark's refusal of several GPUs and the
serving loop's packing plan."""
import os
import subprocess
import sys

import numpy as np

from paper_2402_04403_amd.serve import plan_packs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _pool(sizes):
    return {gid: (n, np.zeros(s, np.int32), np.zeros(s, np.int32)) for gid, (n, s) in enumerate(sizes)}


def test_plan_packs():
    # rows + entries: 30, 300, 50, 2000, 60, 40, 900
    graphs = _pool([(10, 10), (100, 100), (10, 20), (1000, 500), (20, 20), (20, 10), (300, 300)])
    unit, members = plan_packs(graphs, pack_items=500, pack_limit=400)
    # graphs 3 (2000) and 6 (900) stand alone; 0, 1, 2, 4, 5 are packed in id order
    assert unit[3] == (3, 0) and unit[6] == (6, 0)
    packed = [g for g in sorted(graphs) if unit[g][0] < 0]
    assert packed == [0, 1, 2, 4, 5]
    assert sorted(g for m in members.values() for g in m) == packed
    for key, m in members.items():
        assert key < 0 and m == sorted(m)
        assert sum(graphs[g][0] + 2 * len(graphs[g][1]) for g in m) <= 400
        row = 0
        for g in m:  # members side by side: each starts where the previous one ends
            assert unit[g] == (key, row)
            row += graphs[g][0]
    # 0 (30) + 1 (300) + 2 (50) fill 380; 4 (60) opens the next pack with 5 (40)
    assert members == {-1: [0, 1, 2], -2: [4, 5]}


def test_plan_packs_off():
    graphs = _pool([(10, 10), (100, 100)])
    unit, members = plan_packs(graphs, pack_items=0, pack_limit=1 << 22)
    assert members == {} and unit == {0: (0, 0), 1: (1, 0)}
