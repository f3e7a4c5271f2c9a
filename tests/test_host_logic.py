"""Host-side logic that needs no GPU: the benchmark's refusal of several GPUs, its use of
the committed counter summaries, and the serving loop's packing plan."""
import importlib.util
import json
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


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_traffic_only_for_its_kernel_and_workload(tmp_path):
    """The counter summary's HBM bytes are reported only while the kernel source hashes the
    same and the run has the algorithmic bytes per launch the counters were taken at."""
    bench = _bench()
    src = tmp_path / "k.hip"
    src.write_text("kernel v1")
    summary = tmp_path / "c.json"
    summary.write_text(json.dumps({"kernel_source_sha256": bench.source_hash(str(src)),
                                   "bytes_alg_per_launch": 1000, "hbm_bytes_per_launch": 1234.5}))
    assert bench.counters_traffic(1000, str(summary), str(src))[0] == 1234.5
    assert bench.counters_traffic(2000, str(summary), str(src))[0] is None  # another workload
    src.write_text("kernel v2")
    assert bench.counters_traffic(1000, str(summary), str(src))[0] is None  # the kernel changed
    assert bench.counters_traffic(1000, str(tmp_path / "missing.json"), str(src)) == (None, None)


def test_counter_summaries_are_keyed_on_the_bench_lines_bytes():
    """Each committed counter summary carries the algorithmic bytes per launch that the
    committed bench line of its workload prints for the kernel the counters cover (the
    edge pass for the single-vector forms, the whole group loop for the batched one), so
    the bench's traffic lookup finds it."""
    prof = os.path.join(ROOT, "profiles")

    def load(name):
        with open(os.path.join(prof, name)) as f:
            return json.load(f)

    pairs = [("k_pb_rmat27_counters.json", load("bench_rmat27_pb.json")["roofline"]["edge_pass"]),
             ("k_pull_rmat27_counters.json", load("bench_rmat27_pull.json")["roofline"]["edge_pass"]),
             ("k_batch_pull_rmat24_b64_counters.json", load("bench_rmat24_b64_batched.json")["roofline"])]
    for summary, line in pairs:
        assert load(summary)["bytes_alg_per_launch"] == line["bytes_alg_per_launch"], summary


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


def test_batch_workspace_bound_covers_the_library():
    """The serving loop admits jobs on a closed-form bound of the batched workspace: it is
    never below the library's exact size, over random graphs and batches (one group and
    many, both versions, default and given segment lengths)."""
    import ctypes

    import paper_2402_04403_amd as gee
    from paper_2402_04403_amd.serve import batch_workspace_bound

    lib = gee.load()
    fake = ctypes.c_void_p(256)
    rng = np.random.default_rng(12)
    worst = 0.0
    for trial in range(300):
        n = int(rng.integers(1, 1 << 26))
        nnz = int(rng.integers(0, 1 << 30))
        n_hot = int(rng.integers(0, min(n, 1 << 22) + 1))
        B = int(rng.integers(1, 9)) if trial % 3 else int(rng.integers(1, 200))
        Ks = [int(k) for k in rng.integers(1, 300 if trial % 2 else 4097, B)]
        laps = [bool(x) for x in rng.integers(0, 2, B)]
        seg = 0 if trial % 4 else int(rng.integers(1, 1024)) * 64
        csr = gee.Csr(n, nnz, fake, fake, None, n_hot, fake if n_hot else None)
        zoff = list(np.cumsum([0] + Ks[:-1]))
        st, keep = gee._batch_struct(None, Ks, laps, zoff, int(sum(Ks)), None)
        o = gee.EmbedOpts(seg, 0, None, None, 0)
        exact = int(lib.gee_embed_batch_workspace(ctypes.byref(csr), ctypes.byref(st), ctypes.byref(o)))
        if exact == 0:
            continue  # a shape the library refuses (too many segments, say)
        bound = batch_workspace_bound(n, nnz, n_hot, Ks, laps, seg)
        assert bound >= exact, (trial, n, nnz, n_hot, B, seg)
        if B <= 8 and max(Ks) < 300:
            worst = max(worst, bound / exact)
    assert worst < 3.0  # and not wildly above it for the serving loop's one-group jobs
