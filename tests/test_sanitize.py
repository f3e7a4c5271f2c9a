"""The C oracle and the seeded generators under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only, host code).

``tests/sanitize/sanitize_main.c`` is compiled together with ``oracle/gee_oracle.c`` and
``gen/gee_gen.c`` with ``-fsanitize=address,undefined`` and run: every array it hands the
two libraries comes from the sanitizer's allocator, so an access outside any of them, or
undefined behaviour, ends the run with a report. Each result it prints (return code and
a hash of the output bytes) must equal the same call made here through the
uninstrumented libraries that the other tests pin, so the sanitized run covers the
code the pins cover: both versions, weighted and unit records, sampled rows, and the
error paths.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import gen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MAIN = os.path.join(ROOT, "tests", "sanitize", "sanitize_main.c")


def fnv(a) -> str:
    h = 1469598103934665603
    for c in np.ascontiguousarray(a).view(np.uint8).tobytes():
        h ^= c
        h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return f"{h:016x}"


def _call(fn, *args):
    try:
        return 0, fn(*args)
    except oracle.OracleError as e:
        return e.code, None


def _embed_all(want, tag, n, src, dst, w, Y, K):
    rc, cnt = _call(oracle.counts, Y, K)
    want[f"{tag}.counts"] = (rc, fnv(cnt))
    rc, inv = _call(oracle.weights, cnt, K)
    want[f"{tag}.weights"] = (rc, fnv(inv))
    rc, deg = _call(oracle.degrees, n, src, dst, w)
    want[f"{tag}.degrees"] = (rc, fnv(deg))
    rows = np.array([(j * 7919) % n for j in range(min(n, 7))], np.int64)
    for lap in (0, 1):
        rc, Z = _call(oracle.embed, n, src, dst, w, Y, K, bool(lap))
        want[f"{tag}.embed.lap{lap}"] = (rc, fnv(Z))
        rc, Zr = _call(oracle.embed_rows, n, src, dst, w, Y, K, bool(lap), rows)
        want[f"{tag}.rows.lap{lap}"] = (rc, fnv(Zr))


def expected() -> dict:
    want = {}
    empty = fnv(np.zeros(0, np.uint8))
    lib = gen._load()
    p32 = lambda a: a.ctypes.data_as(gen.I32P)
    f32 = lambda a: a.ctypes.data_as(gen.F32P)
    # Erdos-Renyi
    n, s, K = 1000, 5000, 7
    g = gen.er(n, s, 2, weighted=True)
    src, dst, w = g.src.copy(), g.dst.copy(), g.w.copy()
    want["gen.er.src"], want["gen.er.dst"], want["gen.er.w"] = (0, fnv(src)), (0, fnv(dst)), (0, fnv(w))
    Y = np.empty(n, np.int32)
    lib.gen_labels_uniform(n, K, 3, p32(Y))
    want["gen.labels"] = (lib.gen_unlabel_exact(n, 50, 4, p32(Y)), fnv(Y))
    _embed_all(want, "er", n, src, dst, w, Y, K)
    _embed_all(want, "er_unit", n, src, dst, None, Y, K)
    lib.gen_grid_weights(s, 5, f32(w))
    want["gen.grid"] = (0, fnv(w))
    lib.gen_shuffle_records(s, 6, p32(src), p32(dst), f32(w))
    want["gen.shuffle"] = (0, fnv(src))
    _embed_all(want, "er_shuffled", n, src, dst, w, Y, K)
    Y2 = Y.copy()
    Y2[3] = K + 1
    want["err.label"] = (_call(oracle.counts, Y2, K)[0], empty)
    d2 = dst.copy()
    d2[11] = n
    want["err.vertex"] = (_call(oracle.embed, n, src, d2, w, Y, K, False)[0], empty)
    w2 = w.copy()
    w2[5] = -1.0
    d3 = dst.copy()
    d3[11] = 0
    want["err.negw"] = (_call(oracle.embed, n, src, d3, w2, Y, K, True)[0], empty)
    want["err.row"] = (_call(oracle.embed_rows, n, src, d3, None, Y, K, False, np.array([n], np.int64))[0], empty)
    want["err.n"] = (oracle.EINVAL, empty)
    # R-MAT scale 10
    scale = 10
    n, K = 1 << scale, 5
    s = 8 * n
    g = gen.rmat(scale, s, 7)
    want["gen.rmat.src"], want["gen.rmat.dst"] = (0, fnv(g.src)), (0, fnv(g.dst))
    Y = np.empty(n, np.int32)
    lib.gen_labels_uniform(n, K, 8, p32(Y))
    lib.gen_unlabel_bernoulli(n, 0.3, 9, p32(Y))
    want["gen.bern"] = (0, fnv(Y))
    _embed_all(want, "rmat", n, g.src, g.dst, None, Y, K)
    # SBM
    n, cap, K = 300, 20000, 3
    src, dst = np.zeros(cap, np.int32), np.zeros(cap, np.int32)
    s = lib.gen_sbm(n, 3, 0.2, 0.02, 10, cap, p32(src), p32(dst))
    want["gen.sbm"] = (s, fnv(src[:s]))
    want["gen.sbm.cap"] = (-1, empty)
    Y = np.array([1 + (v * 3) // n for v in range(n)], np.int32)
    _embed_all(want, "sbm", n, src[:s].copy(), dst[:s].copy(), None, Y, K)
    src2, dst2 = np.zeros(4000, np.int32), np.zeros(4000, np.int32)
    lib.gen_sbm_records(n, 3, 0.8, 4000, 11, p32(src2), p32(dst2))
    want["gen.sbmr.src"], want["gen.sbmr.dst"] = (0, fnv(src2)), (0, fnv(dst2))
    return want


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_and_generators_clean_under_asan_ubsan(tmp_path):
    exe = tmp_path / "sanitized"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-fast-math",
                           "-ffp-contract=off", "-o", str(exe), MAIN, os.path.join(ROOT, "oracle", "gee_oracle.c"),
                           os.path.join(ROOT, "gen", "gee_gen.c"), "-lm"])
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    got = {}
    for line in r.stdout.splitlines():
        name, rc, h = line.split()
        got[name] = (int(rc), h)
    want = expected()
    assert set(got) == set(want)
    for name in sorted(want):
        assert got[name] == want[name], name
