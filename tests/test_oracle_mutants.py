"""The oracle's pins must catch plausible mistakes (CPU only).

Each mutant is a copy of the oracle's C source with one deliberate slip, compiled into
a temporary directory. The pin battery of ``test_oracle`` runs against it, and at least
one pin must fail. Every mutant stays in bounds, so a wrong result, never a crash, is
what the pins see.
"""
import ctypes
import os
import subprocess

import pytest

import oracle
import test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "gee_oracle.c")

MUTANTS = {
    "update uses W of the wrong endpoint":
        ("Z[u * K + (Y[v] - 1)] += inv[Y[v]] * x;", "Z[u * K + (Y[v] - 1)] += inv[Y[u]] * x;"),
    "second update dropped":
        ("if (Y[u] > 0) Z[v * K + (Y[u] - 1)] += inv[Y[u]] * x; /*", "if (0) Z[v * K + (Y[u] - 1)] += inv[Y[u]] * x; /*"),
    "update lands in the wrong row":
        ("Z[u * K + (Y[v] - 1)] += inv[Y[v]] * x;", "Z[v * K + (Y[v] - 1)] += inv[Y[v]] * x;"),
    "class taken from the row vertex":
        ("Z[u * K + (Y[v] - 1)] += inv[Y[v]] * x;", "if (Y[u] > 0) Z[u * K + (Y[u] - 1)] += inv[Y[v]] * x;"),
    "column off by one (wraps)":
        ("Z[u * K + (Y[v] - 1)] += inv[Y[v]] * x;", "Z[u * K + (Y[v] % K)] += inv[Y[v]] * x;"),
    "class 1 treated as unknown":
        ("if (Y[v] > 0) Z[u * K", "if (Y[v] > 1) Z[u * K"),
    "weights divide by n":
        ("inv[k] = counts[k] > 0 ? 1.0 / (double)counts[k] : 0.0;",
         "inv[k] = counts[k] > 0 ? 1.0 / (double)(counts[0] + counts[k]) : 0.0;"),
    "Laplacian squares one endpoint":
        ("if (laplacian) x = x * r[u] * r[v];\n        if (Y[v] > 0) Z[u * K",
         "if (laplacian) x = x * r[u] * r[u];\n        if (Y[v] > 0) Z[u * K"),
    "self-loop counted once in the degree":
        ("deg[dst[i]] += x;", "if (dst[i] != src[i]) deg[dst[i]] += x;"),
    "degree ignores weights":
        ("double x = w ? (double)w[i] : 1.0;\n        deg[src[i]]", "double x = 1.0;\n        deg[src[i]]"),
    "Laplacian uses 1/d instead of d^-1/2":
        ("d[u] = d[u] > 0.0 ? 1.0 / sqrt(d[u]) : 0.0;", "d[u] = d[u] > 0.0 ? 1.0 / d[u] : 0.0;"),
    "weight ignored in the edge pass":
        ("double x = w ? (double)w[i] : 1.0;\n        if (laplacian) x = x * r[u] * r[v];\n        if (Y[v] > 0) Z[u * K",
         "double x = 1.0;\n        if (laplacian) x = x * r[u] * r[v];\n        if (Y[v] > 0) Z[u * K"),
}

BATTERY = [
    pins.test_exact_bruteforce_all_graphs_on_4_vertices,
    lambda: [pins.test_hand_worked_graphs(c, lap) for c in pins._golden_cases() for lap in (False, True)],
    lambda: pins.test_row_and_column_sums(3),
    pins.test_dense_definition_small,
    pins.test_single_class_gives_degree_over_n,
    pins.test_power_of_two_classes_are_exact,
    pins.test_big_star_hub_sum,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation anchor must match exactly once"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(text.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", str(so), str(mpath), "-lm"])
    saved = oracle._lib
    oracle._lib = oracle._bind(ctypes.CDLL(str(so)))
    caught = []
    try:
        for check in BATTERY:
            try:
                check()
            except (AssertionError, oracle.OracleError):
                caught.append(check)
    finally:
        oracle._lib = saved
    assert caught, f"no pin caught the mutant: {name}"
