"""The pins catch plausible mistakes in the oracle.

Each case compiles a copy of oracle.c with one planted mistake (a dropped
term, a wrong index, a wrong tie rule ...) into a temporary library, points
the oracle at it and checks that at least one pin fails.  Mistakes are only
ever planted here, on the CPU, in a throwaway copy.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTATIONS = {
    "drop_value": ("ell[r] = val[e];", "ell[r] = 1.0;"),
    "wrong_gather_mode": ("factors[w] + (int64_t)idx[(int64_t)w * nnz + e]",
                          "factors[w] + (int64_t)idx[(int64_t)((w + 1) % nmodes) * nnz + e] % dims[w]"),
    "wrong_output_row": ("double *o = out + (int64_t)idx[(int64_t)mode * nnz + e] * rank;",
                         "double *o = out + (int64_t)(idx[(int64_t)mode * nnz + e] % 2) * rank;"),
    "include_output_factor": ("if (w == mode)\n                continue;", ""),
    "ties_to_highest": ("if (loads[w] < loads[best])", "if (loads[w] <= loads[best])"),
    "most_filled": ("if (loads[w] < loads[best])", "if (loads[w] > loads[best])"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new, 1))
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-o", str(so), str(path)])
    return str(so)


def _pins_pass():
    """A compact subset of the pins; returns True when all of them hold."""
    import test_oracle as t
    checks = [
        lambda: t.test_mttkrp_equals_dense_unfolding_times_khatri_rao((7, 6, 5), 60),
        lambda: t.test_mttkrp_equals_dense_unfolding_times_khatri_rao((5, 4, 3, 3), 70),
        lambda: t.test_mttkrp_rank_one_closed_form(3),
        t.test_partition_worked_example,
        t.test_lpt_graham_tight_instance,
        lambda: [t.test_lpt_within_four_thirds_of_brute_force_optimum(s) for s in range(10)],
    ]
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError):
            return False
    return True


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTATIONS[name]
    so = _build(tmp_path, name, old, new)
    saved = oracle._lib
    try:
        oracle._lib = None
        monkeypatch.setattr(oracle, "_SO", so)
        assert not _pins_pass(), f"mutation {name} slipped through the pins"
    finally:
        oracle._lib = saved


def test_unmutated_oracle_passes_the_same_subset():
    oracle._lib = None
    assert _pins_pass()
