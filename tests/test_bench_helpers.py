"""Host logic of bench.py: the bytes models behind roofline.achieved and the
pass fractions, the lookup of the committed counter summaries behind
roofline.traffic, and the row sampler of the accuracy report."""
import glob
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
bench = pytest.importorskip("bench")


def test_bytes_model_of_the_80m_workload():
    dims, nnz, R = (100_000, 80_000, 2_000_000), 80_000_000, 32
    # EC: records in, each input factor once, the output once
    ec = [bench.ec_bytes(dims, nnz, R, 16, d) for d in range(3)]
    assert ec[0] == nnz * 16 + (80_000 + 2_000_000) * R * 4 + 100_000 * R * 4 == 1_559_040_000
    assert ec[0] == ec[1] == ec[2]
    # BF16 factors: the gathered factors at 2 bytes, the FP32 output unchanged
    assert bench.ec_bytes(dims, nnz, R, 16, 0, fac_bytes=2) == ec[0] - (80_000 + 2_000_000) * R * 2
    # DR: each record and its next position in, the record out
    assert bench.remap_bytes(nnz, 16) == nnz * 36 == 2_880_000_000
    # the paper's records: 4(2N+1) = 28 bytes read and written
    can = sum(bench.canonical_bytes(dims, nnz, R, d) for d in range(3))
    assert can == 3 * nnz * 56 + 3 * sum(dims) * R * 4 == 14_277_120_000


def test_bytes_model_of_the_4_mode_workload():
    dims, nnz, R = (50_000, 50_000, 20_000, 1_000), 100_000_000, 64
    can = sum(bench.canonical_bytes(dims, nnz, R, d) for d in range(4))
    # 36-byte records; the half-of-peak target is 7.23 ms per pass
    assert can == 4 * nnz * 72 + 4 * sum(dims) * R * 4
    assert abs(can / 4e12 * 1e3 - 7.23) < 0.01


def test_traffic_summaries_are_used_only_for_their_kernel_sources_and_kappa():
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.txt")))
    checked = 0
    for path in files:
        fam, rest = os.path.basename(path).split("_kernel_", 1)
        fam += "_kernel"
        workload = rest[: -len("_traffic.txt")]
        vals = dict(l.split("=", 1) for l in open(path).read().splitlines()
                    if "=" in l and not l.startswith("#"))
        kernel, kappa = vals["kernel"], int(vals["kappa"])
        if vals["kernel_source_sha256_16"] != bench.kernel_source_hash(bench.SOURCES[fam]):
            assert bench.measured_traffic(kernel, workload, kappa) is None
            continue
        got = bench.measured_traffic(kernel, workload, kappa)
        assert got == float(vals["bytes_per_launch"])
        # the summary's traffic is at least what the kernel must read and write
        assert got >= 0.9 * float(vals["algorithmic_bytes_per_launch"])
        assert bench.measured_traffic(kernel, workload, kappa * 2) is None
        assert bench.measured_traffic(kernel, "no_such_workload", kappa) is None
        checked += 1
    assert bench.measured_traffic("no_such_kernel<1>", "zipf4_1e8", 8192) is None
    if not checked:
        pytest.skip("no counter summary matches the kernel sources of this tree")


def test_sampled_rows_span_the_degree_spectrum():
    col = np.array([5] * 100 + [3] * 10 + [7, 7, 1], dtype=np.int32)
    rows = bench.sample_rows(col, 10, 8, seed=0)
    assert rows == sorted(set(rows))
    assert 5 in rows and 3 in rows            # the hottest rows
    assert any(r in (0, 2, 4, 6, 8, 9) for r in rows)  # an empty row
    assert all(0 <= r < 10 for r in rows)
