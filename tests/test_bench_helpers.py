"""Host logic of bench.py: the bytes model behind roofline.achieved and the
lookup of the committed counter summary behind roofline.traffic."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
bench = pytest.importorskip("bench")


def test_bytes_model_of_the_80m_workload():
    dims, nnz, R = (100_000, 80_000, 2_000_000), 80_000_000, 32
    # EC: records in, each input factor once, the output once
    ec = [bench.algorithmic_bytes(dims, nnz, R, 16, d, False) for d in range(3)]
    assert ec[0] == nnz * 16 + (80_000 + 2_000_000) * R * 4 + 100_000 * R * 4 == 1_559_040_000
    assert ec[0] == ec[1] == ec[2]
    # DR: each record and its next position in, the record out
    assert bench.remap_bytes(nnz, 16) == nnz * 36 == 2_880_000_000
    # the fused launch moves both but reads each record once
    fused = bench.algorithmic_bytes(dims, nnz, R, 16, 0, True)
    assert fused == ec[0] + bench.remap_bytes(nnz, 16) - nnz * 16 == 3_159_040_000


def test_traffic_summary_is_used_only_for_its_kernel_sources_and_kappa():
    fam = "remap_flat_kernel"
    fname, sources = bench.TRAFFIC[fam]
    vals = dict(l.split("=", 1) for l in open(os.path.join(ROOT, "profiles", fname)).read().splitlines()
                if "=" in l and not l.startswith("#"))
    kernel, kappa = vals["kernel"], int(vals["kappa"])
    if vals["kernel_source_sha256_16"] != bench.kernel_source_hash(sources):
        pytest.skip("kernel sources changed since the summary was taken")
    got = bench.measured_traffic(kernel, kappa)
    assert got == float(vals["bytes_per_launch"])
    # the summary's traffic is at least what the kernel must read and write
    assert got >= float(vals["algorithmic_bytes_per_launch"])
    assert bench.measured_traffic(kernel, kappa * 2) is None
    assert bench.measured_traffic("remap_flat_kernel<8,2048>", kappa) is None
    assert bench.measured_traffic("no_such_kernel<1>", kappa) is None
