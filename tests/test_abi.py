"""The C-ABI library loads, exports every declared symbol, and its host-only
planner (no device) reproduces the oracle's partitions and remap ids."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2405_08470_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmttkrp.h")

S = pytest.importorskip("paper_2405_08470_amd.spmttkrp")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(spt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_exported_symbols():
    lib = S.lib()
    decl = _declared()
    assert set(decl) == set(S.EXPORTS)
    for name in decl:
        assert hasattr(lib, name), name
    assert lib.spt_status_str(6) == b"SPT_ERR_NOT_SPD"


@pytest.mark.parametrize("dims,nnz,kappa,cap", [((7, 6, 5), 80, 3, None), ((5, 4, 3, 3), 90, 4, 0),
                                                ((4, 3, 3, 2, 2), 60, 5, None),
                                                ((30, 20), 200, 6, 5),
                                                ((50, 40, 30), 3000, 7, None),
                                                ((9, 8, 7, 6, 5, 4, 3, 2), 500, 4, 10)])
def test_planner_bit_exact_against_oracle(dims, nnz, kappa, cap):
    idx, _ = synth.random_coo(dims, nnz, seed=9, dist="zipf", zipf_s=1.3)
    p = oracle.plan(dims, idx, kappa, split_cap=cap)
    q = S.plan_coo(dims, idx, kappa=kappa, split_cap=cap)
    assert q["kappa"] == kappa
    for d in range(len(dims)):
        assert np.array_equal(p["part"][d], q["part"][d])
        assert np.array_equal(p["b"][d], q["remap"][d])
        assert np.array_equal(p["ptr"][d], q["ptr"][d])


def test_planner_bit_exact_on_skewed_workloads():
    for name, nnz, kappa in (("zipf3_8e7", 300_000, 96), ("zipf5_5e7", 200_000, 128),
                             ("uniform3_1e5", 100_000, 50)):
        spec = synth.scaled(synth.WORKLOADS[name], nnz)
        dims, idx, _ = synth.make_coo(spec)
        p = oracle.plan(dims, idx, kappa)
        q = S.plan_coo(dims, idx, kappa=kappa)
        for d in range(len(dims)):
            assert np.array_equal(p["b"][d], q["remap"][d]), (name, d)
            assert np.array_equal(p["part"][d], q["part"][d]), (name, d)


def test_planner_default_kappa_and_empty_tensor():
    idx = np.zeros((3, 0), dtype=np.int32)
    q = S.plan_coo((4, 3, 2), idx)
    assert q["kappa"] == 1 and q["ptr"].tolist() == [[0, 0]] * 3


@pytest.mark.parametrize("dims,idx,name", [
    ((4,), [[0, 1]], "SPT_ERR_INVALID_ARG"),                       # one mode
    ((4, 3), [[0, 4], [0, 1]], "SPT_ERR_OUT_OF_RANGE"),            # index beyond mode size
    ((4, 3), [[0, -1], [0, 1]], "SPT_ERR_OUT_OF_RANGE"),           # negative index
    ((4, 0), [[0, 1], [0, 0]], "SPT_ERR_OUT_OF_RANGE"),            # empty mode
    ((4, 2 ** 31), [[0, 1], [0, 0]], "SPT_ERR_OUT_OF_RANGE"),      # mode size beyond int32
    (tuple([2] * 9), [[0]] * 9, "SPT_ERR_INVALID_ARG"),            # nine modes
])
def test_planner_rejects_bad_input(dims, idx, name):
    with pytest.raises(S.SptError) as ei:
        S.plan_coo(dims, np.array(idx, dtype=np.int32))
    assert ei.value.name == name
    assert ei.value.message
