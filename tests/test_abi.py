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


@pytest.mark.parametrize("field,value,msg", [
    ("dr", 2, "opts.dr must be 0 or 1"),
    ("dr", -1, "opts.dr must be 0 or 1"),
    ("prep", 2, "opts.prep must be 0 or 1"),
    ("copies", 3, "opts.copies must be 0 or 1"),
    ("layout", 5, "opts.layout must be 0..4"),
    ("layout", -1, "opts.layout must be 0..4"),
])
def test_options_are_validated_before_any_device_work(field, value, msg):
    import ctypes
    o = S._opts(0, None, 0)
    setattr(o, field, value)
    dims = np.array([4, 3, 2], dtype=np.int64)
    idx = np.zeros((3, 1), dtype=np.int32)
    k = ctypes.c_int32()
    st = S.lib().spt_plan_coo(3, dims.ctypes.data, 1, idx.ctypes.data, ctypes.byref(o), None, None, None,
                              ctypes.byref(k))
    assert S._STATUS[st] == "SPT_ERR_INVALID_ARG"
    assert S.lib().spt_last_error().decode() == msg


def test_options_reserved_words_must_be_zero_and_remap_forms_map():
    import ctypes
    o = S._opts(0, None, 0)
    o.reserved = 1
    dims = np.array([4, 3, 2], dtype=np.int64)
    idx = np.zeros((3, 1), dtype=np.int32)
    k = ctypes.c_int32()
    st = S.lib().spt_plan_coo(3, dims.ctypes.data, 1, idx.ctypes.data, ctypes.byref(o), None, None, None,
                              ctypes.byref(k))
    assert S._STATUS[st] == "SPT_ERR_INVALID_ARG"
    assert S._opts(0, None, 0, remap="staged").dr == 0
    assert S._opts(0, None, 0, remap="fused").dr == 1
    with pytest.raises(ValueError):
        S._opts(0, None, 0, remap="pull")
    assert [S._opts(0, None, 0, layout=k).layout for k in ("auto", "word32", "half16", "packed", "compact")] == [0, 1, 2, 3, 4]
    with pytest.raises(ValueError):
        S._opts(0, None, 0, layout="soa")


def test_struct_layouts_of_the_binding_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C sizes and field
    offsets (a struct that grew in the header and not in a mirror would be
    written past its end)."""
    import ctypes
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    mirrors = {"spt_info": S.spt_info, "spt_opts": S.spt_opts, "spt_timing": S.spt_timing}
    src = ["#include <stddef.h>", "#include <stdio.h>", "#include \"spmttkrp.h\"", "int main(void) {"]
    for name, cls in mirrors.items():
        src.append(f'    printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            src.append(f'    printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    src.append("    return 0;\n}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for name, cls in mirrors.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, f"{name}.{f[0]}"
