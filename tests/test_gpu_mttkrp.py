"""GPU parity of spMTTKRP with remapping against the FP64 oracle.

Every call goes through the C ABI.  Tolerances: every output element within
1e-5 of the magnitude sum M_abs of its terms (``parity.check_elementwise``),
and the per-mode relative Frobenius error <= 1e-5 (FP32 storage and
accumulation against FP64); integer results (remap ids, the remapped streams)
bit-exact.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2405_08470_amd import synth
from parity import check_elementwise, mttkrp_abs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)
S = pytest.importorskip("paper_2405_08470_amd.spmttkrp")

TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _dev(factors):
    return [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in factors]


def _run_all_modes(t, dims, fdev, R, fuse=True):
    outs = []
    for d in range(len(dims)):
        out = torch.empty((dims[d], R), dtype=torch.float32, device="cuda")
        S.mttkrp(t, d, fdev, out, flags=S.FUSE_REMAP_NEXT if fuse else 0)
        outs.append(out)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


CASES = [
    # name, dims, nnz, dist, zipf_s, R, kappa, split_cap
    ("uniform3_r16", (1000, 800, 600), 100_000, "uniform", 1.1, 16, 0, None),
    ("zipf3_r32", (3000, 2500, 60_000), 400_000, "zipf", 1.1, 32, 0, None),
    ("zipf5_r32", (1000, 1000, 500, 200, 50), 300_000, "zipf", 1.2, 32, 97, None),
    ("zipf4_r64", (5000, 5000, 2000, 100), 250_000, "zipf", 1.1, 64, 0, None),
    ("zipf3_r8", (400, 300, 200), 50_000, "zipf", 1.3, 8, 13, None),
    ("zipf3_r128", (400, 300, 200), 30_000, "zipf", 1.1, 128, 0, None),
    ("zipf2_nosplit", (500, 400), 40_000, "zipf", 1.5, 16, 31, 0),
    ("zipf8_r16", (9, 8, 7, 6, 5, 4, 3, 2), 20_000, "zipf", 1.1, 16, 5, None),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_mttkrp_all_modes_with_remap(case):
    name, dims, nnz, dist, s, R, kappa, cap = case
    _say("case", name)
    idx, val = synth.random_coo(dims, nnz, seed=17, dist=dist, zipf_s=s)
    Y = synth.random_factors(dims, R, seed=18)
    t = S.tensor_load_coo(dims, idx, val, kappa=kappa, split_cap=cap)
    plan = oracle.plan(dims, idx, S.tensor_info(t)["kappa"], split_cap=cap)
    N = len(dims)
    for d in range(N):
        assert np.array_equal(S.tensor_get_remap(t, d), plan["b"][d]), f"remap ids of mode {d}"
    gi, gv, cm = S.tensor_get_records(t)
    assert cm == 0
    o0 = plan["order"][0]
    assert np.array_equal(gi, idx[:, o0]) and np.array_equal(gv, val[o0])
    fdev = _dev(Y)
    outs = []
    for d in range(N):
        out = torch.full((dims[d], R), float("nan"), dtype=torch.float32, device="cuda")
        S.mttkrp(t, d, fdev, out, flags=S.FUSE_REMAP_NEXT)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        # the stream is now in mode d+1's order, bit for bit
        gi, gv, cm = S.tensor_get_records(t)
        nxt = (d + 1) % N
        assert cm == nxt
        o = plan["order"][nxt]
        assert np.array_equal(gi, idx[:, o]) and np.array_equal(gv, val[o]), f"stream after mode {d}"
    for d in range(N):
        ref = oracle.mttkrp(dims, idx, val, Y, d)
        err = _rel(outs[d], ref)
        ratio = check_elementwise(outs[d], ref, mttkrp_abs(dims, idx, val, Y, d), label=f"mode {d}")
        _say(f"  mode {d}: rel err {err:.2e}, max element error / M_abs {ratio:.2e}")
        assert err <= TOL, (d, err)
    t.free()


def test_remap_cycle_identity_and_determinism():
    dims = (2000, 1500, 40_000)
    idx, val = synth.random_coo(dims, 300_000, seed=5, dist="zipf", zipf_s=1.1)
    Y = synth.random_factors(dims, 32, seed=6)
    t = S.tensor_load_coo(dims, idx, val)
    g0 = S.tensor_get_records(t)
    fdev = _dev(Y)
    a = _run_all_modes(t, dims, fdev, 32)
    g1 = S.tensor_get_records(t)
    assert g1[2] == 0
    assert np.array_equal(g0[0], g1[0]) and np.array_equal(g0[1].view(np.uint32), g1[1].view(np.uint32))
    b = _run_all_modes(t, dims, fdev, 32)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    t.free()


def test_ec_only_one_copy_per_mode_and_state_errors():
    dims = (700, 600, 500, 40)
    idx, val = synth.random_coo(dims, 120_000, seed=8, dist="zipf", zipf_s=1.2)
    Y = synth.random_factors(dims, 16, seed=9)
    fdev = _dev(Y)
    refs = [oracle.mttkrp(dims, idx, val, Y, d) for d in range(4)]
    absr = [mttkrp_abs(dims, idx, val, Y, d) for d in range(4)]
    # one copy per mode: any order of modes, no remapping
    tc = S.tensor_load_coo(dims, idx, val, copies=1)
    for d in (2, 0, 3, 1, 2):
        out = torch.empty((dims[d], 16), dtype=torch.float32, device="cuda")
        S.mttkrp(tc, d, fdev, out)
        assert _rel(out.cpu().numpy(), refs[d]) <= TOL
        check_elementwise(out.cpu().numpy(), refs[d], absr[d], label=f"one copy, mode {d}")
    tc.free()
    # one copy + remap target: wrong order is an error unless auto-remap
    t = S.tensor_load_coo(dims, idx, val)
    out = torch.empty((dims[2], 16), dtype=torch.float32, device="cuda")
    with pytest.raises(S.SptError) as ei:
        S.mttkrp(t, 2, fdev, out)
    assert ei.value.name == "SPT_ERR_STATE"
    S.mttkrp(t, 2, fdev, out, flags=S.AUTO_REMAP)
    assert S.tensor_info(t)["cur_mode"] == 2
    assert _rel(out.cpu().numpy(), refs[2]) <= TOL
    check_elementwise(out.cpu().numpy(), refs[2], absr[2], label="auto remap, mode 2")
    # EC without remap leaves the order alone
    S.mttkrp(t, 2, fdev, out)
    assert S.tensor_info(t)["cur_mode"] == 2
    S.remap_for_mode(t, 1)
    plan = oracle.plan(dims, idx, S.tensor_info(t)["kappa"])
    gi, gv, cm = S.tensor_get_records(t)
    assert cm == 1 and np.array_equal(gi, idx[:, plan["order"][1]])
    S.remap_for_mode(t, 0)
    out0 = torch.empty((dims[0], 16), dtype=torch.float32, device="cuda")
    S.mttkrp(t, 0, fdev, out0, flags=S.FUSE_REMAP_NEXT)
    assert _rel(out0.cpu().numpy(), refs[0]) <= TOL
    check_elementwise(out0.cpu().numpy(), refs[0], absr[0], label="after two hops, mode 0")
    t.free()


@pytest.mark.parametrize("kind", ["empty", "one_nonzero", "kappa_above_nnz", "unit_modes",
                                  "single_hot_row", "ragged_small"])
def test_edge_cases(kind):
    _say("edge", kind)
    R = 16
    if kind == "empty":
        dims, idx, val = (5, 4, 3), np.zeros((3, 0), np.int32), np.zeros(0, np.float32)
        kw = {}
    elif kind == "one_nonzero":
        dims, idx, val = (5, 4, 3), np.array([[4], [0], [2]], np.int32), np.array([1.5], np.float32)
        kw = {}
    elif kind == "kappa_above_nnz":
        dims = (50, 40, 30)
        idx, val = synth.random_coo(dims, 37, seed=1)
        kw = {"kappa": 200}
    elif kind == "unit_modes":
        dims = (1, 300, 1, 7)
        idx, val = synth.random_coo(dims, 5000, seed=2)
        kw = {"kappa": 16}
    elif kind == "single_hot_row":
        dims = (64, 50, 40)
        idx, val = synth.random_coo(dims, 20_000, seed=3)
        idx[0, :] = 7
        kw = {"kappa": 24}
    else:
        dims = (333, 222, 111)
        idx, val = synth.random_coo(dims, 12_345, seed=4, dist="zipf", zipf_s=1.4)
        kw = {"kappa": 77}
    Y = synth.random_factors(dims, R, seed=5)
    t = S.tensor_load_coo(dims, idx, val, **kw)
    outs = _run_all_modes(t, dims, _dev(Y), R)
    for d in range(len(dims)):
        ref = oracle.mttkrp(dims, idx, val, Y, d)
        if kind == "empty":
            assert np.all(outs[d] == 0)
        else:
            assert _rel(outs[d], ref) <= TOL, (kind, d)
            check_elementwise(outs[d], ref, mttkrp_abs(dims, idx, val, Y, d), label=f"{kind} mode {d}")
    assert S.tensor_info(t)["cur_mode"] == 0
    t.free()


def test_load_errors():
    dims = (5, 4, 3)
    idx = np.array([[0, 5], [0, 1], [0, 1]], np.int32)
    with pytest.raises(S.SptError) as ei:
        S.tensor_load_coo(dims, idx, np.ones(2, np.float32))
    assert ei.value.name == "SPT_ERR_OUT_OF_RANGE"
    idx[0, 1] = 1
    t = S.tensor_load_coo(dims, idx, np.ones(2, np.float32))
    Y = _dev(synth.random_factors(dims, 24, seed=1))
    with pytest.raises(S.SptError) as ei:
        S.mttkrp(t, 0, Y, torch.empty((5, 24), device="cuda"))
    assert ei.value.name == "SPT_ERR_UNSUPPORTED"
    Y = _dev(synth.random_factors(dims, 16, seed=1))
    lam = torch.empty(16, dtype=torch.float64, device="cuda")
    S.remap_for_mode(t, 1)
    with pytest.raises(S.SptError) as ei:
        S.cp_als_iter(t, Y, lam)
    assert ei.value.name == "SPT_ERR_STATE"
    t.free()
