"""The device planner (opts.prep = 1) against the host planner and the oracle.

Everything integer is bit-exact: the packed streams, the remap ids of every
mode (which also fixes the next-position arrays), kappa, the largest
partition and the split rows of every mode; ||X||^2 agrees to FP64 rounding
(the summation order differs).  On small tensors the remap ids are also
compared with the oracle's plan (Alg. 1 + the stream order) directly.  The
MTTKRP outputs of the two loads are bit-identical, since the kernels see the
same streams.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2405_08470_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)
S = pytest.importorskip("paper_2405_08470_amd.spmttkrp")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same_tensor(th, td, N, check_mttkrp=None):
    ih, idd = S.tensor_info(th), S.tensor_info(td)
    for k in ("kappa", "nnz", "record_bytes", "max_load", "split_rows", "dims"):
        assert ih[k] == idd[k], k
    assert abs(ih["norm_sq"] - idd["norm_sq"]) <= 1e-12 * max(1.0, abs(ih["norm_sq"]))
    for d in range(N):
        assert np.array_equal(S.tensor_get_remap(th, d), S.tensor_get_remap(td, d)), f"remap ids, mode {d}"
    rh, rd = S.tensor_get_records(th), S.tensor_get_records(td)
    assert np.array_equal(rh[0], rd[0]) and np.array_equal(rh[1].view(np.uint32), rd[1].view(np.uint32))
    return ih, idd


CASES = [
    # name, dims, nnz, dist, zipf_s, kappa, split_cap
    ("uniform3", (1000, 800, 600), 100_000, "uniform", 1.1, 0, None),
    ("zipf3", (3000, 2500, 60_000), 400_000, "zipf", 1.1, 0, None),
    ("zipf5_k97", (1000, 1000, 500, 200, 50), 300_000, "zipf", 1.2, 97, None),
    ("zipf4", (5000, 5000, 2000, 100), 250_000, "zipf", 1.1, 0, None),
    ("zipf2_nosplit", (500, 400), 40_000, "zipf", 1.5, 31, 0),
    ("zipf8", (9, 8, 7, 6, 5, 4, 3, 2), 20_000, "zipf", 1.1, 5, None),
    ("unit_modes", (1, 300, 1), 5_000, "uniform", 1.1, 7, None),
    ("kappa_gt_nnz", (50, 40, 30), 100, "uniform", 1.1, 1000, None),
    ("one_nonzero", (10, 10, 10), 1, "uniform", 1.1, 0, None),
]


@pytest.mark.parametrize("name,dims,nnz,dist,s,kappa,cap", CASES, ids=[c[0] for c in CASES])
def test_device_planner_equals_host_planner(name, dims, nnz, dist, s, kappa, cap):
    _say("case", name)
    idx, val = synth.random_coo(dims, nnz, seed=len(name), dist=dist, zipf_s=s)
    N = len(dims)
    th = S.tensor_load_coo(dims, idx, val, kappa=kappa, split_cap=cap)
    td = S.tensor_load_coo(dims, idx, val, kappa=kappa, split_cap=cap, prep="device")
    _same_tensor(th, td, N)
    if nnz <= 100_000:
        p = oracle.plan(dims, idx, S.tensor_info(td)["kappa"], split_cap=cap)
        for d in range(N):
            assert np.array_equal(S.tensor_get_remap(td, d), p["b"][d])
    R = 16
    Y = synth.random_factors(dims, R, seed=3)
    f = [torch.from_numpy(y).cuda() for y in Y]
    for d in range(N):
        oh = torch.empty((dims[d], R), dtype=torch.float32, device="cuda")
        od = torch.empty_like(oh)
        S.mttkrp(th, d, f, oh, flags=S.FUSE_REMAP_NEXT)
        S.mttkrp(td, d, f, od, flags=S.FUSE_REMAP_NEXT)
        assert torch.equal(oh, od)
    th.free()
    td.free()


def test_device_planner_one_copy_per_mode():
    dims = (3000, 2500, 6000)
    idx, val = synth.random_coo(dims, 200_000, seed=5, dist="zipf")
    th = S.tensor_load_coo(dims, idx, val, copies=1)
    td = S.tensor_load_coo(dims, idx, val, copies=1, prep="device")
    for d in range(3):
        S.remap_for_mode(th, d)
        S.remap_for_mode(td, d)
        rh, rd = S.tensor_get_records(th), S.tensor_get_records(td)
        assert rh[2] == rd[2] == d
        assert np.array_equal(rh[0], rd[0]) and np.array_equal(rh[1].view(np.uint32), rd[1].view(np.uint32))
    th.free()
    td.free()


def test_device_planner_empty_tensor_and_errors():
    dims = (5, 4, 3)
    t = S.tensor_load_coo(dims, np.zeros((3, 0), np.int32), np.zeros(0, np.float32), prep="device")
    info = S.tensor_info(t)
    assert info["nnz"] == 0 and info["norm_sq"] == 0.0
    out = torch.full((5, 8), 7.0, device="cuda")
    Y = [torch.ones((n, 8), device="cuda") for n in dims]
    S.mttkrp(t, 0, Y, out)
    assert torch.count_nonzero(out).item() == 0
    t.free()
    idx = np.array([[0, 1, 4], [0, 3, 2], [0, 2, 7]], dtype=np.int32)  # 7 is outside mode 2
    val = np.ones(3, np.float32)
    msgs = []
    for prep in ("host", "device"):
        with pytest.raises(S.SptError) as ei:
            S.tensor_load_coo(dims, idx, val, prep=prep)
        msgs.append(str(ei.value))
    assert "OUT_OF_RANGE" in msgs[0] and msgs[0] == msgs[1]


@pytest.mark.slow
def test_device_planner_full_size_3mode():
    spec = synth.WORKLOADS["zipf3_8e7"]
    _say(f"case device planner at full size: {spec.name}")
    dims, idx, val = synth.make_coo(spec)
    td = S.tensor_load_coo(dims, idx, val, prep="device")
    th = S.tensor_load_coo(dims, idx, val)
    ih, idd = _same_tensor(th, td, len(dims))
    _say(f"  prep seconds: host {ih['prep_seconds']:.2f}, device {idd['prep_seconds']:.2f}")
    th.free()
    td.free()
