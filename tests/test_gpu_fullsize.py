"""Full-size parity: the benchmark workloads at their stated sizes, in the
launch configuration the benchmark times (default kappa, fused remap), through
the C ABI.

The oracle cannot run the whole MTTKRP of 1e8 nonzeros in test time, so it
computes sampled output rows one by one (``oracle.mttkrp_rows``) on a subset
of rank columns.  Column r of M_d depends only on column r of the factors (a
pinned oracle property), so the columns of the GPU result are compared with
the oracle on the factors' same columns.  Rows: the hottest rows (split across
many partitions), a high-degree row, random non-empty rows, an empty row, the
first and the last row.  Integer work is checked bit-exactly at full size: the
stream after loading and after each fused remap holds record e at position
b_d(e), and b_d is a permutation.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2405_08470_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

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


def _sample_rows(col, I, seed):
    deg = np.bincount(col, minlength=I)
    order = np.argsort(-deg, kind="stable")
    rng = np.random.default_rng(seed)
    nonempty = np.flatnonzero(deg)
    rows = [int(order[0]), int(order[1]), int(order[len(nonempty) // 100])]
    rows += [int(r) for r in rng.choice(nonempty, 3, replace=False)]
    empty = np.flatnonzero(deg == 0)
    if empty.size:
        rows.append(int(empty[0]))
    rows += [0, I - 1]
    return rows


def _check_stream(t, idx, val, mode):
    """Record e sits at position b_mode(e) of the current stream, bit-exact."""
    ridx, rval, cur = S.tensor_get_records(t)
    assert cur == mode
    b = S.tensor_get_remap(t, mode)
    nnz = idx.shape[1]
    seen = np.zeros(nnz, dtype=bool)
    seen[b] = True
    assert seen.all(), "remap ids are not a permutation"
    assert np.array_equal(ridx[:, b], idx)
    assert np.array_equal(rval[b].view(np.uint32), val.view(np.uint32))


def _all_modes(t, dims, fdev, R, check=None):
    outs = []
    for d in range(len(dims)):
        out = torch.empty((dims[d], R), dtype=torch.float32, device="cuda")
        S.mttkrp(t, d, fdev, out, flags=S.FUSE_REMAP_NEXT)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        if check is not None:
            check((d + 1) % len(dims))
    return outs


def _compare(dims, idx, val, Y, outs, cols, label):
    for d in range(len(dims)):
        rows = _sample_rows(idx[d], dims[d], seed=d)
        ref = oracle.mttkrp_rows(dims, idx, val, [y[:, cols] for y in Y], d, rows)
        got = outs[d][rows][:, cols]
        e = _rel(got, ref)
        _say(f"  {label} mode {d}: rows {rows[:3]}... rel {e:.2e}")
        assert e <= TOL


@pytest.mark.parametrize("cfg", [2, 3, 4])
def test_full_size_all_modes_with_remap(cfg):
    spec = synth.CONFIGS[cfg]
    _say(f"case full-size config {cfg}: {spec.name} dims {spec.dims} nnz {spec.nnz} R {spec.rank}")
    dims, idx, val = synth.make_coo(spec)
    Y = synth.make_factors(spec)
    R = spec.rank
    t = S.tensor_load_coo(dims, idx, val)
    info = S.tensor_info(t)
    kappa, nnz = info["kappa"], info["nnz"]
    cap = -(-nnz // kappa)
    _say(f"  kappa {kappa}, max load {info['max_load']}, split rows {info['split_rows']}")
    # least-loaded assignment of pieces no larger than cap: makespan <= mean + cap
    assert all(m <= -(-nnz // kappa) + cap for m in info["max_load"])
    _check_stream(t, idx, val, 0)
    fdev = [torch.from_numpy(y).cuda() for y in Y]
    outs = _all_modes(t, dims, fdev, R, check=lambda m: _check_stream(t, idx, val, m))
    cols = list(range(0, R, R // 8))
    _compare(dims, idx, val, Y, outs, cols, "fp32")
    if cfg == 4:
        # BF16 factor storage and gathers, FP32 accumulation
        Yb = [oracle.bf16_round(y) for y in Y]
        fb = [f.to(torch.bfloat16) for f in fdev]
        outb = _all_modes(t, dims, fb, R)
        _compare(dims, idx, val, Yb, outb, cols, "bf16 kernel")
        for d in range(len(dims)):
            rows = _sample_rows(idx[d], dims[d], seed=d)
            ref = oracle.mttkrp_rows(dims, idx, val, [y[:, cols] for y in Y], d, rows)
            e = _rel(outb[d][rows][:, cols], ref)
            _say(f"  bf16 storage mode {d}: rel {e:.2e}")
            assert e <= 1.5e-2
    assert S.tensor_info(t)["cur_mode"] == 0
    t.free()


def test_full_size_cp_als_sweep_last_mode_one_step():
    """After one CP-ALS sweep at 8e7 nonzeros, the last mode's factor must be
    the FP64 least-squares update from the other (final) factors: on sampled
    rows, Y_last[i] * lambda = M_last[i] V^-1 with V the Hadamard product of
    the other factors' Grams; and every column of Y_last has unit norm."""
    spec = synth.CONFIGS[2]
    _say(f"case full-size CP-ALS sweep: {spec.name}")
    dims, idx, val = synth.make_coo(spec)
    Y0 = synth.make_factors(spec)
    R = spec.rank
    t = S.tensor_load_coo(dims, idx, val)
    f = [torch.from_numpy(y).cuda() for y in Y0]
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    fit = S.cp_als_iter(t, f, lam)
    _say(f"  fit after one sweep {fit:.6f}")
    Y = [x.cpu().numpy() for x in f]
    lam = lam.cpu().numpy()
    N = len(dims)
    d = N - 1
    V = np.ones((R, R))
    for w in range(N - 1):
        yw = Y[w].astype(np.float64)
        V *= yw.T @ yw
    rows = _sample_rows(idx[d], dims[d], seed=7)
    M = oracle.mttkrp_rows(dims, idx, val, Y, d, rows)
    ref = np.linalg.solve(V, M.T).T          # M V^-1 (V symmetric)
    got = Y[d][rows].astype(np.float64) * lam
    e = _rel(got, ref)
    _say(f"  last-mode one-step rel {e:.2e}")
    assert e <= TOL
    norms = np.linalg.norm(Y[d].astype(np.float64), axis=0)
    assert np.allclose(norms[lam > 0], 1.0, atol=1e-5)
    assert 0.0 < fit < 1.0
    t.free()
