"""Full-size parity: the benchmark workloads at their stated sizes, in the
launch configuration the benchmark times (default kappa, remap pass after the
elementwise kernel), through the C ABI.

The oracle cannot run the whole MTTKRP of 1e8 nonzeros in test time, so it
computes a few hundred sampled output rows per mode (``oracle.mttkrp_rows``,
the full loop's rows bit for bit) across the degree spectrum: the hottest rows
(split across many partitions), rows at log-spaced degree ranks, random rows,
empty rows, the first and the last row, on every rank column.  Each element is
held to 1e-5 of the magnitude sum of its terms (``parity``).  Integer work is
checked bit-exactly at full size: the stream after loading and after each
remap holds record e at position b_d(e), and b_d is a permutation.

CP-ALS at full size: one sweep's last update is checked by its backward error
(the GPU factor times the normal matrix against the oracle's MTTKRP, element
by element), which does not depend on the conditioning of the normal matrix,
and ten sweeps' fits against the oracle's stored fits.
"""
import sys

import numpy as np
import pytest

import json
import os

import oracle
from paper_2405_08470_amd import synth
from parity import GAMMA, check_elementwise, degree_spectrum_rows, elementwise_ratio

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


def _rows_and_refs(dims, idx, val, factor_sets, count=160):
    """Sampled rows of every mode and, for each factor set, the oracle's rows
    and their magnitude sums M_abs."""
    out = []
    av = np.abs(np.asarray(val, dtype=np.float64))
    for d in range(len(dims)):
        rows = degree_spectrum_rows(idx[d], dims[d], count, seed=d)
        bk = oracle.bucket_rows(dims, idx, d)
        refs = []
        for Y in factor_sets:
            ref = oracle.mttkrp_rows(dims, idx, val, Y, d, rows, buckets=bk)
            aY = [np.abs(np.asarray(y, dtype=np.float64)) for y in Y]
            refs.append((ref, oracle.mttkrp_rows(dims, idx, av, aY, d, rows, buckets=bk)))
        out.append((rows, refs))
    return out


def _compare(outs, samples, k, label):
    for d, (rows, refs) in enumerate(samples):
        ref, absref = refs[k]
        got = outs[d][rows]
        e = _rel(got, ref)
        ratio = check_elementwise(got, ref, absref, label=f"{label} mode {d}")
        _say(f"  {label} mode {d}: {len(rows)} rows x {got.shape[1]} columns, rel {e:.2e}, "
             f"max element / M_abs {ratio:.2e}")
        assert e <= TOL


@pytest.mark.parametrize("name", ["zipf3_8e7", "zipf5_5e7", "zipf4_1e8"])
def test_full_size_all_modes_with_remap(name):
    spec = synth.WORKLOADS[name]
    _say(f"case full-size {spec.name}: dims {spec.dims} nnz {spec.nnz} R {spec.rank}")
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
    sets = [Y]
    if name == "zipf4_1e8":
        sets.append([oracle.bf16_round(y) for y in Y])
    samples = _rows_and_refs(dims, idx, val, sets)
    _compare(outs, samples, 0, "fp32")
    if name == "zipf4_1e8":
        # BF16 factor storage and gathers, FP32 accumulation: the kernel error
        # against the oracle on the rounded factors, and the storage error
        fb = [f.to(torch.bfloat16) for f in fdev]
        outb = _all_modes(t, dims, fb, R)
        _compare(outb, samples, 1, "bf16 kernel")
        for d, (rows, refs) in enumerate(samples):
            e = _rel(outb[d][rows], refs[0][0])
            _say(f"  bf16 storage mode {d}: rel {e:.2e}")
            assert e <= 1.5e-2
    assert S.tensor_info(t)["cur_mode"] == 0
    t.free()


def test_full_size_cp_als_sweep_last_mode_update_and_fit():
    """One CP-ALS sweep at 8e7 nonzeros.  The last mode's update solves
    Y_last diag(lambda) V = M_last, V the Hadamard product of the other
    (final) factors' Grams, M_last the MTTKRP of the last mode.

    (i) Backward error, every element: with the GPU's returned factors, the
    oracle forms M_last (FP64) and V (FP64 Grams of the FP32 factors); then
        |Y diag(lambda) V - M_last| <= 1e-5 M_abs + 4 u |Y| diag(lambda) |V|,
    u = 2^-24.  The first term is the FP32 MTTKRP's element bound; the second
    the rounding of the FP64 solution to FP32 (each entry of Y within u of
    the exact one, carried through V), plus room for the FP64 steps.  Neither
    grows with the conditioning of V.
    (ii) The fit, which is stationary at the least-squares optimum.  It is
    computed as sqrt(||X||^2 + ||Xhat||^2 - 2<X, Xhat>), which cancels: an
    FP32-level error (2^-24 relative) in the FP32 MTTKRP that <X, Xhat> is
    formed from reaches the fit amplified by ||X|| / ||X - Xhat|| =
    1 / (1 - fit), so the bound is max(1e-6, 8 2^-24 / (1 - fit)).
    Every column of Y_last has unit norm."""
    spec = synth.WORKLOADS["zipf3_8e7"]
    _say(f"case full-size CP-ALS sweep: {spec.name}")
    dims, idx, val = synth.make_coo(spec)
    Y0 = synth.make_factors(spec)
    R = spec.rank
    t = S.tensor_load_coo(dims, idx, val)
    f = [torch.from_numpy(y).cuda() for y in Y0]
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    fit = S.cp_als_iter(t, f, lam)
    t.free()
    Y = [x.cpu().numpy() for x in f]
    lam = lam.cpu().numpy()
    N = len(dims)
    d = N - 1
    grams = [Y[w].astype(np.float64).T @ Y[w].astype(np.float64) for w in range(N)]
    V = np.ones((R, R))
    for w in range(N - 1):
        V *= grams[w]
    bk = oracle.bucket_rows(dims, idx, d)
    M = oracle.mttkrp_parallel(dims, idx, val, Y, d, buckets=bk)
    M_abs = oracle.mttkrp_parallel(dims, idx, np.abs(val.astype(np.float64)),
                                   [np.abs(y.astype(np.float64)) for y in Y], d, buckets=bk)
    Yd = Y[d].astype(np.float64)
    lhs = (Yd * lam) @ V
    u = 2.0 ** -24
    bound = GAMMA * M_abs + 4 * u * ((np.abs(Yd) * lam) @ np.abs(V))
    ratio = elementwise_ratio(lhs, M, bound)
    _say(f"  backward error of the last update: max |Y lambda V - M| / bound {ratio:.3e} "
         f"(cond(V) {float(np.linalg.cond(V)):.3g})")
    assert ratio <= 1.0
    X = np.linalg.solve(V, M.T).T                     # M V^-1
    lam_o = np.linalg.norm(X, axis=0)
    Yn = X / lam_o
    fit_o = oracle.fit_from(oracle.norm_sq(dims, idx, val), M, Yn, lam_o,
                            grams[:N - 1] + [Yn.T @ Yn])
    tol_fit = max(1e-6, 8 * 2.0 ** -24 / (1.0 - fit_o))
    _say(f"  fit gpu {fit:.9f} oracle (exact last update) {fit_o:.9f} (bound {tol_fit:.2e})")
    assert abs(fit - fit_o) <= tol_fit
    norms = np.linalg.norm(Yd, axis=0)
    assert np.allclose(norms[lam > 0], 1.0, atol=1e-5)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "als_fits_full.json")


@pytest.mark.parametrize("name", ["zipf3_8e7", "zipf5_5e7"])
def test_full_size_ten_sweep_fits(name):
    """Ten CP-ALS sweeps on the full-size 3- and 5-mode workloads from their
    seeded factors: the fit after every sweep against the FP64 oracle's
    (stored by tests/golden/make_als_fits.py, which calls only the oracle).
    ALS is not contractive, so the FP32 and FP64 trajectories may part; the
    fits, stationary at each least-squares step, are held to 1e-4."""
    with open(GOLDEN) as fh:
        gold = json.load(fh)["workloads"][name]
    spec = synth.WORKLOADS[name]
    _say(f"case full-size ten sweeps: {spec.name}")
    dims, idx, val = synth.make_coo(spec)
    assert list(dims) == gold["dims"] and spec.nnz == gold["nnz"] and spec.rank == gold["rank"]
    Y0 = synth.make_factors(spec)
    t = S.tensor_load_coo(dims, idx, val, prep="device")
    del idx, val
    f = [torch.from_numpy(y).cuda() for y in Y0]
    lam = torch.empty(spec.rank, dtype=torch.float64, device="cuda")
    fits = [S.cp_als_iter(t, f, lam) for _ in range(len(gold["fits"]))]
    t.free()
    drift = [abs(a - b) for a, b in zip(fits, gold["fits"])]
    for k, (a, b) in enumerate(zip(fits, gold["fits"])):
        _say(f"  sweep {k + 1}: fit gpu {a:.9f} oracle {b:.9f} |diff| {abs(a - b):.2e}")
    assert max(drift) <= 1e-4
