"""BF16 factor storage and gathers with FP32 accumulation, through the C ABI.

Two errors are separated:
  kernel error  -- against the FP64 oracle fed the BF16-rounded factors
                   (widened exactly): the same tolerances as FP32, 1e-5
                   relative per mode and 1e-5 of M_abs per element;
  storage error -- against the FP64 oracle on the FP32 factors: BF16 keeps
                   8 significand bits, so about 2^-8 / sqrt(3) per factor
                   entry, a few 1e-3 relative for a product of two or three.
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [("zipf4_r64", synth.scaled(synth.WORKLOADS["zipf4_1e8"], 300_000, dims=(5000, 5000, 2000, 100))),
         ("zipf3_r32", synth.scaled(synth.WORKLOADS["zipf3_8e7"], 300_000, dims=(3000, 2500, 60_000))),
         ("zipf5_r32", synth.scaled(synth.WORKLOADS["zipf5_5e7"], 200_000)),
         ("uniform3_r16", synth.WORKLOADS["uniform3_1e5"])]


@pytest.mark.parametrize("name,spec", CASES, ids=[c[0] for c in CASES])
def test_mttkrp_bf16_gathers(name, spec):
    print("case", name, flush=True)
    dims, idx, val = synth.make_coo(spec)
    Y = synth.make_factors(spec)
    Yb = [oracle.bf16_round(y) for y in Y]
    t = S.tensor_load_coo(dims, idx, val)
    fb = [torch.from_numpy(y).cuda().to(torch.bfloat16) for y in Y]
    # torch's cast and the oracle's rounding agree bit for bit
    for y, f in zip(Yb, fb):
        assert np.array_equal(f.float().cpu().numpy().view(np.uint32), y.view(np.uint32))
    R = spec.rank
    for d in range(len(dims)):
        out = torch.empty((dims[d], R), dtype=torch.float32, device="cuda")
        S.mttkrp(t, d, fb, out, flags=S.FUSE_REMAP_NEXT)
        got = out.cpu().numpy()
        refb = oracle.mttkrp(dims, idx, val, Yb, d)
        kern = _rel(got, refb)
        stor = _rel(got, oracle.mttkrp(dims, idx, val, Y, d))
        ratio = check_elementwise(got, refb, mttkrp_abs(dims, idx, val, Yb, d), label=f"bf16 mode {d}")
        print(f"  mode {d}: kernel error {kern:.2e} (max element / M_abs {ratio:.2e}), "
              f"storage error {stor:.2e}", flush=True)
        assert kern <= 1e-5
        assert stor <= 1.5e-2
    assert S.tensor_info(t)["cur_mode"] == 0
    t.free()


def test_cp_als_with_bf16_gathers_one_sweep():
    # The GPU rounds its FP32 iterates to BF16, the oracle its FP64 ones; the
    # iterates differ by ~1e-6, which flips the rounding of a ~1e-6 / 2^-8
    # fraction of entries by 2^-8 each: ~sqrt(3e-4) * 4e-3 ~ 7e-5 relative.
    spec = synth.scaled(synth.WORKLOADS["zipf4_1e8"], 200_000, dims=(4000, 4000, 1500, 80))
    dims, idx, val = synth.make_coo(spec)
    Y0 = synth.make_factors(spec)
    t = S.tensor_load_coo(dims, idx, val)
    f = [torch.from_numpy(y).cuda() for y in Y0]
    lam = torch.empty(spec.rank, dtype=torch.float64, device="cuda")
    fit = S.cp_als_iter(t, f, lam, bf16_gather=True)
    Yo, lo, fo = oracle.cp_als(dims, idx, val, Y0, 1, gather=oracle.bf16_round)
    for d in range(len(dims)):
        e = _rel(f[d].cpu().numpy(), Yo[d])
        print(f"  factor {d}: rel {e:.2e}", flush=True)
        assert e <= 3e-4
    assert abs(fit - fo[0]) <= 1e-4
    # and against the FP32-gather oracle the BF16 storage error stays small
    _, _, f32 = oracle.cp_als(dims, idx, val, Y0, 1)
    assert abs(fit - f32[0]) <= 5e-3
    t.free()
