"""The allocation-free entry point spt_mttkrp_noalloc against spt_mttkrp,
through the C ABI: bit-identical outputs and streams on two calls in a row,
the second on a smaller tensor (the fixed buffer keeps the first call's
contents), plus its size limit."""
import numpy as np
import pytest

from paper_2405_08470_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)
S = pytest.importorskip("paper_2405_08470_amd.spmttkrp")


def _pass(fn, t, dims, fdev, R):
    outs = []
    for d in range(len(dims)):
        out = torch.full((dims[d], R), float("nan"), dtype=torch.float32, device="cuda")
        fn(t, d, fdev, out, flags=S.FUSE_REMAP_NEXT)
        outs.append(out)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("warm", [False, True])
def test_noalloc_matches_mttkrp_on_two_calls_second_smaller(warm):
    cases = [((3000, 2500, 60_000), 400_000, 32, 0, "zipf"),
             ((700, 600, 500, 40), 60_000, 16, 97, "zipf")]
    for dims, nnz, R, kappa, dist in cases:
        print("case", dims, nnz, R, "warm" if warm else "cold", flush=True)
        idx, val = synth.random_coo(dims, nnz, seed=31, dist=dist, zipf_s=1.2)
        Y = synth.random_factors(dims, R, seed=32)
        fdev = [torch.from_numpy(y).cuda() for y in Y]
        t = S.tensor_load_coo(dims, idx, val, kappa=kappa)
        assert max(S.tensor_info(t)["split_rows"]) > 0
        if warm:
            ref = _pass(S.mttkrp, t, dims, fdev, R)          # builds the hot-row tables
            got = _pass(S.mttkrp_noalloc, t, dims, fdev, R)  # uses them
        else:
            got = _pass(S.mttkrp_noalloc, t, dims, fdev, R)  # no tables yet: memory only
            ref = _pass(S.mttkrp, t, dims, fdev, R)
        for d in range(len(dims)):
            assert np.array_equal(got[d].view(np.uint32), ref[d].view(np.uint32)), d
        assert S.tensor_info(t)["cur_mode"] == 0
        t.free()


def test_noalloc_rejects_a_carry_beyond_its_buffer():
    # every nonzero in one row, cut into one piece per partition: 65536 carry
    # slots x rank 128 x 4 bytes = 32 MiB > 16 MiB
    dims = (4, 300, 200)
    nnz = 1 << 21
    idx, val = synth.random_coo(dims, nnz, seed=41)
    idx[0, :] = 1
    t = S.tensor_load_coo(dims, idx, val, kappa=65536, prep="device")
    f = [torch.zeros((I, 128), dtype=torch.float32, device="cuda") for I in dims]
    out = torch.empty((dims[0], 128), dtype=torch.float32, device="cuda")
    with pytest.raises(S.SptError) as ei:
        S.mttkrp_noalloc(t, 0, f, out)
    assert ei.value.name == "SPT_ERR_UNSUPPORTED" and "16777216" in ei.value.message
    # rank 8 fits (65536 x 8 x 4 = 2 MiB) and equals spt_mttkrp
    f8 = [torch.from_numpy(y).cuda() for y in synth.random_factors(dims, 8, seed=42)]
    a = torch.empty((dims[0], 8), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    S.mttkrp_noalloc(t, 0, f8, a)
    S.mttkrp(t, 0, f8, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    t.free()
