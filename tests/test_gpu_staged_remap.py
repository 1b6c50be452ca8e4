"""The two forms of dynamic remapping (Alg. 3) against each other on the GPU.

opts.dr = 0 remaps in a pass of its own after the elementwise kernel, writing
the records of each chunk of the stream in destination order;
opts.dr = 1 stores every record at its next position from inside the
elementwise kernel.  Both must leave the same next-mode stream, bit for bit
(integer work), and the MTTKRP outputs must be bit-identical (the elementwise
kernel reads the same stream in the same order).  Cases cover every record
width (12, 16, 32, 48 bytes, i.e. chunks of 131072, 131072, 65536, 32768
records, each
sorted as runs of 4096 that are then merged, offsets past 16 bits stored
above the destination), a partial last chunk, an exact multiple of the
chunk, a chunk plus one record, two runs in one partial chunk, one nonzero,
no nonzeros, both
planners, the gradient's residual stream, which is remapped the same way, and
spt_remap_for_mode over one hop (the same pass) and two hops (a scatter).
"""
import sys

import numpy as np
import pytest

from paper_2405_08470_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)
S = pytest.importorskip("paper_2405_08470_amd.spmttkrp")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # name, dims, nnz, R, layout, record bytes
    ("w12_tail", (3000, 2500, 60_000), 250_001, 32, "auto", 12),
    ("w12_exact", (500, 400, 300), 131072 * 2, 16, "auto", 12),
    ("w12_chunk_plus_one", (300, 200, 100), 131072 + 1, 8, "auto", 12),
    ("w12_4mode_half16", (3000, 2500, 1000, 60), 140_000, 16, "auto", 12),
    ("w12_2mode", (5000, 4000), 60_000, 8, "auto", 12),
    ("w16_tail", (3000, 2500, 60_000), 250_001, 32, "word32", 16),
    ("w16_exact", (500, 400, 300), 131072 * 2, 16, "word32", 16),
    ("w16_chunk_plus_one", (300, 200, 100), 131072 + 1, 8, "word32", 16),
    ("w16_two_runs", (300, 200, 100), 4097, 8, "word32", 16),
    ("w16_5mode", (1000, 1000, 500, 200, 50), 120_000, 16, "half16", 16),
    ("w32_8mode", (20, 20, 20, 20, 20, 20, 20, 20), 50_000, 8, "half16", 32),
    ("w48_8mode", (70_000, 5, 5, 5, 5, 5, 5, 5), 30_000, 8, "word32", 48),
    ("one", (10, 10, 10), 1, 8, "auto", 12),
]


def _run(dims, idx, val, R, remap, prep, Y, layout):
    t = S.tensor_load_coo(dims, idx, val, remap=remap, prep=prep, layout=layout)
    f = [torch.from_numpy(y).cuda() for y in Y]
    streams, outs = [], []
    for d in range(len(dims)):
        out = torch.empty((dims[d], R), dtype=torch.float32, device="cuda")
        S.mttkrp(t, d, f, out, flags=S.FUSE_REMAP_NEXT)
        torch.cuda.synchronize()
        ridx, rval, cur = S.tensor_get_records(t)
        assert cur == (d + 1) % len(dims)
        streams.append((ridx, rval.view(np.uint32)))
        outs.append(out.cpu().numpy())
    info = S.tensor_info(t)
    t.free()
    return streams, outs, info


@pytest.mark.parametrize("name,dims,nnz,R,layout,rb", CASES, ids=[c[0] for c in CASES])
def test_staged_remap_equals_fused_remap(name, dims, nnz, R, layout, rb):
    _say("case", name, dims, nnz)
    idx, val = synth.random_coo(dims, nnz, seed=nnz % 1000, dist="zipf", zipf_s=1.1)
    Y = synth.random_factors(dims, R, seed=4)
    s_st, o_st, i_st = _run(dims, idx, val, R, "staged", "host", Y, layout)
    s_fu, o_fu, i_fu = _run(dims, idx, val, R, "fused", "device", Y, layout)
    assert i_st["record_bytes"] == i_fu["record_bytes"] == rb
    # a power of two of at least 4096 records; the fused form has no pass
    ch = i_st["remap_chunk"]
    assert ch >= 4096 and ch & (ch - 1) == 0 and i_fu["remap_chunk"] == 0
    for d in range(len(dims)):
        assert np.array_equal(s_st[d][0], s_fu[d][0]), f"indices after mode {d}"
        assert np.array_equal(s_st[d][1], s_fu[d][1]), f"values after mode {d}"
        assert np.array_equal(o_st[d].view(np.uint32), o_fu[d].view(np.uint32)), f"output of mode {d}"


def test_staged_remap_empty_tensor_and_remap_for_mode():
    dims = (5, 4, 3)
    t = S.tensor_load_coo(dims, np.zeros((3, 0), np.int32), np.zeros(0, np.float32))
    Y = [torch.ones((n, 8), device="cuda") for n in dims]
    for d in range(3):
        out = torch.full((dims[d], 8), 7.0, device="cuda")
        S.mttkrp(t, d, Y, out, flags=S.FUSE_REMAP_NEXT)
        assert torch.count_nonzero(out).item() == 0
    assert S.tensor_info(t)["cur_mode"] == 0
    t.free()
    # remap_for_mode: one hop (the chunk-ordered pass), then two hops (the
    # chained scatter), each checked against the remap ids
    dims = (300, 200, 500)
    idx, val = synth.random_coo(dims, 20_000, seed=9, dist="zipf")
    t = S.tensor_load_coo(dims, idx, val)

    def check(mode):
        ridx, rval, cur = S.tensor_get_records(t)
        b = S.tensor_get_remap(t, mode)
        assert cur == mode
        assert np.array_equal(ridx[:, b], idx) and np.array_equal(rval[b].view(np.uint32), val.view(np.uint32))
    S.remap_for_mode(t, 1)
    check(1)
    Y = [torch.from_numpy(y).cuda() for y in synth.random_factors(dims, 8, seed=2)]
    out = torch.empty((dims[1], 8), device="cuda")
    S.mttkrp(t, 1, Y, out, flags=S.FUSE_REMAP_NEXT)
    check(2)
    S.remap_for_mode(t, 1)
    check(1)
    t.free()


def test_gradient_identical_with_both_remaps():
    dims = (700, 600, 500, 40, 30)
    idx, val = synth.random_coo(dims, 150_000, seed=17, dist="zipf")
    Y = [0.5 * y for y in synth.random_factors(dims, 16, seed=18)]
    f = [torch.from_numpy(y).cuda() for y in Y]
    res = []
    for remap in ("staged", "fused"):
        t = S.tensor_load_coo(dims, idx, val, remap=remap)
        loss, grads = S.cp_gradient(t, f)
        res.append((loss.item(), [g.cpu().numpy() for g in grads]))
        assert S.tensor_info(t)["cur_mode"] == 0
        t.free()
    assert res[0][0] == res[1][0]
    for a, b in zip(res[0][1], res[1][1]):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
