"""Record layouts (Sec. 3.5: how a nonzero's indices are stored) against each
other on the GPU: 32-bit index words, 16-bit fields and packed bit fields of
ceil(log2 I_w) bits, in 16-byte (or wider) records and in the compact
12-byte record (the indices in 64 bits), 2 to 8 modes.  The layout changes only how indices are decoded, so the
streams must unpack to the same records and the MTTKRP outputs must be
bit-identical across layouts, and equal to the oracle within 1e-5.  Layouts
that do not fit a shape are refused with SPT_ERR_UNSUPPORTED, by both
planners.
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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _passes(dims, idx, val, R, Y, layout, prep):
    t = S.tensor_load_coo(dims, idx, val, layout=layout, prep=prep)
    f = [torch.from_numpy(y).cuda() for y in Y]
    rec = S.tensor_get_records(t)
    outs = []
    for d in range(len(dims)):
        out = torch.empty((dims[d], R), dtype=torch.float32, device="cuda")
        S.mttkrp(t, d, f, out, flags=S.FUSE_REMAP_NEXT)
        outs.append(out.cpu().numpy())
    loss, grads = S.cp_gradient(t, f)
    rb = S.tensor_info(t)["record_bytes"]
    t.free()
    return rb, rec, outs, loss.item(), [g.cpu().numpy() for g in grads]


CASES = [
    # name, dims, nnz, R, {layout: record bytes}
    ("2mode", (5000, 4000), 60_000, 16, {"compact": 12, "word32": 16}),
    ("3mode", (100_000, 80_000, 3000), 100_000, 32, {"compact": 12, "word32": 16}),
    ("4mode", (3000, 2500, 1000, 60), 120_000, 16,
     {"compact": 12, "half16": 16, "packed": 16, "word32": 32}),
    ("4mode_big", (70_000, 2500, 1000, 60), 80_000, 16, {"compact": 12, "packed": 16, "word32": 32}),
    ("5mode", (1000, 1000, 500, 200, 50), 100_000, 32,
     {"compact": 12, "half16": 16, "packed": 16, "word32": 32}),
    ("6mode_big", (70_000, 300, 200, 40, 30, 20), 60_000, 8, {"compact": 12, "packed": 16, "word32": 32}),
    ("7mode", (9, 8, 7, 6, 5, 4, 3), 20_000, 8, {"compact": 12, "word32": 32}),
    ("8mode", (9, 8, 7, 6, 5, 4, 3, 2), 20_000, 8, {"compact": 12, "half16": 32, "word32": 48}),
]


@pytest.mark.parametrize("name,dims,nnz,R,layouts", CASES, ids=[c[0] for c in CASES])
def test_layouts_give_identical_results(name, dims, nnz, R, layouts):
    _say("case", name, dims, nnz, list(layouts))
    idx, val = synth.random_coo(dims, nnz, seed=21, dist="zipf", zipf_s=1.1)
    Y = [0.5 * y for y in synth.random_factors(dims, R, seed=22)]
    ref = None
    for k, (layout, rb) in enumerate(layouts.items()):
        got = _passes(dims, idx, val, R, Y, layout, "device" if k % 2 else "host")
        assert got[0] == rb, (layout, got[0])
        if ref is None:
            ref = got
            for d in range(len(dims)):
                M = oracle.mttkrp(dims, idx, val, Y, d)
                e = float(np.linalg.norm(got[2][d] - M) / np.linalg.norm(M))
                ratio = check_elementwise(got[2][d], M, mttkrp_abs(dims, idx, val, Y, d),
                                          label=f"{layout} mode {d}")
                _say(f"  {layout} mode {d}: rel {e:.2e}, max element / M_abs {ratio:.2e}")
                assert e <= 1e-5
            continue
        assert np.array_equal(got[1][0], ref[1][0]) and np.array_equal(got[1][1].view(np.uint32),
                                                                        ref[1][1].view(np.uint32)), layout
        for d in range(len(dims)):
            assert np.array_equal(got[2][d].view(np.uint32), ref[2][d].view(np.uint32)), (layout, d)
            assert np.array_equal(got[4][d].view(np.uint32), ref[4][d].view(np.uint32)), (layout, d)
        assert got[3] == ref[3]


@pytest.mark.parametrize("dims,layout", [
    ((50, 40, 30), "half16"),                   # 3 modes: 32-bit indices only
    ((50, 40, 30), "packed"),
    ((9, 8, 7, 6, 5, 4, 3), "half16"),          # 7 modes: 32-bit indices only
    ((70_000, 30, 20, 10), "half16"),           # a mode with more than 65536 rows
    ((9, 8, 7, 6, 5, 4, 3, 2), "packed"),       # 16-byte packed fields: 4..6 modes
    ((3_000_000, 3_000_000, 3_000_000), "compact"),  # 66 index bits
    ((70_000, 70_000, 70_000, 70_000), "compact"),   # 68 index bits
])
def test_layout_that_does_not_fit_is_refused(dims, layout):
    idx, val = synth.random_coo(dims, 500, seed=3, dist="uniform")
    msgs = []
    for prep in ("host", "device"):
        with pytest.raises(S.SptError) as ei:
            S.tensor_load_coo(dims, idx, val, layout=layout, prep=prep)
        assert ei.value.name == "SPT_ERR_UNSUPPORTED"
        msgs.append(ei.value.message)
    assert msgs[0] == msgs[1]
