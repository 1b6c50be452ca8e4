"""The library's HIP kernels run on the CPU (tests/cpuhip), checked against
the oracle (no GPU needed).

The library is built with ROCm's clang as host C++ against a stand-in
hip_runtime.h: workgroups run as fibers, cross-lane operations as wave-wide
rendezvous (every lane of the wave must reach them, as the kernels assume),
and every device allocation ends at a PROT_NONE page, so an out-of-bounds
access faults here instead of on a GPU.  The CP-ALS dense kernels and the
device planner are not part of this build.  Device pointers are host
pointers, so numpy buffers are passed directly.

Checks, on small versions of the GPU test shapes (2 to 8 modes, ranks 8 to
128): remap ids and the stream after every remap bit-exact against the
oracle's plan; every output element within 1e-5 of M_abs; BF16 factors
against the oracle on rounded factors; the fused remap, one copy per mode
and the allocation-free entry point bit-identical to the default path; empty
and degenerate tensors.
"""
import ctypes
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2405_08470_amd import synth
from parity import check_elementwise, mttkrp_abs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_08470_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "cpuhip")
CXX = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")
HOST = ["plan.cpp", "api.cpp"]
KERNELS = ["ec_n2", "ec_n3", "ec_n4", "ec_n5", "ec_n6", "ec_n7", "ec_n8", "ec_kernel", "dr_staged", "probe",
           "noalloc", "grad_kernel"]
FUSE = 1
AUTO = 2


_OBJS = {}
_OUTS = {}  # outputs of the first build, by (case, mode)


@pytest.fixture(scope="module", params=["chosen", "plain"])
def lib(request, tmp_path_factory):
    """The CPU build of the library.  "chosen": the elementwise kernel as the
    launch picks it (every kernel reports the same occupancy here, so the
    form that reuses the last gathered row); "plain": that launch built to
    always take the plain form."""
    if not os.path.exists(CXX):
        pytest.skip("ROCm clang++ not available")
    out = tmp_path_factory.mktemp("cpuhip")
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def run(cmd):
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}"

    if not _OBJS:
        odir = tmp_path_factory.mktemp("cpuhip_obj")
        jobs = [[CXX, *flags, "-c", os.path.join(CSRC, f), "-o", str(odir / (f + ".o"))] for f in HOST]
        jobs += [[CXX, *flags, "-c", os.path.join(HERE, f), "-o", str(odir / (f + ".o"))]
                 for f in ("runtime.cpp", "als_stubs.cpp")]
        jobs += [[CXX, *flags, "-x", "c++", "-c", os.path.join(CSRC, f + ".hip"), "-o", str(odir / (f + ".o"))]
                 for f in KERNELS]
        with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
            list(ex.map(run, jobs))
        _OBJS.update({os.path.basename(j[-1]): j[-1] for j in jobs})
    objs = dict(_OBJS)
    if request.param == "plain":
        o = str(out / "ec_kernel.o")
        run([CXX, *flags, "-DSPT_EC_FORM=0", "-x", "c++", "-c", os.path.join(CSRC, "ec_kernel.hip"), "-o", o])
        objs["ec_kernel.o"] = o
    so = str(out / "libspmttkrp_cpu.so")
    run([CXX, "-shared", "-o", so, *objs.values(), "-pthread"])
    L = ctypes.CDLL(so)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.spt_tensor_load_coo.argtypes = [i32, vp, i64, vp, vp, vp, vp, vp]
    L.spt_mttkrp.argtypes = [vp, i32, vp, i32, i32, vp, ctypes.c_uint32, vp]
    L.spt_mttkrp_noalloc.argtypes = [vp, i32, vp, i32, i32, vp, ctypes.c_uint32, vp]
    L.spt_remap_for_mode.argtypes = [vp, i32, vp]
    L.spt_tensor_get_remap.argtypes = [vp, i32, vp]
    L.spt_tensor_get_records.argtypes = [vp, vp, vp, vp]
    L.spt_tensor_info.argtypes = [vp, vp]
    L.spt_tensor_free.argtypes = [vp]
    L.spt_copy_probe.argtypes = [vp, vp, i64, vp]
    L.spt_last_error.restype = ctypes.c_char_p
    yield L
    shutil.rmtree(out, ignore_errors=True)


# the binding's mirrors of the header's structs (their layout is checked
# against the header in test_abi)
from paper_2405_08470_amd.spmttkrp import LAYOUTS, spt_info as Info, spt_opts as Opts  # noqa: E402


class T:
    """A tensor loaded into the CPU build."""

    def __init__(self, L, dims, idx, val, kappa=0, split_cap=None, copies=0, dr=0, layout=0):
        self.L, self.dims, self.N, self.nnz = L, tuple(dims), len(dims), idx.shape[1]
        o = Opts()
        o.kappa, o.copies, o.dr, o.layout = kappa, copies, dr, layout
        o.split_cap = 0 if split_cap is None else (split_cap if split_cap > 0 else -1)
        self._d = np.ascontiguousarray(dims, dtype=np.int64)
        self._i = np.ascontiguousarray(idx, dtype=np.int32)
        self._v = np.ascontiguousarray(val, dtype=np.float32)
        self.h = ctypes.c_void_p()
        rc = L.spt_tensor_load_coo(self.N, self._d.ctypes.data, self.nnz, self._i.ctypes.data,
                                   self._v.ctypes.data, ctypes.byref(o), None, ctypes.byref(self.h))
        assert rc == 0, L.spt_last_error()

    def info(self):
        i = Info()
        assert self.L.spt_tensor_info(self.h, ctypes.byref(i)) == 0
        return i

    def mttkrp(self, mode, factors, R, flags=FUSE, bf16=False, noalloc=False):
        arr = (ctypes.c_void_p * self.N)(*[f.ctypes.data for f in factors])
        out = np.full((self.dims[mode], R), np.nan, dtype=np.float32)
        fn = self.L.spt_mttkrp_noalloc if noalloc else self.L.spt_mttkrp
        rc = fn(self.h, mode, arr, 1 if bf16 else 0, R, out.ctypes.data, flags, None)
        assert rc == 0, self.L.spt_last_error()
        return out

    def remap(self, mode):
        b = np.empty(self.nnz, dtype=np.int64)
        assert self.L.spt_tensor_get_remap(self.h, mode, b.ctypes.data) == 0
        return b

    def records(self):
        idx = np.empty((self.N, self.nnz), dtype=np.int32)
        val = np.empty(self.nnz, dtype=np.float32)
        cur = ctypes.c_int32()
        assert self.L.spt_tensor_get_records(self.h, idx.ctypes.data, val.ctypes.data, ctypes.byref(cur)) == 0
        return idx, val, cur.value

    def free(self):
        self.L.spt_tensor_free(self.h)


def bf16_bits(y):
    """FP32 -> BF16 bit patterns (uint16) of the oracle's rounding."""
    return (oracle.bf16_round(y).view(np.uint32) >> 16).astype(np.uint16)


CASES = [
    # name, dims, nnz, dist, zipf_s, R, kappa, split_cap, layout (auto: the
    # 12-byte records wherever the indices fit 64 bits)
    ("zipf3_r32", (300, 250, 6000), 30_000, "zipf", 1.1, 32, 0, None, "auto"),
    ("zipf5_r32", (100, 100, 50, 20, 5), 20_000, "zipf", 1.2, 32, 97, None, "auto"),
    ("zipf4_r64", (500, 500, 200, 10), 15_000, "zipf", 1.1, 64, 0, None, "auto"),
    ("zipf3_r8", (400, 300, 200), 15_000, "zipf", 1.3, 8, 13, None, "auto"),
    ("zipf3_r128", (400, 300, 200), 5_000, "zipf", 1.1, 128, 0, None, "auto"),
    ("zipf2_nosplit", (500, 400), 15_000, "zipf", 1.5, 16, 31, 0, "auto"),
    ("zipf8_r16", (9, 8, 7, 6, 5, 4, 3, 2), 4_000, "zipf", 1.1, 16, 5, None, "auto"),
    ("uniform3_r16", (60, 50, 40), 8_000, "uniform", 1.1, 16, 0, None, "auto"),
    # 16-byte and wider records
    ("zipf3_r32_word32", (300, 250, 6000), 30_000, "zipf", 1.1, 32, 0, None, "word32"),
    ("zipf5_r32_half16", (100, 100, 50, 20, 5), 20_000, "zipf", 1.2, 32, 97, None, "half16"),
    ("zipf4_r64_packed", (500, 500, 200, 10), 15_000, "zipf", 1.1, 64, 0, None, "packed"),
    ("zipf8_r16_half16", (9, 8, 7, 6, 5, 4, 3, 2), 4_000, "zipf", 1.1, 16, 5, None, "half16"),
    # two remap chunks of 131072 records, the last one partial
    ("zipf3_chunks", (400, 300, 2000), 140_000, "zipf", 1.1, 8, 0, None, "auto"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_all_modes_with_remap_against_the_oracle(lib, case):
    name, dims, nnz, dist, s, R, kappa, cap, layout = case
    idx, val = synth.random_coo(dims, nnz, seed=17, dist=dist, zipf_s=s)
    Y = synth.random_factors(dims, R, seed=18)
    t = T(lib, dims, idx, val, kappa=kappa, split_cap=cap, layout=LAYOUTS[layout])
    assert t.info().record_bytes == (12 if layout == "auto" else 16 if len(dims) <= 6 else 32), name
    plan = oracle.plan(dims, idx, t.info().kappa, split_cap=cap)
    N = len(dims)
    for d in range(N):
        assert np.array_equal(t.remap(d), plan["b"][d]), f"remap ids of mode {d}"
    for d in range(N):
        out = t.mttkrp(d, Y, R)
        gi, gv, cm = t.records()
        nxt = (d + 1) % N
        o = plan["order"][nxt]
        assert cm == nxt and np.array_equal(gi, idx[:, o]) and np.array_equal(gv, val[o]), f"stream after {d}"
        ref = oracle.mttkrp(dims, idx, val, Y, d)
        check_elementwise(out, ref, mttkrp_abs(dims, idx, val, Y, d), label=f"{name} mode {d}")
        # both forms of the elementwise kernel give the same bits (the plain
        # build runs after the chosen one)
        key = (name, d)
        if key in _OUTS:
            assert np.array_equal(out.view(np.uint32), _OUTS[key].view(np.uint32)), f"{name} mode {d} forms"
        else:
            _OUTS[key] = out
    t.free()


def test_bf16_factors_against_the_oracle_on_rounded_factors(lib):
    dims, R = (500, 500, 200, 10), 64
    idx, val = synth.random_coo(dims, 15_000, seed=23, dist="zipf", zipf_s=1.1)
    Y = synth.random_factors(dims, R, seed=24)
    Yb = [oracle.bf16_round(y) for y in Y]
    t = T(lib, dims, idx, val)
    for d in range(len(dims)):
        out = t.mttkrp(d, [bf16_bits(y) for y in Y], R, bf16=True)
        check_elementwise(out, oracle.mttkrp(dims, idx, val, Yb, d), mttkrp_abs(dims, idx, val, Yb, d),
                          label=f"bf16 mode {d}")
    t.free()


def test_fused_remap_one_copy_and_noalloc_give_the_same_bits(lib):
    dims, R = (200, 150, 3000), 32
    idx, val = synth.random_coo(dims, 25_000, seed=27, dist="zipf", zipf_s=1.2)
    Y = synth.random_factors(dims, R, seed=28)
    ts = T(lib, dims, idx, val, kappa=29)
    tf = T(lib, dims, idx, val, kappa=29, dr=1)
    tc = T(lib, dims, idx, val, kappa=29, copies=1)
    tn = T(lib, dims, idx, val, kappa=29)
    for d in range(3):
        a = ts.mttkrp(d, Y, R)
        b = tf.mttkrp(d, Y, R)
        c = tc.mttkrp(d, Y, R, flags=0)
        e = tn.mttkrp(d, Y, R, noalloc=True)
        for x in (b, c, e):
            assert np.array_equal(a.view(np.uint32), x.view(np.uint32)), d
        assert np.array_equal(ts.records()[0], tf.records()[0]) and np.array_equal(ts.records()[0], tn.records()[0])
    for t in (ts, tf, tc, tn):
        t.free()


@pytest.mark.parametrize("kind", ["empty", "one_nonzero", "kappa_above_nnz", "unit_modes", "single_hot_row"])
def test_edge_cases(lib, kind):
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
        idx, val = synth.random_coo(dims, 3000, seed=2)
        kw = {"kappa": 16}
    else:
        dims = (64, 50, 40)
        idx, val = synth.random_coo(dims, 8000, seed=3)
        idx[0, :] = 7
        kw = {"kappa": 24}
    Y = synth.random_factors(dims, R, seed=5)
    t = T(lib, dims, idx, val, **kw)
    for d in range(len(dims)):
        out = t.mttkrp(d, Y, R)
        if kind == "empty":
            assert np.all(out == 0)
        else:
            check_elementwise(out, oracle.mttkrp(dims, idx, val, Y, d), mttkrp_abs(dims, idx, val, Y, d),
                              label=f"{kind} mode {d}")
    assert t.info().cur_mode == 0
    t.free()


@pytest.mark.parametrize("dims,layout,rb", [
    ((5000, 4000), "auto", 12),                     # 32-bit indices in 64 bits
    ((3000, 2500, 1000, 60), "auto", 12),           # 16-bit fields
    ((100_000, 80_000, 3000), "auto", 12),          # 17 + 17 + 12 bit fields
    ((3_000_000, 3_000_000, 3_000_000), "auto", 16),  # 66 index bits: 16-byte words
    ((70_000, 70_000, 70_000, 70_000), "auto", 16),   # 68 bits: packed in 96
    ((3_000_000, 3_000_000, 3_000_000), "compact", None),
    ((70_000, 70_000, 70_000, 70_000), "compact", None),
    ((9, 8, 7, 6, 5, 4, 3, 2), "compact", 12),
])
def test_record_layout_choice(lib, dims, layout, rb):
    """The automatic layout takes the 12-byte record whenever the indices fit
    64 bits; asking for it where they do not fit is refused."""
    idx, val = synth.random_coo(dims, 300, seed=5)
    if rb is None:
        o = Opts()
        o.layout = LAYOUTS[layout]
        d = np.ascontiguousarray(dims, dtype=np.int64)
        i = np.ascontiguousarray(idx, dtype=np.int32)
        v = np.ascontiguousarray(val, dtype=np.float32)
        h = ctypes.c_void_p()
        rc = lib.spt_tensor_load_coo(len(dims), d.ctypes.data, i.shape[1], i.ctypes.data, v.ctypes.data,
                                     ctypes.byref(o), None, ctypes.byref(h))
        assert rc != 0 and b"layout" in lib.spt_last_error()
        return
    t = T(lib, dims, idx, val, layout=LAYOUTS[layout])
    assert t.info().record_bytes == rb
    gi, gv, _ = t.records()
    o = oracle.plan(dims, idx, t.info().kappa)["order"][0]
    assert np.array_equal(gi, idx[:, o]) and np.array_equal(gv, val[o])
    t.free()


def test_misaligned_factor_or_output_is_rejected(lib):
    """Rows move as 16-byte vectors: a factor, output or gradient matrix that
    does not start on a 16-byte boundary is refused before any launch."""
    dims, R = (50, 40, 30), 8
    idx, val = synth.random_coo(dims, 500, seed=4)
    t = T(lib, dims, idx, val)
    Y = synth.random_factors(dims, R, seed=6)
    pad = [np.zeros(y.size + 4, np.float32) for y in Y]  # room for a 4-byte shift
    ptrs = [p.ctypes.data for p in pad]
    assert all(p % 16 == 0 for p in ptrs)
    out = np.zeros(dims[0] * R + 4, np.float32)
    L = lib
    bad = (ctypes.c_void_p * 3)(ptrs[0], ptrs[1] + 4, ptrs[2])
    good = (ctypes.c_void_p * 3)(*ptrs)
    assert L.spt_mttkrp(t.h, 0, bad, 0, R, out.ctypes.data, FUSE, None) != 0
    assert b"16-byte aligned" in L.spt_last_error()
    assert L.spt_mttkrp(t.h, 0, good, 0, R, out.ctypes.data + 4, FUSE, None) != 0
    assert b"16-byte aligned" in L.spt_last_error()
    assert L.spt_mttkrp_noalloc(t.h, 0, bad, 0, R, out.ctypes.data, FUSE, None) != 0
    assert t.info().cur_mode == 0  # nothing ran
    t.free()


def test_copy_probe(lib):
    src = np.arange(4096 * 4, dtype=np.uint32)
    dst = np.zeros_like(src)
    assert lib.spt_copy_probe(src.ctypes.data, dst.ctypes.data, src.nbytes, None) == 0
    assert np.array_equal(src, dst)
    assert lib.spt_copy_probe(src.ctypes.data, dst.ctypes.data, 20, None) != 0
