"""FP64 CPU oracle for all-mode sparse MTTKRP inside CP-ALS.

TEST INFRASTRUCTURE ONLY.  The product library and its Python binding never
import, link or execute anything here; only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` do.  It shares no
code with the GPU path: the only common dependency is the seeded input
generator, which holds none of the method's arithmetic.

What is computed, and from which passage of the paper:

* ``mttkrp``      Eq. (1) (Sec. 2.1.4) elementwise as in Sec. 2.1.5 / Alg. 2;
                  a plain FP64 loop over COO nonzeros (``oracle.c``).
* ``mttkrp_parallel``  the same loop on all host cores: nonzeros bucketed by
                  output row, each row's terms added in input order by the
                  thread that owns the row, so the result is the plain loop's
                  bit for bit.
* ``plan``        Alg. 1 (Sec. 3.4): per-mode vertex ordering by degree and
                  least-filled assignment to kappa blocks; remap ids (Sec. 3.4,
                  3.5) as positions in each mode's stream; partition offsets.
                  Plus the split of vertices heavier than a cap into pieces,
                  which the paper does not have (it is an extension).
* ``cp_als``      CP-ALS (Sec. 2.1.4): the paper only names it; this follows
                  the textbook alternating least squares of Kolda and Bader
                  (SIAM Review 2009), the survey the paper cites for tensors.
* ``fit``         standard CP fit from the last MTTKRP (same source).

Readings taken where the paper is silent or ambiguous are listed next to the
code that takes them (partition order, ties, split pieces, stream order).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compiles oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_SO):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _SO,
                               os.path.join(_HERE, "oracle.c")])
    return _SO


def _load():
    global _lib
    if _lib is None:
        src = os.path.join(_HERE, "oracle.c")
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
            build()
        lib = ctypes.CDLL(_SO)
        lib.orc_mttkrp.restype = ctypes.c_int
        lib.orc_mttkrp.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p]
        lib.orc_bucket_rows.restype = ctypes.c_int
        lib.orc_bucket_rows.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_mttkrp_bucketed.restype = ctypes.c_int
        lib.orc_mttkrp_bucketed.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_int, ctypes.c_void_p]
        lib.orc_max_threads.restype = ctypes.c_int
        lib.orc_max_threads.argtypes = []
        lib.orc_lpt.restype = ctypes.c_int
        lib.orc_lpt.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


# ---------------------------------------------------------------------------
# spMTTKRP, Eq. (1)
# ---------------------------------------------------------------------------

def mttkrp(dims: Sequence[int], idx: np.ndarray, val: np.ndarray,
           factors: Sequence[np.ndarray], mode: int) -> np.ndarray:
    """M_mode(i, r) = sum_{e: i_mode(e)=i} val_e prod_{w!=mode} Y_w(i_w(e), r), in FP64.

    Stored FP32 (or BF16) values and factors are promoted to FP64 exactly.
    """
    lib = _load()
    N = len(dims)
    nnz = int(val.shape[0])
    dims64 = np.ascontiguousarray(dims, dtype=np.int64)
    idx32 = np.ascontiguousarray(idx, dtype=np.int32)
    v64 = np.ascontiguousarray(val, dtype=np.float64)
    R = int(factors[0].shape[1])
    f64 = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
    ptrs = (ctypes.c_void_p * N)(*[_ptr(f) for f in f64])
    out = np.empty((int(dims[mode]), R), dtype=np.float64)
    rc = lib.orc_mttkrp(N, _ptr(dims64), nnz, _ptr(idx32), _ptr(v64), ptrs, R, mode, _ptr(out))
    if rc != 0:
        raise ValueError("oracle mttkrp: bad argument or index out of range")
    return out


def max_threads() -> int:
    """Threads ``mttkrp_parallel`` uses by default (OpenMP's)."""
    return int(_load().orc_max_threads())


def bucket_rows(dims: Sequence[int], idx: np.ndarray, mode: int):
    """Row buckets of one mode: (rowptr [I+1], perm [nnz]) with the nonzeros
    of row i, in input order, at perm[rowptr[i]:rowptr[i+1]]."""
    lib = _load()
    nnz = int(idx.shape[1])
    dims64 = np.ascontiguousarray(dims, dtype=np.int64)
    idx32 = np.ascontiguousarray(idx, dtype=np.int32)
    rowptr = np.empty(int(dims[mode]) + 1, dtype=np.int64)
    perm = np.empty(max(nnz, 1), dtype=np.int64)
    if lib.orc_bucket_rows(len(dims), _ptr(dims64), nnz, _ptr(idx32), mode, _ptr(rowptr), _ptr(perm)) != 0:
        raise ValueError("oracle bucket_rows: bad argument or index out of range")
    return rowptr, perm


def mttkrp_parallel(dims: Sequence[int], idx: np.ndarray, val: np.ndarray,
                    factors: Sequence[np.ndarray], mode: int, buckets=None,
                    nthreads: int = 0, rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """``mttkrp`` on all host cores (``nthreads`` <= 0: OpenMP's default):
    identical to it bit for bit.  ``buckets`` = ``bucket_rows(...)`` of the
    same mode, computed here if not given.  With ``rows``, only those output
    rows, in the order listed: [len(rows), R]."""
    lib = _load()
    N = len(dims)
    nnz = int(val.shape[0])
    if buckets is None:
        buckets = bucket_rows(dims, idx, mode)
    rowptr, perm = buckets
    dims64 = np.ascontiguousarray(dims, dtype=np.int64)
    idx32 = np.ascontiguousarray(idx, dtype=np.int32)
    v64 = np.ascontiguousarray(val, dtype=np.float64)
    R = int(factors[0].shape[1])
    f64 = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
    ptrs = (ctypes.c_void_p * N)(*[_ptr(f) for f in f64])
    if rows is None:
        rl, nrows, nout = None, 0, int(dims[mode])
    else:
        rl = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = nout = int(rl.shape[0])
    out = np.empty((nout, R), dtype=np.float64)
    if nthreads <= 0:
        # small tensors: one thread (a parallel region costs more than the sum)
        nthreads = 0 if nnz >= (1 << 20) else 1
    rc = lib.orc_mttkrp_bucketed(N, _ptr(dims64), nnz, _ptr(idx32), _ptr(v64), ptrs, R, mode,
                                 _ptr(rowptr), _ptr(perm), None if rl is None else _ptr(rl), nrows,
                                 int(nthreads), _ptr(out))
    if rc != 0:
        raise ValueError("oracle mttkrp_parallel: bad argument or index out of range")
    return out


def mttkrp_rows(dims: Sequence[int], idx: np.ndarray, val: np.ndarray,
                factors: Sequence[np.ndarray], mode: int, rows: Sequence[int],
                buckets=None) -> np.ndarray:
    """Eq. (1) restricted to the listed output rows: FP64 [len(rows), R], the
    rows of ``mttkrp`` bit for bit (for full-size tensors, where only sampled
    rows are checked)."""
    return mttkrp_parallel(dims, idx, val, factors, mode, buckets=buckets, rows=rows)


# ---------------------------------------------------------------------------
# Algorithm 1 and the remap ids
# ---------------------------------------------------------------------------

def default_cap(nnz: int, kappa: int) -> int:
    """Pieces of a vertex hold at most ceil(nnz / kappa) hyperedges."""
    return max(1, -(-int(nnz) // int(kappa)))


def lpt_items(deg: np.ndarray, cap: int):
    """Items of Alg. 1 for one mode, in the order they are assigned.

    Every vertex (row) of the mode is an item, including vertices with no
    hyperedge (Alg. 1 iterates all of them).  Extension: a vertex of degree
    above ``cap`` (cap > 0) is cut into k = ceil(deg / cap) pieces whose sizes
    differ by at most one, the first (deg mod k) pieces one larger.
    Order: degree (size) decreasing, then row, then piece (reading: the paper
    sorts by degree and is silent on ties).
    Returns (rows, pieces, sizes) in assignment order.
    """
    deg = np.asarray(deg, dtype=np.int64)
    I = deg.shape[0]
    if cap > 0:
        k = np.where(deg > cap, -(-deg // cap), 1)
    else:
        k = np.ones(I, dtype=np.int64)
    rows = np.repeat(np.arange(I, dtype=np.int64), k)
    first = np.repeat(np.cumsum(k) - k, k)
    piece = np.arange(rows.shape[0], dtype=np.int64) - first
    kk = k[rows]
    q = deg[rows] // kk
    rem = deg[rows] % kk
    size = q + (piece < rem)
    order = np.lexsort((piece, rows, -size))
    return rows[order], piece[order], size[order]


def lpt(sizes: np.ndarray, kappa: int):
    """Least-filled assignment (Alg. 1) of already ordered items; C loop."""
    lib = _load()
    s = np.ascontiguousarray(sizes, dtype=np.int64)
    part = np.empty(s.shape[0], dtype=np.int32)
    loads = np.empty(kappa, dtype=np.int64)
    if lib.orc_lpt(s.shape[0], _ptr(s), int(kappa), _ptr(part), _ptr(loads)) != 0:
        raise ValueError("oracle lpt: bad argument")
    return part, loads


def piece_of_nonzero(row_of_e: np.ndarray, deg: np.ndarray, cap: int) -> np.ndarray:
    """Piece index of each nonzero within its row.

    Reading: the pieces of a split row take the row's nonzeros in input
    (canonical) order, piece j holding ranks [j*q + min(j, rem), ...).
    """
    nnz = row_of_e.shape[0]
    if cap <= 0:
        return np.zeros(nnz, dtype=np.int64)
    order = np.argsort(row_of_e, kind="stable")
    start = np.concatenate([[0], np.cumsum(deg)])[:-1]
    rank = np.empty(nnz, dtype=np.int64)
    rank[order] = np.arange(nnz, dtype=np.int64) - start[row_of_e[order]]
    d = deg[row_of_e]
    k = np.where(d > cap, -(-d // cap), 1)
    q = d // k
    rem = d % k
    big = rem * (q + 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        j = np.where(rank < big, rank // np.maximum(q + 1, 1),
                     rem + (rank - big) // np.maximum(q, 1))
    return j.astype(np.int64)


def plan(dims: Sequence[int], idx: np.ndarray, kappa: int,
         split_cap: Optional[int] = None) -> Dict[str, List[np.ndarray]]:
    """Partitions every mode (Alg. 1) and assigns remap ids.

    split_cap: None -> ceil(nnz/kappa); 0 or negative -> never split (pure
    Alg. 1, a heavy vertex stays whole).

    Returned per mode d:
      part[d]   partition of each nonzero (z_d(e)), int32 [nnz]
      loads[d]  nonzeros per partition, int64 [kappa]
      ptr[d]    partition offsets in the mode-d stream, int64 [kappa+1]
      b[d]      remap id of each nonzero = its position in the mode-d stream
      order[d]  the mode-d stream: order[d][p] = nonzero at position p
      item_rows / item_pieces / item_part[d]: the items and their blocks

    Stream order (reading; the paper fixes only that a stream is grouped by
    partition id and that the mode-0 stream follows the mode-0 indices): the
    mode-d stream is sorted by the key
        (z_d, i_d, z_{d-1}, i_{d-1}, ..., z_{d+1}, i_{d+1}, e)
    with mode numbers taken mod N, i.e. by partition, then by the output row,
    then by the same pair of the previous modes going backwards, then by the
    input position e.  Sec. 3.1 and 3.4 hold: each partition is contiguous
    and the mode-0 stream is ordered by the mode-0 indices within each
    partition.
    """
    idx = np.asarray(idx)
    N = len(dims)
    nnz = idx.shape[1]
    cap = default_cap(nnz, kappa) if split_cap is None else int(split_cap)
    out: Dict[str, List[np.ndarray]] = {k: [] for k in
                                        ("part", "loads", "ptr", "b", "order", "deg",
                                         "item_rows", "item_pieces", "item_part")}
    for d in range(N):
        rows_d = idx[d].astype(np.int64)
        deg = np.bincount(rows_d, minlength=int(dims[d])).astype(np.int64)
        it_rows, it_pieces, it_sizes = lpt_items(deg, cap)
        it_part, loads = lpt(it_sizes, kappa)
        # block of (row, piece)
        kmax = int(it_pieces.max()) + 1 if it_pieces.size else 1
        table = np.full((int(dims[d]), kmax), -1, dtype=np.int64)
        table[it_rows, it_pieces] = it_part
        piece = piece_of_nonzero(rows_d, deg, cap)
        z = table[rows_d, piece].astype(np.int32)
        out["part"].append(z)
        out["loads"].append(loads)
        out["ptr"].append(np.concatenate([[0], np.cumsum(loads)]).astype(np.int64))
        out["deg"].append(deg)
        out["item_rows"].append(it_rows)
        out["item_pieces"].append(it_pieces)
        out["item_part"].append(it_part)
    e = np.arange(nnz, dtype=np.int64)
    for d in range(N):
        key_msf = []  # most significant first
        for k in range(N):
            w = (d - k) % N
            key_msf.append(out["part"][w].astype(np.int64))
            key_msf.append(idx[w].astype(np.int64))
        key_msf.append(e)
        order = np.lexsort(tuple(reversed(key_msf)))
        b = np.empty(nnz, dtype=np.int64)
        b[order] = e
        out["order"].append(order.astype(np.int64))
        out["b"].append(b)
    return out


# ---------------------------------------------------------------------------
# BF16 storage of factors (the precision direction; the paper is silent)
# ---------------------------------------------------------------------------

def bf16_round(x: np.ndarray) -> np.ndarray:
    """FP32 values rounded to BF16 (8-bit exponent, 7-bit fraction) to nearest,
    ties to even, returned widened back to FP32 exactly.  Defined on the bit
    pattern: the lower 16 bits are dropped after adding half an ulp of the
    kept part (0x7FFF plus the lowest kept bit); NaNs stay NaN."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7F800000) == 0x7F800000
    nan &= (u & 0x007FFFFF) != 0
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    r = np.where(nan, (u & 0xFFFF0000) | 0x00400000, r)
    return r.astype(np.uint32).view(np.float32).reshape(np.shape(x))


# ---------------------------------------------------------------------------
# CP-ALS and fit (textbook; the paper only names the method)
# ---------------------------------------------------------------------------

def norm_sq(dims: Sequence[int], idx: np.ndarray, val: np.ndarray) -> float:
    """||X||_F^2 of the tensor whose repeated coordinates are summed first."""
    nnz = val.shape[0]
    if nnz == 0:
        return 0.0
    # coordinates in lexicographic order, input order among equal ones
    total = 1
    for I in dims:
        total *= int(I)
    if total < 2 ** 63:
        key = np.zeros(nnz, dtype=np.int64)
        for d, I in enumerate(dims):
            key = key * int(I) + idx[d].astype(np.int64)
        order = np.argsort(key, kind="stable")
        k = key[order]
        new = np.ones(nnz, dtype=bool)
        new[1:] = k[1:] != k[:-1]
    else:
        order = np.lexsort(tuple(idx[d] for d in reversed(range(len(dims)))))
        s = idx[:, order]
        new = np.ones(nnz, dtype=bool)
        new[1:] = np.any(s[:, 1:] != s[:, :-1], axis=0)
    grp = np.cumsum(new) - 1
    # each coordinate's values summed in input order
    sums = np.bincount(grp, weights=np.asarray(val, dtype=np.float64)[order])
    return float(np.dot(sums, sums))


class NotSPD(ArithmeticError):
    pass


def _chol(V: np.ndarray) -> np.ndarray:
    """Cholesky of the normal matrix; one ridge retry of 1e-12 tr(V)/R."""
    try:
        return np.linalg.cholesky(V)
    except np.linalg.LinAlgError:
        R = V.shape[0]
        Vr = V + (1e-12 * np.trace(V) / R) * np.eye(R)
        try:
            return np.linalg.cholesky(Vr)
        except np.linalg.LinAlgError as exc:
            raise NotSPD(str(exc)) from exc


def als_update(M: np.ndarray, grams: Sequence[np.ndarray], mode: int):
    """Y_mode = M V^-1 with V the Hadamard product of the other Grams; then the
    columns are scaled to unit 2-norm.  Returns (Y, lambda).  A zero column
    keeps lambda = 0 and stays zero."""
    R = M.shape[1]
    V = np.ones((R, R), dtype=np.float64)
    for w, G in enumerate(grams):
        if w != mode:
            V = V * G
    L = _chol(V)
    # Y^T = V^{-1} M^T via two triangular solves
    Z = np.linalg.solve(L, M.T)
    Y = np.linalg.solve(L.T, Z).T
    lam = np.sqrt(np.sum(Y * Y, axis=0))
    scale = np.where(lam > 0, 1.0 / np.where(lam > 0, lam, 1.0), 0.0)
    return Y * scale[None, :], lam


def fit_from(normX2: float, M_last: np.ndarray, Y_last: np.ndarray,
             lam: np.ndarray, grams: Sequence[np.ndarray]) -> float:
    """fit = 1 - ||X - Xhat|| / ||X|| with
    <X, Xhat> = sum_r lam_r sum_i M_last(i,r) Y_last(i,r) and
    ||Xhat||^2 = lam^T (Hadamard of all Grams) lam."""
    inner = float(np.sum(np.sum(M_last * Y_last, axis=0) * lam))
    H = np.ones_like(grams[0])
    for G in grams:
        H = H * G
    xhat2 = float(lam @ H @ lam)
    res2 = max(0.0, normX2 + xhat2 - 2.0 * inner)
    return 1.0 - np.sqrt(res2) / np.sqrt(normX2)


def cp_als(dims: Sequence[int], idx: np.ndarray, val: np.ndarray,
           factors: Sequence[np.ndarray], iters: int, gather=None):
    """Fixed-count CP-ALS in FP64, modes updated in the order 0..N-1.

    gather: optional map applied to each factor before it enters MTTKRP
    (e.g. storage rounding of the gathered copies); the solve, Grams and fit
    use the unrounded factors.  Returns (factors, lam, fits) with one fit per
    completed iteration.
    """
    N = len(dims)
    Y = [np.asarray(f, dtype=np.float64).copy() for f in factors]
    grams = [y.T @ y for y in Y]
    normX2 = norm_sq(dims, idx, val)
    # MTTKRP on all host cores: the plain loop's result bit for bit
    buckets = [bucket_rows(dims, idx, d) for d in range(N)]
    fits = []
    lam = np.ones(Y[0].shape[1])
    for _ in range(iters):
        M = None
        for d in range(N):
            G = Y if gather is None else [gather(y) for y in Y]
            M = mttkrp_parallel(dims, idx, val, G, d, buckets=buckets[d])
            Y[d], lam = als_update(M, grams, d)
            grams[d] = Y[d].T @ Y[d]
        fits.append(fit_from(normX2, M, Y[N - 1], lam, grams))
    return Y, lam, fits


# ---------------------------------------------------------------------------
# Gradient of the CP fit over the observed nonzeros (the differentiation
# direction; the adjoint of the model at the nonzeros is an MTTKRP, Eq. (1))
# ---------------------------------------------------------------------------

def model_at(idx: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """m_e = sum_r prod_w Y_w(i_w(e), r) at every nonzero, FP64."""
    nnz = idx.shape[1]
    out = np.empty(nnz, dtype=np.float64)
    f64 = [np.asarray(f, dtype=np.float64) for f in factors]
    step = 1 << 20
    for a in range(0, nnz, step):
        b = min(nnz, a + step)
        p = np.ones((b - a, f64[0].shape[1]))
        for w, f in enumerate(f64):
            p *= f[idx[w, a:b]]
        out[a:b] = p.sum(axis=1)
    return out


def cp_loss_grad(dims: Sequence[int], idx: np.ndarray, val: np.ndarray,
                 factors: Sequence[np.ndarray]):
    """loss = 1/2 sum_e (x_e - m_e)^2 and d loss / d Y_d = MTTKRP of the
    residuals (m_e - x_e) for every mode d, all in FP64."""
    m = model_at(idx, factors)
    r = m - np.asarray(val, dtype=np.float64)
    loss = 0.5 * float(np.dot(r, r))
    grads = [mttkrp(dims, idx, r, factors, d) for d in range(len(dims))]
    return loss, grads


def full_tensor(dims: Sequence[int], idx: np.ndarray, val: np.ndarray) -> np.ndarray:
    """Dense FP64 tensor with repeated coordinates summed (tiny sizes only)."""
    X = np.zeros(tuple(int(i) for i in dims), dtype=np.float64)
    np.add.at(X, tuple(idx[d] for d in range(len(dims))), val.astype(np.float64))
    return X
