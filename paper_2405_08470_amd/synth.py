"""Seeded synthetic sparse tensors and factor matrices.

This module only draws inputs.  It holds none of the spMTTKRP arithmetic, so
both the FP64 oracle (``oracle/``) and the GPU path can consume the same
inputs without sharing any code of the method itself.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter mode: the k-th
draw of stream ``sid`` under seed ``seed`` is ``mix(key(seed, sid) + (k+1)*G)``
with G the golden-ratio increment.  Every array has its own stream id, so a
prefix of any array is reproducible without generating the others.

Workloads stand in for the paper's FROSTT / recommender tensors (Sec. 5.1.3,
Table 3), which are not available here: 3- to 5-mode tensors, uniform or
Zipf-skewed indices, tens of millions of nonzeros.
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence, Tuple

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 21


def _threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _chunked(n: int, fn) -> None:
    """Runs fn(a, b) over [0, n) in chunks; numpy releases the GIL inside."""
    spans = [(a, min(n, a + _CHUNK)) for a in range(0, n, _CHUNK)]
    if len(spans) <= 1:
        for a, b in spans:
            fn(a, b)
        return
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda ab: fn(*ab), spans))


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (variant 13 of Stafford's mixers)."""
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, sid: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = np.array([(seed & 0xFFFFFFFF) * 0x10001 + sid * 0x1000193], dtype=np.uint64)
        return _mix(s * _GAMMA + np.uint64(0x632BE59BD9B4E019))[0]


def raw_u64(seed: int, sid: int, n: int, start: int = 0) -> np.ndarray:
    """Draws ``start .. start+n-1`` of stream ``sid`` as uint64."""
    out = np.empty(n, dtype=np.uint64)
    key = _key(seed, sid)

    def body(a: int, b: int) -> None:
        with np.errstate(over="ignore"):
            ctr = np.arange(start + a + 1, start + b + 1, dtype=np.uint64)
            out[a:b] = _mix(key + ctr * _GAMMA)

    _chunked(n, body)
    return out


def uniform01(seed: int, sid: int, n: int, start: int = 0) -> np.ndarray:
    """FP64 uniforms in [0, 1) from the top 53 bits of each draw."""
    return (raw_u64(seed, sid, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, sid: int, n: int) -> np.ndarray:
    """FP64 standard normals by Box-Muller on pairs of uniforms."""
    m = (n + 1) // 2
    u = uniform01(seed, sid, 2 * m)
    u1 = 1.0 - u[0::2]  # (0, 1]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * m, dtype=np.float64)
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:n]


def permutation(seed: int, sid: int, n: int) -> np.ndarray:
    """A seeded uniform random permutation of [0, n) (argsort of 64-bit keys)."""
    return np.argsort(raw_u64(seed, sid, n), kind="stable").astype(np.int64)


def zipf_ranks(seed: int, sid: int, n: int, size: int, s: float) -> np.ndarray:
    """Ranks k in [0, size) with P(k) proportional to (k+1)^-s, by inverse CDF."""
    w = np.arange(1, size + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    out = np.empty(n, dtype=np.int64)
    key = _key(seed, sid)

    def body(a: int, b: int) -> None:
        with np.errstate(over="ignore"):
            ctr = np.arange(a + 1, b + 1, dtype=np.uint64)
            u = (_mix(key + ctr * _GAMMA) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        k = np.searchsorted(cdf, u, side="right")
        np.minimum(k, size - 1, out=k)
        out[a:b] = k

    _chunked(n, body)
    return out


# Stream ids: mode d indices -> d; factor w -> 16 + w; values -> 32;
# noise -> 33; starting-point perturbation of factor w -> 40 + w;
# permutations of mode d -> 48 + d; top-up draws -> 64 + top-up iteration.
SID_FACTOR = 16
SID_VALUES = 32
SID_NOISE = 33
SID_START = 40
SID_PERM = 48
SID_TOPUP = 64


@dataclasses.dataclass(frozen=True)
class TensorSpec:
    """Recipe of one synthetic COO tensor."""

    name: str
    dims: Tuple[int, ...]
    nnz: int
    rank: int
    dist: str = "uniform_distinct"   # or "zipf"
    zipf_s: float = 1.1
    values: str = "uniform"          # "lognormal", or "planted" (see planted_parts)
    seed: int = 1
    als_iters: int = 5
    noise_sd: float = 0.0            # planted values: standard deviation of the noise

    @property
    def nmodes(self) -> int:
        return len(self.dims)


# The workloads of the benchmark configurations (3-, 4- and 5-mode, uniform
# and skewed).  Index permutations are applied to every Zipf mode so hot rows
# do not sit at low ids.
WORKLOADS = {
    "uniform3_1e5": TensorSpec("uniform3_1e5", (1000, 800, 600), 100_000, 16,
                  "uniform_distinct", values="uniform", seed=1, als_iters=5),
    "zipf3_8e7": TensorSpec("zipf3_8e7", (100_000, 80_000, 2_000_000), 80_000_000, 32,
                  "zipf", 1.1, "uniform", seed=2, als_iters=10),
    "zipf5_5e7": TensorSpec("zipf5_5e7", (10_000, 10_000, 5_000, 200, 50), 50_000_000, 32,
                  "zipf", 1.2, "lognormal", seed=3, als_iters=10),
    "zipf4_1e8": TensorSpec("zipf4_1e8", (50_000, 50_000, 20_000, 1_000), 100_000_000, 64,
                  "zipf", 1.1, "uniform", seed=4, als_iters=10),
    # Observed entries of a planted rank-16 model plus N(0, 0.01^2) noise:
    # the gradient-fit workload.
    "planted4_5e7": TensorSpec("planted4_5e7", (20_000, 20_000, 10_000, 500), 50_000_000, 16,
                  "uniform_distinct", values="planted", seed=5, als_iters=0,
                  noise_sd=0.01),
}


def scaled(spec: TensorSpec, nnz: int, dims: Optional[Sequence[int]] = None,
           rank: Optional[int] = None, seed: Optional[int] = None) -> TensorSpec:
    """Same distribution, other size (for tests the oracle finishes quickly)."""
    return dataclasses.replace(
        spec, nnz=int(nnz), dims=tuple(dims) if dims is not None else spec.dims,
        rank=spec.rank if rank is None else int(rank),
        seed=spec.seed if seed is None else int(seed),
        name=f"{spec.name}@{nnz}")


def _first_copies(keys: np.ndarray) -> np.ndarray:
    """Boolean mask keeping the first occurrence of every key (draw order)."""
    srt = np.sort(keys)
    rep = np.unique(srt[1:][srt[1:] == srt[:-1]])
    keep = np.ones(keys.size, dtype=bool)
    if rep.size:
        pos = np.searchsorted(rep, keys)
        hit = np.flatnonzero(rep[np.minimum(pos, rep.size - 1)] == keys)
        # among the positions holding a repeated key, keep the first of each
        order = np.lexsort((hit, keys[hit]))
        h = hit[order]
        k = keys[h]
        later = np.ones(h.size, dtype=bool)
        later[0] = False
        later[1:] = k[1:] == k[:-1]
        keep[h[later]] = False
    return keep


def _uniform_distinct(spec: TensorSpec) -> np.ndarray:
    """Distinct coordinates, uniform per mode; first-drawn copies are kept."""
    dims = spec.dims
    total = 1
    for i in dims:
        total *= int(i)
    if spec.nnz > total:
        raise ValueError("more distinct nonzeros requested than the tensor holds")
    if total >= 2 ** 63:
        raise ValueError("linearised coordinates exceed 63 bits")
    keys = np.empty(0, dtype=np.int64)
    rnd = 0
    need = spec.nnz
    while True:
        draw = int(need * 1.05) + 64
        cols = []
        for d, I in enumerate(dims):
            sid = d if rnd == 0 else SID_TOPUP + rnd * 8 + d
            u = raw_u64(spec.seed, sid, draw)
            cols.append((u % np.uint64(I)).astype(np.int64))
        lin = np.zeros(draw, dtype=np.int64)
        for d, I in enumerate(dims):
            lin = lin * int(I) + cols[d]
        allk = np.concatenate([keys, lin])
        keys = allk[_first_copies(allk)]
        if keys.size >= spec.nnz:
            keys = keys[: spec.nnz]
            break
        need = spec.nnz - keys.size
        rnd += 1
    idx = np.empty((len(dims), spec.nnz), dtype=np.int32)
    rem = keys.copy()
    for d in range(len(dims) - 1, -1, -1):
        idx[d] = (rem % dims[d]).astype(np.int32)
        rem //= dims[d]
    return idx


def _zipf(spec: TensorSpec) -> np.ndarray:
    idx = np.empty((spec.nmodes, spec.nnz), dtype=np.int32)
    for d, I in enumerate(spec.dims):
        k = zipf_ranks(spec.seed, d, spec.nnz, I, spec.zipf_s)
        perm = permutation(spec.seed, SID_PERM + d, I)
        idx[d] = perm[k].astype(np.int32)
    return idx


def make_coo(spec: TensorSpec) -> Tuple[Tuple[int, ...], np.ndarray, np.ndarray]:
    """Returns (dims, indices int32 [N, nnz] 0-based, values float32 [nnz])."""
    if spec.dist == "uniform_distinct":
        idx = _uniform_distinct(spec)
    elif spec.dist == "zipf":
        idx = _zipf(spec)
    else:
        raise ValueError(spec.dist)
    if spec.values == "uniform":
        val = uniform01(spec.seed, SID_VALUES, spec.nnz).astype(np.float32)
    elif spec.values == "lognormal":
        val = np.exp(normal(spec.seed, SID_VALUES, spec.nnz)).astype(np.float32)
    elif spec.values == "planted":
        raise ValueError("planted values are the model at the nonzeros plus noise: "
                         "draw the parts with planted_parts() and evaluate the model there")
    else:
        raise ValueError(spec.values)
    return tuple(int(i) for i in spec.dims), idx, val


def planted_parts(spec: TensorSpec):
    """Draws of a planted workload: (dims, indices int32 [N, nnz], planted
    factors P_w (FP32, I_w x R, entries N(0,1) * R^(-1/(2N)) so that the model
    at a nonzero has unit variance), noise (FP64 [nnz], N(0, noise_sd^2))).
    The observed value is x_e = sum_r prod_w P_w(i_w(e), r) + noise_e; that
    sum is left to the caller."""
    if spec.values != "planted":
        raise ValueError("not a planted workload")
    dims = tuple(int(i) for i in spec.dims)
    if spec.dist == "uniform_distinct":
        idx = _uniform_distinct(spec)
    else:
        idx = _zipf(spec)
    scale = float(spec.rank) ** (-1.0 / (2 * spec.nmodes))
    P = [(normal(spec.seed, SID_FACTOR + w, I * spec.rank) * scale).astype(np.float32)
         .reshape(I, spec.rank) for w, I in enumerate(dims)]
    noise = normal(spec.seed, SID_NOISE, spec.nnz) * spec.noise_sd
    return dims, idx, P, noise


def planted_start(spec: TensorSpec, P: Sequence[np.ndarray], sd: float = 0.1) -> List[np.ndarray]:
    """Starting point of a fit: the planted factors plus N(0, sd^2) entries."""
    return [(P[w].astype(np.float64) + sd * normal(spec.seed, SID_START + w, P[w].size)
             .reshape(P[w].shape)).astype(np.float32) for w in range(len(P))]


def make_factors(spec: TensorSpec, rank: Optional[int] = None) -> List[np.ndarray]:
    """Row-major I_w x R FP32 factor matrices with N(0, 1) entries."""
    R = spec.rank if rank is None else rank
    out = []
    for w, I in enumerate(spec.dims):
        out.append(normal(spec.seed, SID_FACTOR + w, I * R).astype(np.float32).reshape(I, R))
    return out


def random_coo(dims: Sequence[int], nnz: int, seed: int, dist: str = "uniform",
               zipf_s: float = 1.1) -> Tuple[np.ndarray, np.ndarray]:
    """Small COO tensors for tests: duplicates allowed (not distinct)."""
    idx = np.empty((len(dims), nnz), dtype=np.int32)
    for d, I in enumerate(dims):
        if dist == "zipf":
            k = zipf_ranks(seed, d, nnz, I, zipf_s)
            idx[d] = permutation(seed, SID_PERM + d, I)[k].astype(np.int32)
        else:
            idx[d] = (raw_u64(seed, d, nnz) % np.uint64(I)).astype(np.int32)
    val = (uniform01(seed, SID_VALUES, nnz) * 2.0 - 1.0).astype(np.float32)
    return idx, val


def random_factors(dims: Sequence[int], rank: int, seed: int) -> List[np.ndarray]:
    return [normal(seed, SID_FACTOR + w, I * rank).astype(np.float32).reshape(I, rank)
            for w, I in enumerate(dims)]
