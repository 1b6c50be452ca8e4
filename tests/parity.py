"""Element-by-element parity bounds shared by the GPU tests.

Every output element of an FP32 spMTTKRP is compared with the FP64 oracle
against the magnitude of the terms it sums:

    |M_gpu(i, r) - M_ref(i, r)| <= GAMMA * M_abs(i, r),
    M_abs(i, r) = sum_{e : i_mode(e) = i} |val_e| prod_{w != mode} |Y_w(i_w(e), r)|

M_abs is the oracle's MTTKRP of |val| and |Y|, so it bounds every partial sum
of the element whatever the summation order; an element with M_abs = 0 (a row
without nonzeros) must be exactly 0.

Why GAMMA = 1e-5, the relative tolerance the path is held to, applied to each
element.  With u = 2^-24, FP32 products of N factors and a sum of the terms
along a chain of m additions (in any order) err by at most gamma_m * M_abs,
gamma_m = m u / (1 - m u) (Higham, Accuracy and Stability of Numerical
Algorithms, Sec. 3.1).  That worst case assumes every rounding error has the
same sign and every partial sum is as large as M_abs.  Modelled as random, the
errors add to about u sqrt(m / 3) M_abs when all terms have one sign (1.2e-6
for a chain of m = 1300) and to about u M_abs when their signs are random, as
with the centred normal factors of every workload here (partial sums grow like
sqrt(k) while M_abs grows like k).  An element beyond 1e-5 M_abs therefore
points to a wrong or missing term, not to rounding.
"""
import numpy as np

import oracle

GAMMA = 1e-5


def mttkrp_abs(dims, idx, val, factors, mode, rows=None):
    """M_abs of the listed rows (all rows if None)."""
    av = np.abs(np.asarray(val, dtype=np.float64))
    af = [np.abs(np.asarray(f, dtype=np.float64)) for f in factors]
    if rows is None:
        return oracle.mttkrp(dims, idx, av, af, mode)
    return oracle.mttkrp_rows(dims, idx, av, af, mode, rows)


def elementwise_ratio(got, ref, absref):
    """max over elements of |got - ref| / absref (inf where absref = 0 and
    got != 0)."""
    got = np.asarray(got, dtype=np.float64)
    diff = np.abs(got - ref)
    zero = absref == 0
    if np.any(diff[zero] != 0):
        return float("inf")
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(zero, 0.0, diff / np.where(zero, 1.0, absref))
    return float(r.max()) if r.size else 0.0


def check_elementwise(got, ref, absref, gamma=GAMMA, label=""):
    ratio = elementwise_ratio(got, ref, absref)
    assert ratio <= gamma, f"{label}: max |gpu - oracle| / M_abs = {ratio:.3e} > {gamma:.1e}"
    return ratio


def rel_fro(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def degree_spectrum_rows(col, I, count, seed):
    """About `count` output rows across the degree spectrum of one mode: the
    hottest rows, rows at log-spaced degree ranks, random non-empty rows,
    empty rows, and the first and last row."""
    deg = np.bincount(col, minlength=I)
    order = np.argsort(-deg, kind="stable")
    nonempty = int(np.count_nonzero(deg))
    rng = np.random.default_rng(seed)
    rows = set(int(r) for r in order[:8])
    ranks = np.unique(np.geomspace(1, max(nonempty, 1), num=count // 2).astype(np.int64) - 1)
    rows.update(int(order[k]) for k in ranks if k < nonempty)
    ne = np.flatnonzero(deg)
    rows.update(int(r) for r in rng.choice(ne, min(ne.size, count // 4), replace=False))
    empty = np.flatnonzero(deg == 0)
    rows.update(int(r) for r in empty[:4])
    rows.update((0, I - 1))
    return sorted(rows)


def check_grad_elements(dims, idx, val, Y, grads):
    """Every element of the gradient of 1/2 sum (x - m)^2 within

        1e-5 * MTTKRP(|r|, |Y|) + (R + N + 1) u * MTTKRP(m_abs + |x|, |Y|)

    of the oracle's, where r = m - x and m_abs_e = sum_r prod_w |Y_w(i_w(e), r)|
    come from the oracle in FP64.  The second term covers the FP32 residual
    of the forward pass: R products of N factors summed and x subtracted err by
    at most (R + N + 1) u (m_abs_e + |x_e|) per nonzero; the first term the
    adjoint's own sum, as for any spMTTKRP.  Returns the largest ratio of the
    error to the bound."""
    N, R = len(dims), Y[0].shape[1]
    m = oracle.model_at(idx, Y)
    r = m - np.asarray(val, dtype=np.float64)
    aY = [np.abs(np.asarray(y, dtype=np.float64)) for y in Y]
    m_abs = oracle.model_at(idx, aY)
    side = m_abs + np.abs(np.asarray(val, dtype=np.float64))
    u = 2.0 ** -24
    worst = 0.0
    for d in range(N):
        ref = oracle.mttkrp(dims, idx, r, Y, d)
        bound = GAMMA * oracle.mttkrp(dims, idx, np.abs(r), aY, d) + \
            (R + N + 1) * u * oracle.mttkrp(dims, idx, side, aY, d)
        ratio = elementwise_ratio(grads[d], ref, bound)
        assert ratio <= 1.0, f"gradient {d}: max |gpu - oracle| / bound = {ratio:.3e}"
        worst = max(worst, ratio)
    return worst
