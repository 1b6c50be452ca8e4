"""Gradient CP fit on the GPU: forward (model at every nonzero) and the
hand-written adjoint (spMTTKRP of the residuals) against the FP64 oracle,
and the autograd.Function that wraps them.

Element bound of a gradient entry.  The forward kernel forms each residual
r_e = m_e - x_e in FP32 from R products of N factors: it errs by at most
(R + N + 1) u (m_abs_e + |x_e|), m_abs_e = sum_r prod_w |Y_w(i_w(e), r)|,
u = 2^-24.  The adjoint then sums the terms r_e prod_{w != d} Y_w like any
spMTTKRP.  So each gradient element must lie within
    1e-5 * MTTKRP(|r|, |Y|) + (R + N + 1) u * MTTKRP(m_abs + |x|, |Y|)
of the oracle's (r and m_abs from the oracle in FP64).
"""
import numpy as np
import pytest

import oracle
from paper_2405_08470_amd import synth
from parity import check_grad_elements

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)
S = pytest.importorskip("paper_2405_08470_amd.spmttkrp")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dims,nnz,R,dist,copies", [
    ((2000, 2000, 1000, 50), 300_000, 16, "uniform", 0),
    ((3000, 2500, 40_000), 300_000, 32, "zipf", 0),
    ((700, 600, 500, 40, 30), 200_000, 16, "zipf", 0),
    ((2000, 2000, 1000, 50), 200_000, 16, "uniform", 1),
])
def test_gradient_matches_oracle(dims, nnz, R, dist, copies):
    print("case", dims, nnz, R, dist, copies, flush=True)
    idx, val = synth.random_coo(dims, nnz, seed=61, dist=dist)
    Y = [0.5 * y for y in synth.random_factors(dims, R, seed=62)]
    t = S.tensor_load_coo(dims, idx, val, copies=copies)
    f = [torch.from_numpy(y).cuda() for y in Y]
    loss, grads = S.cp_gradient(t, f)
    lo, go = oracle.cp_loss_grad(dims, idx, val, Y)
    assert abs(loss.item() - lo) <= 1e-6 * lo
    for d in range(len(dims)):
        e = _rel(grads[d].cpu().numpy(), go[d])
        print(f"  grad {d}: rel {e:.2e}", flush=True)
        assert e <= 1e-5
    w = check_grad_elements(dims, idx, val, Y, [g.cpu().numpy() for g in grads])
    print(f"  max element error / bound {w:.2e}", flush=True)
    # the tensor's own stream is untouched and still in mode 0's order
    assert S.tensor_info(t)["cur_mode"] == 0
    loss2, grads2 = S.cp_gradient(t, f)
    assert loss2.item() == loss.item()
    for a, b in zip(grads, grads2):
        assert torch.equal(a, b)
    t.free()


def test_autograd_function_and_descent():
    dims = (300, 250, 200, 20)
    R = 16
    idx, _ = synth.random_coo(dims, 40_000, seed=71)
    P = [0.6 * y for y in synth.random_factors(dims, R, seed=72)]
    noise = 0.01 * synth.normal(73, 0, idx.shape[1])
    # values: the planted model at the nonzeros (computed here) plus noise
    planted = np.prod([P[w][idx[w]].astype(np.float64) for w in range(len(dims))], axis=0).sum(axis=1)
    val = (planted + noise).astype(np.float32)
    t = S.tensor_load_coo(dims, idx, val)
    start = [torch.from_numpy(p + 0.05 * synth.random_factors(dims, R, seed=74)[w]).cuda()
             for w, p in enumerate(P)]
    params = [torch.nn.Parameter(s.clone()) for s in start]
    loss = S.cp_fit_loss(t, params)
    loss.backward()
    lo, go = oracle.cp_loss_grad(dims, idx, val, [s.cpu().numpy() for s in start])
    for p, g in zip(params, go):
        assert _rel(p.grad.cpu().numpy(), g) <= 1e-5
    check_grad_elements(dims, idx, val, [s.cpu().numpy() for s in start],
                        [p.grad.cpu().numpy() for p in params])
    opt = torch.optim.Adam(params, lr=2e-3)
    first = None
    for it in range(60):
        opt.zero_grad()
        loss = S.cp_fit_loss(t, params)
        if first is None:
            first = loss.item()
        loss.backward()
        opt.step()
    assert loss.item() < 0.5 * first
    t.free()


def test_loss_alone_launches_no_adjoint_and_backward_matches_gradient():
    dims = (400, 300, 200, 30)
    R = 16
    idx, val = synth.random_coo(dims, 60_000, seed=81)
    Y = [0.5 * y for y in synth.random_factors(dims, R, seed=82)]
    t = S.tensor_load_coo(dims, idx, val)
    N = len(dims)
    params = [torch.nn.Parameter(torch.from_numpy(y).cuda()) for y in Y]
    # forward only: the model-at-nonzeros kernel, no spMTTKRP launch
    S.timing_control(t, True, want=False)
    with torch.no_grad():
        loss0 = S.cp_fit_loss(t, params)
    tm = S.timing_control(t, True)
    assert tm["calls"] == [0] * N, tm["calls"]
    loss = S.cp_fit_loss(t, params)
    tm = S.timing_control(t, True)
    assert tm["calls"] == [0] * N, tm["calls"]
    loss.backward()
    tm = S.timing_control(t, False)
    assert tm["calls"] == [1] * N, tm["calls"]
    # the same bits as the one-call gradient
    lref, gref = S.cp_gradient(t, [p.detach() for p in params])
    assert loss.item() == lref.item() == loss0.item()
    for p, g in zip(params, gref):
        assert torch.equal(p.grad, g)
    # a second forward on other factors before the first backward: the
    # backward re-forms its own residuals first
    for p in params:
        p.grad = None
    la = S.cp_fit_loss(t, params)
    other = [torch.from_numpy(0.3 * y).cuda() for y in Y]
    S.cp_loss(t, other)
    la.backward()
    for p, g in zip(params, gref):
        assert torch.equal(p.grad, g)
    t.free()
