#!/usr/bin/env python3
"""All-mode spMTTKRP with dynamic remapping inside CP-ALS on one MI355X.

Workload (default): the 3-mode Zipf tensor 100000 x 80000 x 2000000 with 80M
nonzeros (indices Zipf(1.1) per mode, shuffled), FP32 values U(0,1), rank 32
FP32 factors N(0,1) -- synthetic, seeded, shaped like the paper's 3-mode
recommender / knowledge-base tensors.

Phases (inputs resident in HBM before any timed region):
  A  all-mode spMTTKRP with dynamic remapping (mode 0 -> 1 -> 2 -> 0), each
     mode's elementwise kernel followed by the remap pass that writes each
     chunk of 4096 consecutive records in destination order: K timed
     passes -> `value` (ms per all-mode pass) and per-kernel event times;
     then the same passes with the remap fused into the elementwise kernel
     (every record stored at its next position from inside it);
  B  CP-ALS sweeps (A's work plus the FP64 normal-equation update of every
     factor): K timed steps -> `ms_per_step`;
  C  the same spMTTKRP on one mode-ordered copy per mode (no remapping) ->
     the remapping share of A (the paper's breakdown experiment, Sec. 5.2);
  D  A's passes with BF16 factor storage and gathers (FP32 accumulation);
  E  the 4-mode 50000 x 50000 x 20000 x 1000 Zipf(1.1) tensor, 1e8 nonzeros,
     rank 64: all-mode passes with FP32 and with BF16 factors, and the
     relative difference of their outputs per mode;
  F  the 4-mode 20000 x 20000 x 10000 x 500 tensor of 5e7 distinct uniform
     entries of a planted rank-16 model plus N(0, 0.01^2) noise: the gradient
     of the least-squares fit over the nonzeros (forward model at the
     nonzeros + adjoint spMTTKRP of the residuals), timed beside the plain
     FP32 all-mode spMTTKRP of the same tensor;
  the FP64 oracle on a bounded sample of the A tensor on the host cores.
Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "all-modes spMTTKRP ms/iter + HBM GB/s vs peak; bf16 vs fp32 at stated rel err"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


CSRC = "paper_2405_08470_amd/csrc/"
# kernel family -> (committed counter summary, sources the kernel is built from)
TRAFFIC = {
    "ec_kernel": ("ec_kernel_zipf3_8e7_traffic.txt", (CSRC + "ec_kernel.hip", CSRC + "kernels.hpp")),
    "remap_flat_kernel": ("remap_flat_kernel_zipf3_8e7_traffic.txt",
                            (CSRC + "dr_staged.hip", CSRC + "kernels.hpp")),
}


def kernel_source_hash(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, kappa):
    """HBM-side bytes per launch of the kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, scaled by what the counters
    read for a plain copy of known size), or None when the summary is missing
    or was taken on other kernel sources or another partition count."""
    fam = kernel.split("<")[0]
    if fam not in TRAFFIC:
        return None
    fname, sources = TRAFFIC[fam]
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    vals = dict(l.split("=", 1) for l in lines if "=" in l and not l.startswith("#"))
    if (vals.get("kernel_source_sha256_16") != kernel_source_hash(sources) or vals.get("kernel") != kernel
            or vals.get("kappa") != str(kappa)):
        return None
    return float(vals["bytes_per_launch"])


def algorithmic_bytes(dims, nnz, R, rec_bytes, mode, remap):
    """Bytes one launch of the mode's kernel must move: stream the records in
    (and, when remapping, their next positions and the records out), read each
    input factor once and write the output once."""
    per_nnz = rec_bytes + (4 + rec_bytes if remap else 0)
    fac = sum(dims[w] for w in range(len(dims)) if w != mode) * R * 4
    return nnz * per_nnz + fac + dims[mode] * R * 4


def remap_bytes(nnz, rec_bytes):
    """Bytes the remap of one mode must move: read each record and its next
    position, write the record."""
    return nnz * (2 * rec_bytes + 4)


def copy_bandwidth(torch, gib=4.0, reps=10):
    n = int(gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def cpu_baseline(dims, idx, val, factors, budget_s):
    """The oracle (plain FP64 COO loop, one thread) on the first S nonzeros
    for every mode, scaled linearly to the whole tensor."""
    import oracle
    N = len(dims)
    f64 = [np.asarray(f, dtype=np.float64) for f in factors]
    nnz = idx.shape[1]
    probe = min(nnz, 500_000)
    t0 = time.perf_counter()
    for d in range(N):
        oracle.mttkrp(dims, idx[:, :probe], val[:probe], f64, d)
    tp = time.perf_counter() - t0
    S = int(min(nnz, max(probe, probe * budget_s / max(tp, 1e-6))))
    t0 = time.perf_counter()
    for d in range(N):
        oracle.mttkrp(dims, idx[:, :S], val[:S], f64, d)
    ts = time.perf_counter() - t0
    return ts * 1e3 * nnz / S, S, ts


def timed_passes(torch, S, t, K, W, fn):
    """W untimed, then K timed calls of fn(); wall ms per call and the
    library's per-mode kernel-event totals over the timed calls."""
    for _ in range(W):
        fn()
    torch.cuda.synchronize()
    S.timing_control(t, True, want=False)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(K):
        fn()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) * 1e3 / K
    tm = S.timing_control(t, False)
    return wall, tm


def per_call(tm, key, N):
    return [tm[key][d] / max(1, tm["calls"][d]) for d in range(N)]


def phase_bf16_wide(torch, S, synth, K, W):
    """Phase E: FP32 against BF16 factors on the 4-mode rank-64 workload."""
    spec = synth.WORKLOADS["zipf4_1e8"]
    t0 = time.perf_counter()
    dims, idx, val = synth.make_coo(spec)
    Y = synth.make_factors(spec)
    log(f"phase E: generated {spec.name} in {time.perf_counter() - t0:.1f}s")
    N, R = len(dims), spec.rank
    t = S.tensor_load_coo(dims, idx, val, prep="device")
    del idx, val
    info = S.tensor_info(t)
    f32 = [torch.from_numpy(y).cuda() for y in Y]
    fbf = [f.to(torch.bfloat16) for f in f32]
    outs = [torch.empty((dims[d], R), dtype=torch.float32, device="cuda") for d in range(N)]
    res = {}
    keep = []
    for name, fac in (("fp32", f32), ("bf16", fbf)):
        def run(fac=fac):
            for d in range(N):
                S.mttkrp(t, d, fac, outs[d], flags=S.FUSE_REMAP_NEXT)
        wall, tm = timed_passes(torch, S, t, K, W, run)
        ec, rm = per_call(tm, "ec_ms", N), per_call(tm, "remap_ms", N)
        res[name] = {"ms_per_pass": round(wall, 4), "ec_kernel_ms": [round(x, 4) for x in ec],
                     "remap_kernel_ms": [round(x, 4) for x in rm]}
        keep.append([o.clone() for o in outs])
        log(f"phase E {name}: {wall:.3f} ms per all-mode pass; EC {['%.3f' % x for x in ec]} ms, "
            f"remap {['%.3f' % x for x in rm]} ms")
    err = [float(torch.linalg.vector_norm(keep[1][d] - keep[0][d]) / torch.linalg.vector_norm(keep[0][d]))
           for d in range(N)]
    log(f"phase E: BF16 vs FP32 factors, rel diff per mode {['%.2e' % e for e in err]}")
    t.free()
    return {"workload": f"{spec.name}: 4-mode {'x'.join(map(str, dims))}, {spec.nnz} nonzeros, "
                        f"Zipf({spec.zipf_s}) shuffled, rank {R}",
            "kappa": info["kappa"], **res,
            "bf16_rel_diff_vs_fp32": [float("%.3g" % e) for e in err],
            "speedup_bf16": round(res["fp32"]["ms_per_pass"] / res["bf16"]["ms_per_pass"], 3)}


def planted_values(idx, P, noise):
    """x_e = sum_r prod_w P_w(i_w(e), r) + noise_e (the planted workload's
    observed values), evaluated here in chunks, FP64 then rounded to FP32."""
    nnz = idx.shape[1]
    out = np.empty(nnz, dtype=np.float32)
    step = 1 << 22
    for a in range(0, nnz, step):
        b = min(nnz, a + step)
        p = np.ones((b - a, P[0].shape[1]), dtype=np.float64)
        for w in range(len(P)):
            p *= P[w][idx[w, a:b]]
        out[a:b] = (p.sum(axis=1) + noise[a:b]).astype(np.float32)
    return out


def phase_gradient(torch, S, synth, K, W):
    """Phase F: gradient of the CP fit over the nonzeros vs plain spMTTKRP."""
    spec = synth.WORKLOADS["planted4_5e7"]
    t0 = time.perf_counter()
    dims, idx, P, noise = synth.planted_parts(spec)
    val = planted_values(idx, P, noise)
    start = synth.planted_start(spec, P)
    log(f"phase F: generated {spec.name} in {time.perf_counter() - t0:.1f}s")
    N, R = len(dims), spec.rank
    t = S.tensor_load_coo(dims, idx, val, prep="device")
    del idx, val
    info = S.tensor_info(t)
    fac = [torch.from_numpy(y).cuda() for y in start]
    grads = [torch.empty_like(f) for f in fac]
    outs = [torch.empty((dims[d], R), dtype=torch.float32, device="cuda") for d in range(N)]

    def grad():
        S.cp_gradient(t, fac, grads)

    def plain():
        for d in range(N):
            S.mttkrp(t, d, fac, outs[d], flags=S.FUSE_REMAP_NEXT)

    wall_g, tm_g = timed_passes(torch, S, t, K, W, grad)
    wall_p, tm_p = timed_passes(torch, S, t, K, W, plain)
    loss_start = float(S.cp_gradient(t, fac, grads)[0].item())
    pf = [torch.from_numpy(p).cuda() for p in P]
    loss_planted = float(S.cp_gradient(t, pf, [torch.empty_like(p) for p in pf])[0].item())
    noise_half_ss = 0.5 * float(np.dot(noise, noise))
    t.free()
    log(f"phase F: gradient {wall_g:.3f} ms (forward + {N} adjoint modes); plain FP32 all-mode "
        f"spMTTKRP {wall_p:.3f} ms; loss at start {loss_start:.4g}, at the planted factors "
        f"{loss_planted:.6g} (half the noise sum of squares {noise_half_ss:.6g})")
    return {"workload": f"{spec.name}: 4-mode {'x'.join(map(str, dims))}, {spec.nnz} distinct uniform "
                        f"nonzeros of a planted rank-{R} model + N(0, {spec.noise_sd}^2) noise",
            "kappa": info["kappa"],
            "gradient_ms": round(wall_g, 4),
            "adjoint_ec_kernel_ms": [round(x, 4) for x in per_call(tm_g, "ec_ms", N)],
            "adjoint_remap_kernel_ms": [round(x, 4) for x in per_call(tm_g, "remap_ms", N)],
            "plain_fp32_all_mode_ms": round(wall_p, 4),
            "plain_ec_kernel_ms": [round(x, 4) for x in per_call(tm_p, "ec_ms", N)],
            "plain_remap_kernel_ms": [round(x, 4) for x in per_call(tm_p, "remap_ms", N)],
            "loss_at_start": loss_start, "loss_at_planted": loss_planted,
            "half_noise_sum_sq": noise_half_ss}


def ablation(torch, S, dims, idx, val, fac, outs, K, W, name):
    """The all-mode pass across partition counts kappa (the analog of the
    paper's threadblock-count sweep), with the remap fused into the
    elementwise kernel instead of staged, with the heavy-row split off (pure
    Alg. 1), and, for four modes or more, with each record layout: ms per
    pass, per-mode kernel times, largest partition."""
    N = len(dims)
    rows = []
    settings = [(k, None, "staged", "auto") for k in (2048, 4096, 8192, 16384, 32768, 65536)]
    settings += [(8192, None, "fused", "auto"), (8192, 0, "staged", "auto")]
    if N >= 4:
        # the record layouts (Sec. 3.5) with a kernel for this shape
        small = max(dims) <= 65536
        lays = (["half16"] if small and N != 7 else []) + (["packed"] if N <= 6 else []) + ["word32"]
        settings += [(8192, None, "staged", lay) for lay in lays]
    for kappa, cap, remap, layout in settings:
        t = S.tensor_load_coo(dims, idx, val, kappa=kappa, split_cap=cap, prep="device", remap=remap,
                              layout=layout)
        info = S.tensor_info(t)

        def run(tt=t):
            for d in range(N):
                S.mttkrp(tt, d, fac, outs[d], flags=S.FUSE_REMAP_NEXT)
        kk, ww = (K, W) if cap is None else (1, 0)
        wall, tm = timed_passes(torch, S, t, kk, ww, run)
        ec, rm = per_call(tm, "ec_ms", N), per_call(tm, "remap_ms", N)
        t.free()
        row = {"kappa": kappa, "split": cap is None, "remap": remap, "layout": layout,
               "record_bytes": info["record_bytes"], "ms_per_pass": round(wall, 4),
               "ec_kernel_ms": [round(x, 4) for x in ec], "remap_kernel_ms": [round(x, 4) for x in rm],
               "max_partition": info["max_load"], "mean_partition": round(len(val) / kappa, 1)}
        log(f"ablation {row}")
        rows.append(row)
    return {"ablation": name, "rows": rows}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="zipf3_8e7",
                    help="uniform3_1e5, zipf3_8e7 (default), zipf5_5e7 or zipf4_1e8")
    ap.add_argument("--nnz", type=int, default=None, help="override the nonzero count")
    ap.add_argument("--kappa", type=int, default=0)
    ap.add_argument("--no-ec-only", action="store_true", help="skip phase C")
    ap.add_argument("--no-fused", action="store_true", help="skip the fused-remap passes of phase A")
    ap.add_argument("--no-als", action="store_true", help="skip phase B")
    ap.add_argument("--no-bf16", action="store_true", help="skip phase D")
    ap.add_argument("--no-wide", action="store_true", help="skip phases E and F")
    ap.add_argument("--no-host-prep", action="store_true", help="skip the host-planner load timing")
    ap.add_argument("--prep", choices=("device", "host"), default="device",
                    help="planner of the timed tensors (default: device)")
    ap.add_argument("--ablation", action="store_true",
                    help="instead of the benchmark line: the all-mode pass across kappa, with the "
                         "remap fused, and with the heavy-row split off (one JSON line)")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the multi-GPU sharding of this path is a design "
              "(see the design notes), not built", file=sys.stderr)
        return 2

    import torch
    from paper_2405_08470_amd import synth
    import paper_2405_08470_amd.spmttkrp as S

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    spec = synth.WORKLOADS[args.workload]
    if args.nnz:
        spec = synth.scaled(spec, args.nnz)
    K, W = args.steps, args.warmup
    R = spec.rank
    t0 = time.perf_counter()
    dims, idx, val = synth.make_coo(spec)
    Y0 = synth.make_factors(spec)
    log(f"generated {spec.name}: dims {dims} nnz {spec.nnz} R {R} in {time.perf_counter() - t0:.1f}s")
    N = len(dims)

    prep_host = None
    if not args.no_host_prep:
        th = S.tensor_load_coo(dims, idx, val, kappa=args.kappa)
        prep_host = S.tensor_info(th)["prep_seconds"]
        th.free()
        log(f"host planner load: {prep_host:.2f}s")
    t = S.tensor_load_coo(dims, idx, val, kappa=args.kappa, prep=args.prep)
    info = S.tensor_info(t)
    log(f"loaded ({args.prep} planner): kappa {info['kappa']} record {info['record_bytes']} B prep "
        f"{info['prep_seconds']:.2f}s max partition {info['max_load']} split rows {info['split_rows']}")
    fac = [torch.from_numpy(np.ascontiguousarray(y)).cuda() for y in Y0]
    outs = [torch.empty((dims[d], R), dtype=torch.float32, device="cuda") for d in range(N)]
    if args.ablation:
        t.free()
        print(json.dumps(ablation(torch, S, dims, idx, val, fac, outs, K, W, spec.name)), flush=True)
        return 0

    def all_modes(tt, fuse):
        for d in range(N):
            S.mttkrp(tt, d, fac, outs[d], flags=S.FUSE_REMAP_NEXT if fuse else 0)

    # ---- phase A: all-mode spMTTKRP with dynamic remapping (staged remap pass)
    for _ in range(W):
        all_modes(t, True)
    torch.cuda.synchronize()
    S.timing_control(t, True, want=False)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(K):
        all_modes(t, True)
    torch.cuda.synchronize()
    wall_a = (time.perf_counter() - w0) * 1e3 / K
    tm_a = S.timing_control(t, False)
    ec_ms = per_call(tm_a, "ec_ms", N)
    rm_ms = per_call(tm_a, "remap_ms", N)
    fix_ms = per_call(tm_a, "fixup_ms", N)
    log(f"phase A: {wall_a:.3f} ms per all-mode pass; EC kernel per mode {['%.3f' % x for x in ec_ms]} ms, "
        f"staged remap {['%.3f' % x for x in rm_ms]} ms, fixup {['%.3f' % x for x in fix_ms]} ms")

    # the paper's fused form: every record stored at its next position from
    # inside the elementwise kernel
    fused = None
    if not args.no_fused:
        tf = S.tensor_load_coo(dims, idx, val, kappa=args.kappa, prep=args.prep, remap="fused")

        def fused_pass():
            for d in range(N):
                S.mttkrp(tf, d, fac, outs[d], flags=S.FUSE_REMAP_NEXT)
        wall_f, tm_f = timed_passes(torch, S, tf, K, W, fused_pass)
        tf.free()
        ec_f = per_call(tm_f, "ec_ms", N)
        fused = {"ms_per_pass": round(wall_f, 4), "ec_remap_kernel_ms": [round(x, 4) for x in ec_f]}
        log(f"fused remap: {wall_f:.3f} ms per all-mode pass; EC+remap kernel {['%.3f' % x for x in ec_f]} ms")

    # the remap alone (spt_remap_for_mode, one hop per call: the remap pass
    # without the elementwise kernel), N hops per pass
    def remap_pass():
        for d in range(N):
            S.remap_for_mode(t, (d + 1) % N)
    wall_r, _ = timed_passes(torch, S, t, K, W, remap_pass)
    log(f"remap alone: {wall_r:.3f} ms per pass of {N} one-hop remaps")

    rec = info["record_bytes"]
    bytes_ec = [algorithmic_bytes(dims, spec.nnz, R, rec, d, False) for d in range(N)]
    bytes_rm = remap_bytes(spec.nnz, rec)
    # the whole step of one mode: elementwise kernel + remap
    bytes_a = [b + bytes_rm for b in bytes_ec]
    pass_gbps = sum(bytes_a) / ((sum(ec_ms) + sum(rm_ms)) * 1e-3) / 1e9
    canon = 4 * (2 * N + 1)
    bytes_canon = [spec.nnz * 2 * canon + sum(dims[w] for w in range(N) if w != d) * R * 4 + dims[d] * R * 4
                   for d in range(N)]
    # the dominant kernel of the pass and its roofline
    if sum(rm_ms) > sum(ec_ms):
        kernel = f"remap_flat_kernel<{rec // 4},{S.stage_chunk(rec)}>"
        dom_bytes, dom_ms = bytes_rm, sum(rm_ms) / N
    else:
        kernel = f"ec_kernel<{N},{R},{rec // 4}>"
        dom_bytes, dom_ms = sum(bytes_ec) / N, sum(ec_ms) / N
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9

    # ---- phase D: the same passes with BF16 factor gathers (FP32 accumulation)
    bf16 = None
    if not args.no_bf16:
        ref = [o.clone() for o in outs]          # FP32-gather results of phase A
        fac32 = fac
        fac = [f.to(torch.bfloat16) for f in fac32]
        for _ in range(W):
            all_modes(t, True)
        torch.cuda.synchronize()
        S.timing_control(t, True, want=False)
        w0 = time.perf_counter()
        for _ in range(K):
            all_modes(t, True)
        torch.cuda.synchronize()
        wall_d = (time.perf_counter() - w0) * 1e3 / K
        tm_d = S.timing_control(t, False)
        ec_d, rm_d = per_call(tm_d, "ec_ms", N), per_call(tm_d, "remap_ms", N)
        err = [float(torch.linalg.vector_norm(outs[d] - ref[d]) / torch.linalg.vector_norm(ref[d]))
               for d in range(N)]
        bytes_d = [b - (sum(dims[w] for w in range(N) if w != d) * R * 2) for d, b in enumerate(bytes_ec)]
        bf16 = {"ms_per_pass": round(wall_d, 4), "ec_kernel_ms": [round(x, 4) for x in ec_d],
                "remap_kernel_ms": [round(x, 4) for x in rm_d],
                "rel_err_vs_fp32_gather": [float("%.3g" % e) for e in err],
                "ec_kernel_GBps": round(sum(bytes_d) / (sum(ec_d) * 1e-3) / 1e9, 1)}
        fac = fac32
        del ref
        log(f"phase D: BF16 gathers {wall_d:.3f} ms per all-mode pass; EC "
            f"{['%.3f' % x for x in ec_d]} ms; rel err vs FP32 gathers {['%.2e' % e for e in err]}")

    # ---- phase B: CP-ALS sweeps
    ms_step = None
    als_ms = None
    fit = None
    if not args.no_als:
        lam = torch.empty(R, dtype=torch.float64, device="cuda")
        for _ in range(W):
            S.cp_als_iter(t, fac, lam, want_fit=False)
        torch.cuda.synchronize()
        S.timing_control(t, True, want=False)
        w0 = time.perf_counter()
        for _ in range(K):
            S.cp_als_iter(t, fac, lam, want_fit=False)
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - w0) * 1e3 / K
        tm_b = S.timing_control(t, False)
        als_ms = sum(tm_b["als_ms"]) / K
        fit = S.cp_als_iter(t, fac, lam, want_fit=True)
        log(f"phase B: {ms_step:.3f} ms per CP-ALS sweep (dense FP64 step {als_ms:.3f} ms, beside the remap "
            f"pass on a side stream); fit after "
            f"{W + K + 1} sweeps {fit:.6f}")
    t.free()

    # ---- phase C: one mode-ordered copy per mode, no remapping
    ec_only = None
    ec_only_kernel = None
    if not args.no_ec_only:
        tc = S.tensor_load_coo(dims, idx, val, kappa=args.kappa, copies=1, prep=args.prep)
        for _ in range(W):
            all_modes(tc, False)
        torch.cuda.synchronize()
        S.timing_control(tc, True, want=False)
        w0 = time.perf_counter()
        for _ in range(K):
            all_modes(tc, False)
        torch.cuda.synchronize()
        ec_only = (time.perf_counter() - w0) * 1e3 / K
        tm_c = S.timing_control(tc, False)
        ec_only_kernel = [tm_c["ec_ms"][d] / max(1, tm_c["calls"][d]) for d in range(N)]
        tc.free()
        log(f"phase C: {ec_only:.3f} ms per all-mode pass without remapping; kernels "
            f"{['%.3f' % x for x in ec_only_kernel]} ms")

    copy_gbps = copy_bandwidth(torch)
    log(f"plain copy (torch) {copy_gbps:.0f} GB/s")

    cpu = None
    if args.cpu_budget > 0:
        ms_full, S_n, ts = cpu_baseline(dims, idx, val, Y0, args.cpu_budget)
        cpu = {"value": round(ms_full, 3), "unit": "ms/iter", "cores": 1, "kind": "oracle",
               "sample": f"first {S_n} of {spec.nnz} nonzeros, all {N} modes, FP64 COO loop "
                         f"({ts:.1f} s), scaled linearly to the whole tensor"}
        log(f"cpu oracle: {ms_full:.0f} ms per all-mode pass (extrapolated from {S_n} nonzeros)")

    wide_bf16 = wide_grad = None
    if not args.no_wide:
        del idx, val
        wide_bf16 = phase_bf16_wide(torch, S, synth, K, W)
        wide_grad = phase_gradient(torch, S, synth, K, W)

    traffic = measured_traffic(kernel, info["kappa"])
    line = {
        "metric": METRIC,
        "value": round(wall_a, 4),
        "unit": "ms/iter",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_step, 4) if ms_step is not None else round(wall_a, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{spec.name}: {N}-mode {'x'.join(map(str, dims))}, {spec.nnz} nonzeros, "
                        f"{spec.dist}" + (f"({spec.zipf_s}) shuffled" if spec.dist == "zipf" else "")
                        + f" indices, {spec.values} values, rank {R} FP32 factors",
            "dims": list(dims), "nnz": spec.nnz, "rank": R, "kappa": info["kappa"],
            "record_bytes": rec, "step": "one CP-ALS sweep (all modes: spMTTKRP + remap + FP64 update)",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": round(traffic) if traffic is not None else None, "kernel": kernel,
            "bytes_per_launch": int(dom_bytes), "avg_launch_ms": round(dom_ms, 4),
        },
        "cpu_baseline": cpu,
        "breakdown": {
            "ec_kernel_ms": [round(x, 4) for x in ec_ms],
            "remap_kernel_ms": [round(x, 4) for x in rm_ms],
            "fixup_ms": [round(x, 4) for x in fix_ms],
            "pass_GBps": round(pass_gbps, 1),
            "pass_frac": round(pass_gbps / HBM_PEAK_GBPS, 4),
            "fused_remap": fused,
            "als_dense_ms_per_sweep": round(als_ms, 4) if als_ms is not None else None,
            "als_dense_overlaps_remap": True,
            "ec_only_ms_per_pass": round(ec_only, 4) if ec_only is not None else None,
            "ec_only_kernel_ms": [round(x, 4) for x in ec_only_kernel] if ec_only_kernel else None,
            "remap_share": round(1 - ec_only / wall_a, 4) if ec_only is not None else None,
            "remap_alone_ms_per_pass": round(wall_r, 4),
            "canonical_record_GBps": round(sum(bytes_canon) / ((sum(ec_ms) + sum(rm_ms)) * 1e-3) / 1e9, 1),
            "fit": fit,
            "bf16_gather": bf16,
            "bf16_rank64_4mode": wide_bf16,
            "gradient_rank16_4mode": wide_grad,
            f"prep_seconds_{args.prep}_planner": round(info["prep_seconds"], 3),
            "prep_seconds_host_planner": round(prep_host, 3) if prep_host is not None else None,
            "copy_GBps": round(copy_gbps, 1),
            "split_rows": info["split_rows"],
            "max_partition": info["max_load"],
        },
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
