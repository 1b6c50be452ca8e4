"""Writes als_fits_full.json: the FP64 oracle's CP-ALS fit after each of the
first 10 sweeps on the full-size 3-mode (80M nonzeros, rank 32) and 5-mode
(50M nonzeros, rank 32) Zipf workloads, started from the workloads' seeded
N(0, 1) factors.

Calls only ``oracle/`` and the input generator.  Run from the repository root:
    python tests/golden/make_als_fits.py
(about 2 minutes per workload on 8 cores).
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2405_08470_amd import synth  # noqa: E402

WORKLOADS = ("zipf3_8e7", "zipf5_5e7")
SWEEPS = 10


def main():
    src = os.path.join(ROOT, "oracle")
    h = hashlib.sha256()
    for f in ("oracle.c", "__init__.py"):
        with open(os.path.join(src, f), "rb") as fh:
            h.update(fh.read())
    out = {"generator": "tests/golden/make_als_fits.py (oracle.cp_als, FP64)",
           "oracle_sha256_16": h.hexdigest()[:16], "sweeps": SWEEPS, "workloads": {}}
    for name in WORKLOADS:
        spec = synth.WORKLOADS[name]
        t0 = time.time()
        dims, idx, val = synth.make_coo(spec)
        Y0 = synth.make_factors(spec)
        _, lam, fits = oracle.cp_als(dims, idx, val, Y0, SWEEPS)
        out["workloads"][name] = {"dims": list(dims), "nnz": spec.nnz, "rank": spec.rank,
                                  "fits": [float(f) for f in fits],
                                  "lambda_last": [float(x) for x in lam]}
        print(f"{name}: fits {['%.9f' % f for f in fits]} ({time.time() - t0:.0f} s)", flush=True)
        del idx, val
    with open(os.path.join(HERE, "als_fits_full.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
