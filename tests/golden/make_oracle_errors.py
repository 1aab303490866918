"""Writes tests/golden/oracle_errors_lowrank1e5s.json: the FP64 oracle's relative Frobenius error
(Section 5's metric) of its own sketch of the scaled-signal low-rank workload (1e5 x 2e4, rank 200,
s_i = sqrt(mn)/i, noise 1e-3; k1 = k2 = 200, c = 5), sketch seeds 0, 1, 2, each estimated on the
same 1e7 sampled entries (error seed 1000 + sketch seed) that the benchmark draws for the GPU's
sketches of that workload.  Calls only the oracle and the shared input generators.

    python tests/golden/make_oracle_errors.py [--seeds 0,1,2] [--samples 10000000]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import cabs as oc  # noqa: E402
from oracle.matrices import Matrix  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", default="0,1,2")
    ap.add_argument("--samples", type=int, default=10_000_000)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                   "oracle_errors_lowrank1e5s.json"))
    a = ap.parse_args()
    spec, cfg = workloads.config("lowrank1e5s")
    k, iters = cfg["k"], cfg["iters"]
    rec = {"workload": "lowrank1e5s: 1e5 x 2e4, rank 200, s_i = sqrt(mn)/i, noise 1e-3, k1 = k2 = 200, c = 5",
           "samples": a.samples, "error_seed": "1000 + sketch seed", "seeds": {}}
    for s in [int(x) for x in a.seeds.split(",") if x]:
        t0 = time.perf_counter()
        res = oc.cabs(spec, oc.Params.square(k, kmeans_iters=iters, seed=s))
        ratio, num, den = oc.rel_error_sampled(Matrix(spec), res.C, res.Umid, res.Rt, a.samples, 1000 + s)
        rec["seeds"][str(s)] = {"rel_error": ratio, "sum_sq_residual": num, "sum_sq_entries": den,
                                "oracle_seconds": time.perf_counter() - t0}
        print(f"seed {s}: rel error {ratio:.6g} ({time.perf_counter() - t0:.1f} s)", flush=True)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
