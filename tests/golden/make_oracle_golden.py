"""Writes the stored expected values under tests/golden/.  Calls only oracle/
(and su2_inputs for the workload description); nothing here comes from the
HIP path.

oracle_su2_32x32x32x32_hot.json: the 32^4 periodic lattice, hot start (Haar,
Philox seed 1), beta in {2.2, 2.3, 2.4, 2.5}, 1000 heat-bath sweeps of the
oracle chain (FP64 arithmetic, FP32 link storage); per sweep the plaquette
(P, P_s, P_t) after the sweep, plus the attempt and cap-failure totals.  The
GPU's long-run averages are compared with these within 3 sigma
(autocorrelation-corrected).

Usage: python tests/golden/make_oracle_golden.py [--sweeps N]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import su2_inputs  # noqa: E402


def run(dims, beta, seed, start, sweeps):
    ch = oracle.Chain(dims, beta, seed, start)
    hist = []
    t0 = time.time()
    for i in range(sweeps):
        ch.sweep(1)
        hist.append([round(float(v), 12) for v in ch.plaquette()])
        if (i + 1) % 100 == 0:
            print(f"  beta {beta}: {i + 1} sweeps, P = {hist[-1][0]:.6f}, "
                  f"{time.time() - t0:.0f} s", flush=True)
    return dict(beta=beta, history=hist, attempts=ch.attempts, failures=ch.failures)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sweeps", type=int, default=None)
    args = ap.parse_args()
    w = su2_inputs.WORKLOADS["su2_32x32x32x32_hot"]
    sweeps = args.sweeps or w["sweeps"]
    out = dict(workload="su2_32x32x32x32_hot", dims=list(w["dims"]), seed=w["seed"],
               start="hot", sweeps=sweeps, prec32=True, threads=oracle.num_threads(), runs=[])
    for beta in w["betas"]:
        out["runs"].append(run(w["dims"], beta, w["seed"], w["start"], sweeps))
        with open(os.path.join(HERE, "oracle_su2_32x32x32x32_hot.json"), "w") as fh:
            json.dump(out, fh, separators=(",", ":"))
    print("done")


if __name__ == "__main__":
    main()
