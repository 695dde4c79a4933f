"""Writes the float64 oracle's results for the two large workloads at their
stated sizes, for the full-size GPU parity tests (too slow to recompute in
a test run):

  fullsize_w4.npz  N = 1,048,576 rows x 33 features, 33-256-3 net,
                   minibatches of 4096 rows, lr 0.1, 20 epochs;
  fullsize_w5.npz  the wide 64-1024-3 net on the first 65,536 of its
                   4,194,304 rows, minibatches of 16384 rows, lr 0.1,
                   5 epochs.

Each file holds the trained parameters (theta, packed [W1 | b1 | W2 | b2],
float64) and the per-epoch losses (loss_hist).  Inputs and initial
parameters come from the seeded generator (paper_1908_07847_amd.synth, which
holds none of the method's arithmetic); the training is oracle.train (the
plain float64 loop of section 2.2), nothing else.

Run:  python tests/golden/make_fullsize.py [w4] [w5]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1908_07847_amd import synth  # noqa: E402

CASES = {"w4": dict(workload=4, rows=None, epochs=20), "w5": dict(workload=5, rows=65536, epochs=5)}


def make(name: str) -> str:
    c = CASES[name]
    w = synth.single(c["workload"], n_rows=c["rows"])
    oracle.set_threads(0)
    t0 = time.time()
    q, hist = oracle.train(w["X"], w["T"], oracle.Params.of(w["theta"]), w["lr"], c["epochs"], batch=w["batch"])
    out = os.path.join(HERE, f"fullsize_{name}.npz")
    np.savez(out, theta=q.flat(), loss_hist=hist, rows=w["X"].shape[0], epochs=c["epochs"], batch=w["batch"])
    print(f"{out}: {w['X'].shape[0]} rows, {c['epochs']} epochs, {time.time() - t0:.0f} s; losses {hist}")
    return out


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
