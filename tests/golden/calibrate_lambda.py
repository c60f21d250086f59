"""Calibrate the temperature lambda of the workloads whose lambda is not given.

For each workload: run one oracle iteration (seed 0, iteration 0, from the workload's
initial state and nominal sequence), then bisect lambda so that the effective sample
size 1 / sum w^2 of the normalised weights is 5 % of K, rounded to two significant
digits.  Calls only the oracle.  Usage: python tests/golden/calibrate_lambda.py
"""
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))
import workloads as W  # noqa: E402
from oracle import mppi  # noqa: E402


def ess_fraction(S, lam):
    S = S[np.isfinite(S)]
    e = np.exp(-(S - S.min()) / lam)
    w = e / e.sum()
    return 1.0 / np.sum(w * w) / S.size


def calibrate(wl, target=0.05):
    r = mppi.iteration(wl, wl.x0, mppi.initial_sequence(wl), 0)
    lo, hi = 1e-3, 1e6
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if ess_fraction(r.S, mid) < target:
            lo = mid
        else:
            hi = mid
    lam = 0.5 * (lo + hi)
    digits = 2 - int(math.floor(math.log10(lam))) - 1
    return round(lam, digits)


if __name__ == "__main__":
    print("bicycle", calibrate(W.bicycle()))
    for nu in (1.0, 2.0, 4.0):
        print("quadrotor nu", nu, calibrate(W.quadrotor(nu=nu)))
