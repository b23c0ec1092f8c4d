"""Write tests/golden/cnn_root0.npz: FP64 oracle full-CROWN bounds for input 0 of the
3x32x32 CNN workload (eps = 2/255), used by the full-size GPU parity tests.

Calls only the oracle and the seeded workload generator (no GPU code).  Takes about
five minutes of CPU time.  Stored: lo, hi (all ReLU layers, C-major, float64, with the
rounding allowance), the raw (no allowance) final margin bounds, and the allowance-
free intermediate bounds are not stored (they are recomputed where needed).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import crown as O  # noqa: E402


def main():
    w = W.cnn_cifar(1)
    bounds = O.crown_bounds(w.net, w.x_lo[0], w.x_hi[0], use_slack=True)
    lo = np.concatenate([b[0] for b in bounds])
    hi = np.concatenate([b[1] for b in bounds])
    L = len(w.net)
    lower = O.spec_lower(w.net, L, w.spec[0], bounds, w.x_lo[0], w.x_hi[0])
    upper = -O.spec_lower(w.net, L, -w.spec[0].astype(np.float64), bounds, w.x_lo[0], w.x_hi[0])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cnn_root0.npz")
    np.savez_compressed(out, lo=lo, hi=hi, lower=lower, upper=upper)
    print("wrote", out)


if __name__ == "__main__":
    main()
