"""Write pde2d_n128_N1024.json: oracle q_i and dq_i/dz for every sample of
the 2D PDE-form workload (P1 on 128 x 128 cells, 16 x 16 KL modes, 25
sources of width 0.05, constant target 0.5, r = 1; KL coefficients from seed
2306 for N = 1024 and the control from seed 101), by the oracle's Newton
with sparse LU and its adjoint.  Calls only the oracle; run from the
repository root (about a minute on 8 cores):

    python tests/golden/make_pde2d_n128.py
"""
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import saa_inputs as si  # noqa: E402
from oracle import fem2d, saa  # noqa: E402

N = 1024


def main():
    prob = fem2d.Problem2D(n=128, kl_per_dim=16, target=fem2d.TARGET_CONST, u_target=0.5)
    xi = si.kl_coefficients(si.SEED_XI_MEDIUM, N, prob.kl_per_dim)
    z = si.control(si.SEED_Z_EVAL[0])
    t = time.time()
    q, g = saa.per_sample_parallel(prob, xi, z, workers=min(16, os.cpu_count() or 1))
    print(f"{N} samples in {time.time() - t:.1f} s", flush=True)
    out = {"n": prob.n, "N": N, "kl_per_dim": prob.kl_per_dim, "target": "const", "u_target": prob.u_target,
           "seed_xi": si.SEED_XI_MEDIUM, "seed_z": si.SEED_Z_EVAL[0],
           "q": [float(v) for v in q], "g": [[float(v) for v in row] for row in g]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pde2d_n128_N1024.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
