"""Write pde3d_n48_samples.json: oracle q_i and dq/dz_i for sampled samples
of the 3D workload (Q1 on 48^3, K1 = 10, 64 sources of width 0.08, constant
target 0.5, KL coefficients from seed 2313 for N = 256, control from seed
2314).  The Newton and adjoint linear solves use the oracle's CG stand-in
(relative residual 1e-14): a sparse LU of these 103823-unknown Jacobians
takes hours.  Calls only the oracle; run from the repository root:

    python tests/golden/make_pde3d_n48.py
"""
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import saa_inputs as si  # noqa: E402
from oracle import fem3d  # noqa: E402

N = 256
SAMPLES = [0, 255]


def main():
    prob = fem3d.Problem3D()
    xi = si.kl_coefficients(si.SEED_XI_3D, N, prob.kl_per_dim, dim=3)
    z = si.control(si.SEED_Z_3D, prob.d_z)
    ops = fem3d.operators(prob)
    out = {"n": prob.n, "N": N, "kl_per_dim": prob.kl_per_dim, "n_src_per_dim": prob.n_src_per_dim,
           "src_sigma": prob.src_sigma, "kl_shift": prob.kl_shift, "kl_exp": prob.kl_exp,
           "seed_xi": si.SEED_XI_3D, "seed_z": si.SEED_Z_3D, "samples": {}}
    for i in SAMPLES:
        t = time.time()
        s = fem3d.solve_sample(ops, xi[i], z, linear="cg")
        out["samples"][str(i)] = {"q": s["q"], "g": s["g"].tolist(), "newton_iters": s["newton_iters"]}
        print(f"sample {i}: q {s['q']:.15e}  {time.time() - t:.1f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pde3d_n48_samples.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
