"""The MR-DINO surrogate kernels at the full evaluation size, N = 65536
samples (r_m 100, d_Z 25, width 256, depth 4, r_u 200; Sec. 3.3, eq. (rbnet)),
in the tile shape the autotuner picks for that size, against the FP64 oracle
with the same float32-rounded weights on every 256th sample and the last one.

Tolerances are those of the 1000-sample test (tests/test_gpu_mrdino.py, with
their derivation from the operand roundings): FP32 1e-5 on q and 1e-4 on
dq/dz; BF16 2e-3 on q and 4e-2 on dq/dz (1e-2 for the median); FP8 5e-2 and
0.6 (0.15 median), guards of a path with no accuracy target."""
import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa
import saa_inputs as si
from oracle import surrogate, training

pytestmark = pytest.mark.gpu

R_M, D_Z, R_U, N = 100, 25, 200, 65536


@pytest.fixture(scope="module")
def full(gpu_lib):
    prob = saa.problem_medium()
    xi = si.kl_coefficients(4101, N, prob.kl_per_dim)
    z = si.control(4102)
    widths = [R_M + D_Z, 256, 256, 256, 256, R_U]
    layers = si.random_mlp(4103, widths, bias_scale=0.1)
    flat32 = training.flatten(layers).astype(np.float32)
    layers64 = training.unflatten(flat32.astype(np.float64), widths)
    c = 0.3 * np.random.default_rng(4104).standard_normal(R_U)
    model = saa.Model(R_M, D_Z, R_U, 256, 4)
    model.set_params(flat32)
    model.set_qoi(c, 0.05)
    ctx = saa.Context(prob, N)
    ctx.set_samples(torch.from_numpy(xi).cuda())
    idx = np.append(np.arange(0, N, 256), N - 1)
    ref_model = surrogate.Surrogate(layers64, R_M, D_Z, c.astype(np.float32).astype(np.float64), 0.05)
    q_ref, g_ref = surrogate.qoi_and_grad(ref_model, surrogate.encode(xi[idx], R_M), z)
    yield ctx, model, z, idx, q_ref, g_ref
    ctx.close()
    model.close()


@pytest.mark.parametrize("prec,tol_q,tol_g", [(saa.FP32, 1e-5, 1e-4), (saa.BF16, 2e-3, 4e-2), (saa.FP8, 5e-2, 6e-1)])
def test_full_size_sampled_outputs(full, prec, tol_q, tol_g):
    ctx, model, z, idx, q_ref, g_ref = full
    print(f"case mrdino full size N={N} prec={prec}", flush=True)
    q, g, _ = ctx.per_sample(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=prec))
    q, g = q.cpu().numpy(), g.cpu().numpy()
    assert q.shape == (N,) and g.shape == (N, D_Z) and np.isfinite(q).all() and np.isfinite(g).all()
    eq = np.abs(q[idx] - q_ref) / np.abs(q_ref)
    eg = np.linalg.norm(g[idx] - g_ref, axis=1) / np.linalg.norm(g_ref, axis=1)
    print(f"  q rel max {eq.max():.3e}; g rel max {eg.max():.3e} median {np.median(eg):.3e}")
    assert eq.max() <= tol_q
    assert np.median(eg) <= tol_g / 4 and eg.max() <= tol_g
    # a second call (the tile shape now comes from the tuning cache) gives the same values
    q2, g2, _ = ctx.per_sample(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=prec))
    assert np.array_equal(q2.cpu().numpy(), q) and np.array_equal(g2.cpu().numpy(), g)
