"""GPU parity of the MR-DINO surrogate of the 3D problem (Sec. 3.3, eq.
(rbnet), with the shapes of the 3D workload: r_m = 200 leading KL modes of
the K1^3 sine field, d_Z = 64 controls, width 512, depth 4, r_u = 400)
against the FP64 oracle with the same (float32-rounded) weights.

The fused kernel carries 32 samples per workgroup at width 512; N = 100 is
three full workgroups and a ragged one.  Tolerances as in 2D: FP32 1e-5 on
q (1e-4 on dq/dz), BF16 2e-2 on J and grad J; FP8 is reported with bounds
at about twice the measured errors."""
import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa
import saa_inputs as si
from oracle import cvar, surrogate, training

pytestmark = pytest.mark.gpu

R_M, D_Z, R_U, W = 200, 64, 400, 512


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def setup3(gpu_lib):
    prob = saa.Problem(dim=3, n=8, n_src_per_dim=4, src_sigma=0.08, kl_per_dim=6, kl_shift=25.0, kl_exp=1.5)
    assert prob.d_z == D_Z and prob.kl_per_dim ** 3 >= R_M
    N = 100
    xi = si.kl_coefficients(4301, N, prob.kl_per_dim, dim=3)
    z = si.control(4302, D_Z)
    widths = [R_M + D_Z, W, W, W, W, R_U]
    flat32 = training.flatten(si.random_mlp(4303, widths, bias_scale=0.1)).astype(np.float32)
    layers64 = training.unflatten(flat32.astype(np.float64), widths)
    c = 0.3 * np.random.default_rng(4304).standard_normal(R_U)
    c0 = 0.05
    model = saa.Model(R_M, D_Z, R_U, W, 4)
    model.set_params(flat32)
    model.set_qoi(c, c0)
    ctx = saa.Context(prob, N)
    ctx.set_samples(torch.from_numpy(xi).cuda())
    ref_model = surrogate.Surrogate(layers64, R_M, D_Z, c.astype(np.float32).astype(np.float64), c0)
    q_ref, g_ref = surrogate.qoi_and_grad(ref_model, surrogate.encode(xi, R_M), z)
    yield prob, xi, z, model, ctx, q_ref, g_ref, widths
    ctx.close()
    model.close()


# Bounds derived as for the 2D surrogate (BF16 unit roundoff 2^-9 through the
# forward and reverse chains of products); FP8 has no accuracy target.
@pytest.mark.parametrize("prec,tol_q,tol_g", [(saa.FP32, 1e-5, 1e-4), (saa.BF16, 2e-3, 4e-2), (saa.FP8, 5e-2, 6e-1)])
def test_per_sample_3d(setup3, prec, tol_q, tol_g):
    prob, xi, z, model, ctx, q_ref, g_ref, widths = setup3
    print(f"case mrdino3d per_sample prec={prec}", flush=True)
    q, g, rep = ctx.per_sample(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=prec))
    q, g = q.cpu().numpy(), g.cpu().numpy()
    eq = np.abs(q - q_ref) / np.abs(q_ref)
    eg = np.linalg.norm(g - g_ref, axis=1) / np.linalg.norm(g_ref, axis=1)
    print(f"  q rel max {eq.max():.3e} mean {eq.mean():.3e}; g rel max {eg.max():.3e} median {np.median(eg):.3e}")
    assert eq.max() <= tol_q
    assert np.median(eg) <= tol_g / 4 and eg.max() <= tol_g


@pytest.mark.parametrize("prec,tol,tol_g", [(saa.FP32, 1e-5, 1e-5), (saa.BF16, 2e-2, 2e-2), (saa.FP8, 2e-2, 0.3)])
def test_objective_3d(setup3, prec, tol, tol_g):
    prob, xi, z, model, ctx, q_ref, g_ref, widths = setup3
    ref = cvar.objective(q_ref, g_ref, z, 0.95, 1e-4, 1e-3)
    J, grad, rep = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=prec))
    print(f"  prec={prec} relJ {abs(J - ref['J']) / abs(ref['J']):.3e} relgrad {_rel(grad, ref['grad']):.3e}")
    assert abs(J - ref["J"]) <= tol * abs(ref["J"])
    assert _rel(grad, ref["grad"]) <= tol_g


def test_eval_outputs_3d(setup3):
    """phi and dphi/dz (forward mode, FP32) against the oracle's forward-mode
    Jacobian at width 512 with 64 controls."""
    prob, xi, z, model, ctx, q_ref, g_ref, widths = setup3
    out = model.eval(ctx, z)
    phi, dphi = out["phi"].cpu().numpy(), out["dphidz"].cpu().numpy()
    layers64 = training.unflatten(model.get_params().astype(np.float64), widths)
    x = np.concatenate([surrogate.encode(xi, R_M), np.broadcast_to(z, (xi.shape[0], D_Z))], axis=1)
    phi_ref, jac_ref = surrogate.jacobian_z(layers64, x, R_M)
    e_phi, e_jac = _rel(phi, phi_ref), _rel(dphi, np.transpose(jac_ref, (0, 2, 1)))
    print(f"  phi rel {e_phi:.3e}; dphi/dz rel {e_jac:.3e}")
    assert e_phi <= 1e-5 and e_jac <= 1e-5
    assert _rel(out["q"].cpu().numpy(), q_ref) <= 1e-5 and _rel(out["dqdz"].cpu().numpy(), g_ref) <= 1e-4


def test_graph_replay_3d(setup3):
    prob, xi, z, model, ctx, q_ref, g_ref, widths = setup3
    eager = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=saa.BF16, timing=1))
    for _ in range(3):
        J, g, r = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=saa.BF16))
    assert r["graph"] == 1 and J == eager[0] and np.array_equal(g, eager[1])
