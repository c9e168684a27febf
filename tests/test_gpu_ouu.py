"""GPU outer OUU solve (Sec. 2.1 eq. (ouu) / (CVaR_ouu); Sec. 4.2: box Z_ad,
bound-constrained L-BFGS) against the oracle's L-BFGS-B on the oracle
objective, from the same start.

PDE form (FP64, n = 32, 16 samples, sinusoidal target, box [-1.5, 1.5]^25
with some bounds active): optimal J to 1e-9 relative, z* to 1e-5, identical
active sets, and the GPU optimum is first-order optimal under the oracle
gradient.  Joint (z, t) form: the same optimum.  MR-DINO form (FP32 kernel,
random network): optimal J to 1e-5 relative.
"""
import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa
import saa_inputs as si
from oracle import cvar, fem2d, ouu, saa as osaa, surrogate, training

pytestmark = pytest.mark.gpu

LB, UB = -1.5, 1.5


@pytest.fixture(scope="module")
def pde(gpu_lib):
    prob = saa.problem_small(target=saa.TARGET_SIN)
    xi = si.kl_coefficients(si.SEED_XI_SMALL, 16, prob.kl_per_dim)
    oprob = fem2d.Problem2D(n=prob.n, kl_per_dim=prob.kl_per_dim, target=prob.target)

    def fg(z):
        r = osaa.objective_grad(oprob, xi, z)
        return r["J"], r["grad"]
    z_ref, J_ref, nfev = ouu.solve(fg, np.full(prob.d_z, 0.5), LB, UB, pgtol=1e-10)
    ctx = saa.Context(prob, 16)
    ctx.set_samples(torch.from_numpy(xi).cuda())
    yield prob, ctx, fg, z_ref, J_ref
    ctx.close()


def test_pde_ouu_matches_oracle(pde):
    prob, ctx, fg, z_ref, J_ref = pde
    print("case ouu pde fp64", flush=True)
    z, rep = ctx.ouu_solve(np.full(prob.d_z, 0.5), LB, UB, opt=saa.options(prec=saa.FP64), pgtol=1e-10, ftol=0.0)
    print(f"  J {rep['J']:.15g} ref {J_ref:.15g}; it {rep['iterations']} ev {rep['evaluations']} "
          f"status {rep['status']} active {rep['n_active']} |z-z_ref| {np.abs(z - z_ref).max():.2e}")
    assert rep["status"] in (saa.OUU_PGTOL, saa.OUU_FTOL, saa.OUU_LINESEARCH)
    assert abs(rep["J"] - J_ref) <= 1e-9 * abs(J_ref)
    assert np.abs(z - z_ref).max() <= 1e-5
    act = (z <= LB) | (z >= UB)
    assert np.array_equal(act, (z_ref <= LB) | (z_ref >= UB)) and 0 < act.sum() < prob.d_z
    J_o, g_o = fg(z)
    assert abs(J_o - rep["J"]) <= 1e-10 * abs(J_o)
    assert np.abs(ouu.projected_gradient(z, g_o, LB, UB)).max() <= 1e-7


def test_joint_t_form_reaches_the_same_optimum(pde):
    """min over (z, t) of J_hat equals min over z of min_t J_hat.  With 16
    samples the smoothing width must be wide enough for J_hat to be well
    conditioned in t (eps = 2e-2); the joint optimum is checked against the
    t-minimised GPU optimum and for first-order optimality under the oracle
    gradient at the same eps."""
    prob, ctx, fg, z_ref, J_ref = pde
    print("case ouu pde joint t", flush=True)
    opt = saa.options(prec=saa.FP64, eps=2e-2)
    z1, rep1 = ctx.ouu_solve(np.full(prob.d_z, 0.5), LB, UB, opt=opt, pgtol=1e-10, ftol=0.0)
    z, rep = ctx.ouu_solve(np.full(prob.d_z, 0.5), LB, UB, opt=opt, pgtol=1e-10, ftol=0.0, joint_t=1)
    print(f"  J {rep['J']:.15g} vs {rep1['J']:.15g}; it {rep['iterations']} status {rep['status']} t {rep['t']}")
    assert abs(rep["J"] - rep1["J"]) <= 1e-9 * abs(rep1["J"])
    assert np.abs(z - z1).max() <= 1e-4
    J_t, _, r = ctx.objective_grad(z, opt=opt)
    assert abs(rep["t"] - r["t_star"]) <= 1e-6 * max(1.0, abs(r["t_star"]))
    oprob = fem2d.Problem2D(n=prob.n, kl_per_dim=prob.kl_per_dim, target=prob.target)
    xi = si.kl_coefficients(si.SEED_XI_SMALL, 16, prob.kl_per_dim)
    g_o = osaa.objective_grad(oprob, xi, z, eps=2e-2)["grad"]
    assert np.abs(ouu.projected_gradient(z, g_o, LB, UB)).max() <= 1e-6


def test_mrdino_ouu_matches_oracle(gpu_lib):
    prob = saa.problem_medium()
    r_m, d_z, r_u, N = 100, 25, 200, 512
    xi = si.kl_coefficients(4101, N, prob.kl_per_dim)
    widths = [r_m + d_z, 256, 256, 256, 256, r_u]
    flat32 = training.flatten(si.random_mlp(4103, widths, bias_scale=0.1)).astype(np.float32)
    c = 0.3 * np.random.default_rng(4104).standard_normal(r_u)
    model = saa.Model(r_m, d_z, r_u, 256, 4)
    model.set_params(flat32)
    model.set_qoi(c, 0.05)
    ref_model = surrogate.Surrogate(training.unflatten(flat32.astype(np.float64), widths), r_m, d_z,
                                    c.astype(np.float32).astype(np.float64), 0.05)
    xhat = surrogate.encode(xi, r_m)

    def fg(z):
        q, g = surrogate.qoi_and_grad(ref_model, xhat, z)
        r = cvar.objective(q, g, z, 0.95, 1e-4, 1e-3)
        return r["J"], r["grad"]
    z_ref, J_ref, _ = ouu.solve(fg, np.zeros(d_z), -1.0, 1.0, pgtol=1e-9)
    ctx = saa.Context(prob, N)
    ctx.set_samples(torch.from_numpy(xi).cuda())
    print("case ouu mrdino fp32", flush=True)
    z, rep = ctx.ouu_solve(np.zeros(d_z), -1.0, 1.0, form=saa.FORM_MRDINO, model=model,
                           opt=saa.options(prec=saa.FP32), pgtol=1e-7)
    print(f"  J {rep['J']:.10g} ref {J_ref:.10g}; it {rep['iterations']} status {rep['status']}")
    assert abs(rep["J"] - J_ref) <= 1e-5 * abs(J_ref)
    assert abs(fg(z)[0] - J_ref) <= 1e-5 * abs(J_ref)
    ctx.close()


def test_ouu_rejects_bad_arguments(pde):
    prob, ctx, fg, z_ref, J_ref = pde
    z0 = np.zeros(prob.d_z)
    for kw in [dict(lb=1.0, ub=-1.0), dict(lb=np.nan, ub=1.0)]:
        with pytest.raises(saa.SaaError) as e:
            ctx.ouu_solve(z0, **kw)
        assert e.value.status == saa.SAA_E_INVALID
    with pytest.raises(saa.SaaError):
        ctx.ouu_solve(np.full(prob.d_z, np.inf))
    with pytest.raises(saa.SaaError):
        ctx.ouu_solve(z0, memory=0)
    with pytest.raises(saa.SaaError):
        ctx.ouu_solve(z0, joint_t=1, opt=saa.options(t_mode=1, t_in=0.0))
