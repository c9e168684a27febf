"""GPU parity of the expectation-type risk measures (Sec. 2.1-2.2: mean,
mean + kappa variance, smoothed probability of failure, smoothed buffered
probability of exceedance) against the oracle's definitions.

Reduction alone (per-sample q, dq/dz read back from the device, N = 20000):
1e-12 relative.  PDE form end to end (FP64, 64 samples): J and grad J to
1e-9, with adjoints solved exactly for the samples of non-zero weight.
"""
import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa
import saa_inputs as si
from oracle import fem2d, risk, saa as osaa, training

pytestmark = pytest.mark.gpu

R_M, D_Z, R_U = 100, 25, 200


def _ref(kind, q, g, z, kappa, tau, eps, alpha=1e-3):
    if kind == saa.RISK_MEAN:
        return risk.mean(q, g, z, alpha)
    if kind == saa.RISK_MEAN_VAR:
        return risk.mean_var(q, g, z, kappa, alpha)
    if kind == saa.RISK_BPOE:
        return risk.bpoe(q, g, z, tau, eps, alpha)
    return risk.pof(q, g, z, tau, eps, alpha)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def surr(gpu_lib):
    prob = saa.problem_medium()
    N = 20000
    xi = si.kl_coefficients(5101, N, prob.kl_per_dim)
    z = si.control(5102)
    widths = [R_M + D_Z, 256, 256, 256, 256, R_U]
    model = saa.Model(R_M, D_Z, R_U, 256, 4)
    model.set_params(training.flatten(si.random_mlp(5103, widths, bias_scale=0.1)).astype(np.float32))
    model.set_qoi(0.3 * np.random.default_rng(5104).standard_normal(R_U), 0.05)
    ctx = saa.Context(prob, N)
    ctx.set_samples(torch.from_numpy(xi).cuda())
    q, g, _ = ctx.per_sample(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=saa.FP32))
    yield ctx, model, z, q.cpu().numpy(), g.cpu().numpy()
    ctx.close()


@pytest.mark.parametrize("kind", [saa.RISK_MEAN, saa.RISK_MEAN_VAR, saa.RISK_POF, saa.RISK_BPOE])
def test_reduction_matches_oracle(surr, kind):
    ctx, model, z, q, g = surr
    tau = float(np.quantile(q, 0.8))
    eps = 0.25 * float(np.std(q)) if kind != saa.RISK_BPOE else 0.1   # bPOE smooths a dimensionless argument
    print(f"case risk reduction kind={kind}", flush=True)
    opt = saa.options(prec=saa.FP32, risk=kind, risk_kappa=0.7, risk_tau=tau, eps=eps)
    J, grad, rep = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=opt)
    ref = _ref(kind, q, g, z, 0.7, tau, eps)
    print(f"  J rel {abs(J - ref['J']) / abs(ref['J']):.2e}; grad rel {_rel(grad, ref['grad']):.2e}")
    assert abs(J - ref["J"]) <= 1e-12 * abs(ref["J"])
    assert _rel(grad, ref["grad"]) <= 1e-12
    assert abs(rep["t_star"] - ref["t"]) <= 1e-13 * max(1.0, abs(ref["t"])) and rep["dJ_dt"] == 0.0
    if kind == saa.RISK_BPOE:
        assert 0.0 < rep["t_star"] < float("inf") and 0.2 < J < 1.0
    # the replayed graph gives the same bits as the eager evaluation
    J2, grad2, rep2 = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=opt)
    J3, grad3, rep3 = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=opt)
    assert rep3["graph"] == 1 and J3 == J and np.array_equal(grad3, grad)


@pytest.fixture(scope="module")
def pde(gpu_lib):
    prob = saa.problem_small(target=saa.TARGET_SIN)
    xi = si.kl_coefficients(si.SEED_XI_SMALL, 64, prob.kl_per_dim)
    z = si.control(si.SEED_Z_SMALL)
    oref = osaa.objective_grad(fem2d.Problem2D(n=prob.n, kl_per_dim=prob.kl_per_dim, target=prob.target), xi, z)
    ctx = saa.Context(prob, 64)
    ctx.set_samples(torch.from_numpy(xi).cuda())
    yield ctx, z, oref["q"], oref["g"]
    ctx.close()


@pytest.mark.parametrize("kind", [saa.RISK_MEAN, saa.RISK_MEAN_VAR, saa.RISK_POF, saa.RISK_BPOE])
def test_pde_form_matches_oracle(pde, kind):
    ctx, z, q, g = pde
    tau = float(np.quantile(q, 0.7))
    eps = 0.3 * float(np.std(q)) if kind != saa.RISK_BPOE else 0.1
    print(f"case risk pde kind={kind}", flush=True)
    opt = saa.options(prec=saa.FP64, risk=kind, risk_kappa=2.0, risk_tau=tau, eps=eps)
    J, grad, rep = ctx.objective_grad(z, opt=opt)
    ref = _ref(kind, q, g, z, 2.0, tau, eps)
    assert abs(J - ref["J"]) <= 1e-9 * abs(ref["J"])
    assert _rel(grad, ref["grad"]) <= 1e-9
    x = q - tau
    if kind == saa.RISK_POF:
        want = int(np.sum((x > 0) & (x < eps)))
    elif kind == saa.RISK_BPOE:
        want = int(np.sum(ref["t"] * x + 1.0 > 0))
    else:
        want = 64
    assert rep["n_adjoints"] == want and 0 < want


def test_risk_options_are_validated(pde):
    ctx, z, q, g = pde
    for kw in [dict(risk=5), dict(risk=-1), dict(risk=saa.RISK_MEAN, t_mode=1, t_in=0.0),
               dict(risk=saa.RISK_MEAN_VAR, risk_kappa=-1.0), dict(risk=saa.RISK_POF, risk_tau=float("nan"))]:
        with pytest.raises(saa.SaaError) as e:
            ctx.objective_grad(z, opt=saa.options(**kw))
        assert e.value.status == saa.SAA_E_INVALID
