"""GPU parity of the smoothed-CVaR reduction alone (Sec. 2.1-2.2): t*, J,
dJ/dt and grad J from the device reduction against the FP64 oracle
evaluated on the very same per-sample q_i and dq_i/dz (read back from the
device), so that only the reduction is compared.

The per-sample values come from the surrogate form with a random network:
N = 20000 samples is large enough to use many workgroups, and the cases span
the regimes of the t* search: a few probe passes then an active set of a few
samples (eps = 1e-4), a wide smoothing zone, an active set larger than its
capacity (eps far above, or comparable to, the spread of q: multi-workgroup
refinement passes then a secant step), beta = 0 (degenerate minimiser), a tail of 20 samples, and a
prescribed t.  Tolerance: 1e-12 relative on J and grad J (only the
summation order differs); t* to 1e-14 relative, since grad J moves with t*
through s_eps'' (at most 1.5 / eps).
"""
import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa
import saa_inputs as si
from oracle import cvar, training

pytestmark = pytest.mark.gpu

R_M, D_Z, R_U = 100, 25, 200
TOL = 1e-12
TOL_T = 1e-14


@pytest.fixture(scope="module")
def data(gpu_lib):
    prob = saa.problem_medium()
    N = 20000
    xi = si.kl_coefficients(5001, N, prob.kl_per_dim)
    z = si.control(5002)
    widths = [R_M + D_Z, 256, 256, 256, 256, R_U]
    layers = si.random_mlp(5003, widths, bias_scale=0.1)
    model = saa.Model(R_M, D_Z, R_U, 256, 4)
    model.set_params(training.flatten(layers).astype(np.float32))
    rng = np.random.default_rng(5004)
    model.set_qoi(0.3 * rng.standard_normal(R_U), 0.05)
    ctx = saa.Context(prob, N)
    ctx.set_samples(torch.from_numpy(xi).cuda())
    q, g, _ = ctx.per_sample(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=saa.FP32))
    return ctx, model, z, q.cpu().numpy(), g.cpu().numpy()


def _t_error(q, t_gpu, t_ref, beta, eps, t_mode):
    """Relative t* error where the root of Phi(t) = N (1 - beta) is unique.
    When N (1 - beta) is an integer k and the k-th largest q exceeds the
    (k+1)-th by eps or more (always for beta = 0), Phi equals k on the whole
    piece [q_(k+1), q_(k) - eps] and every t there minimises J_hat with the
    same J and grad J; the GPU's t* must then lie on that piece (widened by
    1e-6 eps, where the smoothing changes J by O(1e-18 eps)), and 0 is
    returned."""
    rel = abs(t_gpu - t_ref) / max(abs(t_ref), 1e-300)
    if t_mode == 1:
        return rel
    target = q.size * (1.0 - beta)
    k = int(round(target))
    if 1 <= k <= q.size and abs(target - k) <= 1e-9 * target:
        qs = np.sort(q)[::-1]
        lo = qs[k] if k < q.size else -np.inf
        hi = qs[k - 1] - eps
        if hi >= lo:
            assert lo - 1e-6 * eps <= t_gpu <= hi + 1e-6 * eps, (lo, hi, t_gpu)
            return 0.0
    return rel


@pytest.mark.parametrize("beta,eps,t_mode", [
    (0.95, 1e-4, 0),
    (0.9, 1e-2, 0),
    (0.5, 1e3, 0),       # every sample inside the smoothing zone: active-set overflow
    (0.95, 2.0, 0),      # eps comparable to the spread of q (trained surrogates): overflow, refinement passes
    (0.0, 1e-4, 0),      # beta = 0: t* = min q - eps
    (0.999, 1e-6, 0),    # tail of 20 samples
    (0.95, 1e-4, 1),     # prescribed t
])
def test_reduction_matches_oracle(data, beta, eps, t_mode):
    ctx, model, z, q, g = data
    print(f"case cvar beta={beta} eps={eps} t_mode={t_mode} N={q.size}", flush=True)
    t_in = float(np.quantile(q, 0.9)) if t_mode == 1 else 0.0
    opt = saa.options(prec=saa.FP32, beta=beta, eps=eps, t_mode=t_mode, t_in=t_in)
    J, grad, rep = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=opt)
    ref = cvar.objective(q, g, z, beta, eps, 1e-3, t_mode=t_mode, t_in=t_in)
    et = _t_error(q, rep["t_star"], ref["t"], beta, eps, t_mode)
    eJ = abs(J - ref["J"]) / abs(ref["J"])
    eg = np.linalg.norm(grad - ref["grad"]) / np.linalg.norm(ref["grad"])
    ed = abs(rep["dJ_dt"] - ref["dJdt"])
    print(f"  t* {rep['t_star']:.17g} rel {et:.2e}; J rel {eJ:.2e}; grad rel {eg:.2e}; dJ/dt diff {ed:.2e}")
    assert et <= TOL_T and eJ <= TOL and eg <= TOL
    assert ed <= 1e-10
    if t_mode == 0:
        assert abs(rep["dJ_dt"]) <= 1e-10          # stationarity in t


def test_reduction_is_deterministic(data):
    ctx, model, z, q, g = data
    opt = saa.options(prec=saa.FP32, beta=0.95, eps=1e-4)
    runs = [ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=opt) for _ in range(3)]
    for J, grad, rep in runs[1:]:
        assert J == runs[0][0] and np.array_equal(grad, runs[0][1]) and rep["t_star"] == runs[0][2]["t_star"]


@pytest.fixture(scope="module")
def many(gpu_lib):
    """N = 1000003 (not a multiple of any tile): the multi-workgroup passes
    keep their 256 workgroups and each walks a contiguous chunk of about
    3900 samples tile by tile, so a workgroup's own active segment can
    overflow; the 20000-sample set above gives each thread at most one
    sample.  A 4 x 4 grid keeps the context small (the surrogate form does
    not touch it)."""
    prob = saa.Problem(n=4, kl_per_dim=10)
    N = 1000003
    xi = si.kl_coefficients(5005, N, prob.kl_per_dim)
    z = si.control(5006)
    widths = [R_M + D_Z, 256, 256, 256, 256, R_U]
    layers = si.random_mlp(5007, widths, bias_scale=0.1)
    model = saa.Model(R_M, D_Z, R_U, 256, 4)
    model.set_params(training.flatten(layers).astype(np.float32))
    rng = np.random.default_rng(5008)
    model.set_qoi(0.3 * rng.standard_normal(R_U), 0.05)
    ctx = saa.Context(prob, N)
    ctx.set_samples(torch.from_numpy(xi).cuda())
    del xi
    q, g, _ = ctx.per_sample(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=saa.FP32))
    return ctx, model, z, q.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("beta,eps", [
    (0.95, 1e-4),
    (0.5, 1e3),          # every sample inside the smoothing zone: per-workgroup overflow, refinement passes
])
def test_reduction_many_samples_per_workgroup(many, beta, eps):
    ctx, model, z, q, g = many
    print(f"case cvar N={q.size} beta={beta} eps={eps}", flush=True)
    opt = saa.options(prec=saa.FP32, beta=beta, eps=eps)
    J, grad, rep = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=opt)
    ref = cvar.objective(q, g, z, beta, eps, 1e-3)
    et = _t_error(q, rep["t_star"], ref["t"], beta, eps, 0)
    eJ = abs(J - ref["J"]) / abs(ref["J"])
    eg = np.linalg.norm(grad - ref["grad"]) / np.linalg.norm(ref["grad"])
    print(f"  t* rel {et:.2e}; J rel {eJ:.2e}; grad rel {eg:.2e}; dJ/dt {rep['dJ_dt']:.2e}")
    assert et <= TOL_T and eJ <= TOL and eg <= TOL
    assert abs(rep["dJ_dt"]) <= 1e-10


@pytest.mark.parametrize("risk,kw", [(saa.RISK_CVAR, {}), (saa.RISK_CVAR, {"t_mode": 1, "t_in": 21.0}),
                                     (saa.RISK_MEAN_VAR, {"risk_kappa": 0.5}), (saa.RISK_POF, {"risk_tau": 21.0}),
                                     (saa.RISK_BPOE, {"risk_tau": 21.0})])
def test_standalone_reduction_matches_objective(data, risk, kw):
    """saa_risk_reduce on the device arrays q, g gives bitwise the J, dJ/dt,
    grad and t of the reduction inside saa_objective_grad on the same q, g."""
    ctx, model, z, q, g = data
    opt = saa.options(prec=saa.FP32, risk=risk, **kw)
    J, grad, rep = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=opt)
    qd = torch.from_numpy(q).cuda()
    gd = torch.from_numpy(g).cuda()
    Jr, dJr, gr, tr = saa.risk_reduce(qd, gd, z, opt)
    assert Jr == J and np.array_equal(gr, grad) and tr == rep["t_star"] and dJr == rep["dJ_dt"]
