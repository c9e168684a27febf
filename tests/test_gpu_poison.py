"""NaN-poisoned workspaces (a debugging mode of the library): with
SAA_POISON_WORKSPACE set when a context is created, every objective and
per-sample call first fills the context's per-call buffers with NaN bytes.
A kernel that read any of them before writing it would turn the results into
NaN or change them; these tests require bitwise the results of an ordinary
context, for the 2D and 3D PDE forms and the surrogate form (eager call,
graph capture and replay)."""
import os

import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa
import saa_inputs as si
from oracle import training

pytestmark = pytest.mark.gpu


def _contexts(prob, xi):
    out = []
    for poison in (False, True):
        if poison:
            os.environ["SAA_POISON_WORKSPACE"] = "1"
        try:
            ctx = saa.Context(prob, xi.shape[0])
        finally:
            os.environ.pop("SAA_POISON_WORKSPACE", None)
        ctx.set_samples(torch.from_numpy(xi).cuda())
        out.append(ctx)
    return out


def _same(a, b):
    (Ja, ga, ra), (Jb, gb, rb) = a, b
    assert np.isfinite(Jb) and np.all(np.isfinite(gb))
    assert Ja == Jb and np.array_equal(ga, gb) and ra["t_star"] == rb["t_star"]


@pytest.mark.parametrize("prec", [saa.FP32_DC64, saa.FP64])
def test_poisoned_pde_form_2d(gpu_lib, prec):
    prob = saa.problem_small()
    xi = si.kl_coefficients(si.SEED_XI_SMALL, 64, prob.kl_per_dim)
    z = si.control(si.SEED_Z_SMALL)
    print(f"case poison 2D n=32 N=64 prec={prec}", flush=True)
    plain, poisoned = _contexts(prob, xi)
    opt = saa.options(prec=prec)
    for _ in range(2):
        _same(plain.objective_grad(z, opt=opt), poisoned.objective_grad(z, opt=opt))
    qa, ga, _ = plain.per_sample(z, opt=opt)
    qb, gb, _ = poisoned.per_sample(z, opt=opt)
    assert torch.equal(qa, qb) and torch.equal(ga, gb)
    plain.close()
    poisoned.close()


def test_poisoned_pde_form_3d(gpu_lib):
    prob = saa.Problem(dim=3, n=8, n_src_per_dim=2, src_sigma=0.08, kl_per_dim=3, kl_shift=25.0, kl_exp=1.5,
                       kl_amp=20.0)
    xi = si.kl_coefficients(2401, 6, 3, dim=3)
    z = si.control(2402, prob.d_z)
    print("case poison 3D n=8 N=6", flush=True)
    plain, poisoned = _contexts(prob, xi)
    opt = saa.options(prec=saa.FP32_DC64)
    _same(plain.objective_grad(z, opt=opt), poisoned.objective_grad(z, opt=opt))
    plain.close()
    poisoned.close()


@pytest.mark.parametrize("prec", [saa.BF16, saa.FP32])
def test_poisoned_surrogate_form(gpu_lib, prec):
    prob = saa.problem_medium()
    N = 1000
    xi = si.kl_coefficients(4001, N, prob.kl_per_dim)
    z = si.control(4002)
    widths = [125, 256, 256, 256, 256, 200]
    model = saa.Model(100, 25, 200, 256, 4)
    model.set_params(training.flatten(si.random_mlp(4003, widths, bias_scale=0.1)).astype(np.float32))
    model.set_qoi(0.3 * np.random.default_rng(4004).standard_normal(200), 0.05)
    print(f"case poison surrogate N={N} prec={prec}", flush=True)
    plain, poisoned = _contexts(prob, xi)
    opt = saa.options(prec=prec)
    ref = plain.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=opt)
    for _ in range(3):   # eager, captured, replayed
        _same(ref, poisoned.objective_grad(z, form=saa.FORM_MRDINO, model=model, opt=opt))
    plain.close()
    poisoned.close()
    model.close()
