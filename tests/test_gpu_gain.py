"""What derivative-informed training gains (paper Sec. 3.2, 4.2.1): with the
same data, initialisation and epochs, MR-DINO is compared with MR-NO (L2-only
loss) on held-out samples projected on the training POD basis, and on the SAA
objective gradient against the PDE form at a fixed control."""
import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa
import saa_inputs as si
from oracle import training

pytestmark = pytest.mark.gpu

N_TRAIN, N_VAL, R_M, R_U, N_POD, EPOCHS = 512, 128, 100, 64, 256, 120


@pytest.fixture(scope="module")
def trained(gpu_lib):
    prob = saa.Problem(n=64, kl_per_dim=16)
    ctx = saa.Context(prob, N_TRAIN)
    ctx.set_samples(torch.from_numpy(si.kl_coefficients(si.SEED_XI_TRAIN, N_TRAIN, 16)).cuda())
    Zt = torch.from_numpy(si.controls(si.SEED_Z_TRAIN, N_TRAIN)).cuda()
    data = saa.TrainData(ctx, Zt, r_m=R_M, r_u=R_U, n_pod=N_POD)
    vctx = saa.Context(prob, N_VAL)
    vctx.set_samples(torch.from_numpy(si.kl_coefficients(si.SEED_XI_VALID, N_VAL, 16)).cuda())
    Zv = torch.from_numpy(si.controls(si.SEED_Z_VALID, N_VAL)).cuda()
    vdata = saa.TrainData(vctx, Zv, r_m=R_M, r_u=R_U, basis=data)
    widths = [R_M + ctx.d_z, 256, 256, 256, 256, R_U]
    init = saa.init_params(si.glorot_mlp(2315, widths), data.output_scale())
    out = {}
    for name, dino in (("dino", 1), ("no", 0)):
        model = saa.Model(R_M, ctx.d_z, R_U, 256, 4)
        model.set_params(init)
        hist, secs = saa.train(model, data, saa.train_cfg(batch=64, epochs=EPOCHS, lr_drop_epoch=EPOCHS // 2,
                                                           dino=dino, seed=7))
        out[name] = dict(model=model, train=saa.data_errors(model, data), val=saa.data_errors(model, vdata),
                         hist=hist, secs=secs)
    return prob, vctx, out


def test_dino_improves_heldout_jacobian_and_state(trained):
    prob, vctx, out = trained
    for k in ("dino", "no"):
        print(k, "train", out[k]["train"], "val", out[k]["val"], "seconds", out[k]["secs"])
    d, n = out["dino"]["val"], out["no"]["val"]
    assert d[1] < 0.5 * n[1]          # held-out reduced Jacobian error
    assert d[0] < n[0]                # held-out reduced state error


def test_dino_improves_saa_gradient(trained):
    prob, vctx, out = trained
    z = si.control(si.SEED_Z_EVAL[1])
    errs = {}
    for beta in (0.0, 0.5):
        opt = saa.options(beta=beta)
        Jp, gp, _ = vctx.objective_grad(z, opt=opt)
        for k in ("dino", "no"):
            Js, gs, _ = vctx.objective_grad(z, form=saa.FORM_MRDINO, model=out[k]["model"],
                                            opt=saa.options(beta=beta, prec=saa.FP32))
            errs[(k, beta)] = (abs(Js - Jp) / abs(Jp), float(np.linalg.norm(gs - gp) / np.linalg.norm(gp)))
    print(errs)
    for beta in (0.0, 0.5):
        assert errs[("dino", beta)][1] < errs[("no", beta)][1]


def test_error_estimate_and_pde_fallback(trained):
    """The estimate compares surrogate and PDE form on held-out samples; a
    poor surrogate (MR-NO) or a tight tolerance switches to the PDE form."""
    prob, vctx, out = trained
    N = 300
    ctx = saa.Context(prob, N)
    ctx.set_samples(torch.from_numpy(si.kl_coefficients(si.SEED_XI_HELDOUT, N, 16)).cuda())
    saa.attach_holdout(ctx, vctx)
    z = si.control(si.SEED_Z_EVAL[2])
    Jpde, gpde, _ = ctx.objective_grad(z, opt=saa.options())
    # loose tolerance: surrogate result, estimate reported
    Js, gs, rep = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=out["dino"]["model"],
                                     opt=saa.options(prec=saa.FP32, fallback_tol=10.0))
    assert rep["status"] == saa.SAA_OK and rep["fallback_used"] == 0 and 0.0 < rep["err_estimate"] < 10.0
    Jv, gv, _ = vctx.objective_grad(z, form=saa.FORM_MRDINO, model=out["dino"]["model"], opt=saa.options(prec=saa.FP32))
    Jvp, gvp, _ = vctx.objective_grad(z, opt=saa.options())
    manual = max(abs(Jv - Jvp) / abs(Jvp), np.linalg.norm(gv - gvp) / np.linalg.norm(gvp))
    assert abs(rep["err_estimate"] - manual) <= 1e-9 * manual
    # tight tolerance: the PDE form on the main samples, flagged
    Jf, gf, rep = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=out["no"]["model"],
                                     opt=saa.options(prec=saa.FP32, fallback_tol=1e-6))
    assert rep["status"] == saa.SAA_W_FALLBACK and rep["fallback_used"] == 1
    assert Jf == Jpde and np.array_equal(gf, gpde)
    # detached: no estimate
    saa.attach_holdout(ctx, None)
    _, _, rep = ctx.objective_grad(z, form=saa.FORM_MRDINO, model=out["no"]["model"], opt=saa.options(prec=saa.FP32))
    assert rep["err_estimate"] == -1.0 and rep["fallback_used"] == 0
    ctx.close()
