"""The persisted autotuner: every tile shape of the fused surrogate kernel
gives bitwise the same q_i and dq_i/dz (widths 256 and 512), a choice made
by timing at first use is written to the cache file and read back by a new
process, and 3D threads-per-sample choices are recorded the same way."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa
import saa_inputs as si
from oracle import training

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def private_cache(tmp_path_factory):
    old = os.environ.get("SAA_TUNE_CACHE")
    os.environ["SAA_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "in_process.txt")
    yield
    if old is None:
        del os.environ["SAA_TUNE_CACHE"]
    else:
        os.environ["SAA_TUNE_CACHE"] = old


@pytest.mark.parametrize("width,r_m,d_z,r_u,dim,nvar", [(256, 100, 25, 200, 2, 3), (512, 200, 64, 400, 3, 2)])
@pytest.mark.parametrize("prec", [saa.BF16, saa.FP8])
def test_every_tile_shape_gives_the_same_results(gpu_lib, width, r_m, d_z, r_u, dim, nvar, prec):
    N = 1000
    if dim == 2:
        prob = saa.Problem(n=16, kl_per_dim=16)
        xi = si.kl_coefficients(6001, N, 16)
    else:
        prob = saa.Problem(dim=3, n=8, n_src_per_dim=4, src_sigma=0.08, kl_per_dim=6, kl_exp=1.5)
        xi = si.kl_coefficients(6001, N, 6, dim=3)
    widths = [r_m + d_z, width, width, width, width, r_u]
    model = saa.Model(r_m, d_z, r_u, width, 4)
    model.set_params(training.flatten(si.random_mlp(6002, widths)).astype(np.float32))
    model.set_qoi(0.3 * np.random.default_rng(6003).standard_normal(r_u), 0.05)
    ctx = saa.Context(prob, N)
    ctx.set_samples(torch.from_numpy(xi).cuda())
    z = si.control(6004, d_z)
    key = f"mlp/w{width}/p{1 if prec == saa.BF16 else 2}/N1024"
    outs = []
    for v in range(nvar):
        saa.tune_set(key, v)
        assert saa.tune_get(key) == v
        q, g, _ = ctx.per_sample(z, form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=prec))
        outs.append((q.cpu().numpy(), g.cpu().numpy()))
    print(f"case tile shapes width={width} prec={prec}: {nvar} shapes", flush=True)
    for q, g in outs[1:]:
        assert np.array_equal(q, outs[0][0]) and np.array_equal(g, outs[0][1])
    ctx.close()
    model.close()


_CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np, torch
import paper_2305_20053_amd as saa, saa_inputs as si
from oracle import training
key = "mlp/w256/p1/N4096"
if sys.argv[1] == "tune":
    assert saa.tune_get(key) is None
    prob = saa.Problem(n=16, kl_per_dim=16)
    model = saa.Model(100, 25, 200, 256, 4)
    model.set_params(training.flatten(si.random_mlp(6005, [125, 256, 256, 256, 256, 200])).astype(np.float32))
    ctx = saa.Context(prob, 3000)
    ctx.set_samples(torch.from_numpy(si.kl_coefficients(6006, 3000, 16)).cuda())
    ctx.per_sample(si.control(6007), form=saa.FORM_MRDINO, model=model, opt=saa.options(prec=saa.BF16))
print("CHOICE", saa.tune_get(key), flush=True)
"""


def test_choice_is_persisted_for_the_next_process(gpu_lib, tmp_path):
    path = tmp_path / "cache.txt"
    env = dict(os.environ, SAA_TUNE_CACHE=str(path))
    code = _CHILD.format(root=ROOT)
    a = subprocess.run([sys.executable, "-c", code, "tune"], env=env, capture_output=True, text=True, timeout=240)
    assert a.returncode == 0, a.stderr[-2000:]
    choice = [ln for ln in a.stdout.splitlines() if ln.startswith("CHOICE")][0].split()[1]
    assert choice in ("0", "1", "2")
    lines = path.read_text().splitlines()
    assert any(ln.split()[0].endswith("/mlp/w256/p1/N4096") and ln.split()[1] == choice for ln in lines), lines
    b = subprocess.run([sys.executable, "-c", code, "read"], env=env, capture_output=True, text=True, timeout=240)
    assert b.returncode == 0, b.stderr[-2000:]
    assert f"CHOICE {choice}" in b.stdout


def test_3d_threads_per_sample_recorded(gpu_lib):
    prob = saa.Problem(dim=3, n=8, n_src_per_dim=2, src_sigma=0.08, kl_per_dim=3, kl_exp=1.5)
    ctx = saa.Context(prob, 5)
    ctx.set_samples(torch.from_numpy(si.kl_coefficients(6008, 5, 3, dim=3)).cuda())
    ctx.objective_grad(si.control(6009, prob.d_z), opt=saa.options(prec=saa.FP32_DC64))
    bs, ba = ctx.launch3(saa.FP32_DC64)
    assert saa.tune_get(f"state3/p{saa.FP32_DC64}/n8/N5") == bs and bs in (256, 512, 1024)
    ctx.close()
