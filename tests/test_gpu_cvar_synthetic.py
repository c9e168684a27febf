"""The CVaR reduction (Sec. 2.1-2.2, eq. (CVaR_saa_ouu)) on synthetic q_i
chosen to drive each branch of the device t* search, through
saa_risk_reduce on caller arrays, against the FP64 oracle on the same
values:

* a dense window (about 58k of 65536 samples within 5 eps of t*, as a trained
  surrogate gives): refinement passes and the cubic finish;
* uniform q with eps set so that the active window holds about 700, 1000 and
  1400 samples: both sides of the 1024-value capacity of the one-workgroup
  Newton iteration;
* heavy ties (37 distinct values) where N (1 - beta) is an integer and Phi
  is flat at the target (any t on the flat piece minimises J);
* large magnitudes (q ~ 1e6 with eps = 1e-4) and ragged small N.

Tolerance: 1e-12 relative on J and grad J (only the summation order
differs); t* to 1e-14 relative where the root is unique, else on the flat
piece.  dJ/dt at the returned t* to 1e-10, or to a few times what one ulp of
t* moves it by (J''(t*) ulp(t*)) when that is larger, as at q ~ 1e6.  The
allocation-free entry point must give bitwise the same results."""
import zlib

import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa
from oracle import cvar

pytestmark = pytest.mark.gpu

DZ = 25


def _case(name):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    if name == "dense":
        q = 0.18 + 5e-4 * rng.standard_normal(65536)
        return q, 0.95, 1e-4
    if name.startswith("uniform"):
        N = 50000
        window = {"uniform700": 700, "uniform1000": 1000, "uniform1400": 1400}[name]
        return rng.random(N), 0.95, window / (5.0 * N)
    if name == "ties":
        vals = np.sort(rng.random(37))
        return vals[rng.integers(0, 37, 30000)], 0.9, 1e-3
    if name == "large":
        return 1e6 + rng.random(20000), 0.95, 1e-4
    if name.startswith("ragged"):
        N = int(name[6:])
        return rng.standard_normal(N), 0.5 if N < 4 else 0.95, 1e-2
    raise ValueError(name)


def _t_ok(q, t_gpu, t_ref, beta, eps):
    target = q.size * (1.0 - beta)
    k = int(round(target))
    if 1 <= k <= q.size and abs(target - k) <= 1e-9 * target:
        qs = np.sort(q)[::-1]
        lo = qs[k] if k < q.size else -np.inf
        hi = qs[k - 1] - eps
        if hi >= lo:   # Phi = k on [lo, hi]: every t there is a minimiser
            return lo - 1e-6 * eps <= t_gpu <= hi + 1e-6 * eps
    return abs(t_gpu - t_ref) <= 1e-14 * abs(t_ref)


@pytest.mark.parametrize("name", ["dense", "uniform700", "uniform1000", "uniform1400", "ties", "large",
                                  "ragged1", "ragged2", "ragged257", "ragged1023"])
def test_reduction_on_synthetic_q(gpu_lib, name):
    q, beta, eps = _case(name)
    rng = np.random.default_rng(7)
    g = rng.standard_normal((q.size, DZ))
    z = rng.random(DZ)
    print(f"case synthetic cvar {name} N={q.size} beta={beta} eps={eps:.3g}", flush=True)
    opt = saa.options(beta=beta, eps=eps)
    qd = torch.from_numpy(q).cuda()
    gd = torch.from_numpy(g).cuda()
    J, dJdt, grad, t = saa.risk_reduce(qd, gd, z, opt)
    ref = cvar.objective(q, g, z, beta, eps, opt.alpha)
    eJ = abs(J - ref["J"]) / abs(ref["J"])
    eg = np.linalg.norm(grad - ref["grad"]) / np.linalg.norm(ref["grad"])
    print(f"  t* {t:.17g} oracle {ref['t']:.17g}; J rel {eJ:.2e}; grad rel {eg:.2e}; dJ/dt {dJdt:.2e}")
    assert _t_ok(q, t, ref["t"], beta, eps)
    assert eJ <= 1e-12 and eg <= 1e-12
    curv = np.sum(cvar.d2splus(q - t, eps)) / (q.size * (1.0 - beta))
    assert abs(dJdt) <= max(1e-10, 4.0 * curv * np.spacing(abs(t)))
    J2, dJdt2, grad2, t2 = saa.risk_reduce(qd, gd, z, opt, noalloc=True)
    assert J2 == J and dJdt2 == dJdt and np.array_equal(grad2, grad) and t2 == t
