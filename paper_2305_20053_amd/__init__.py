"""Python binding of the MI355X SAA smoothed-CVaR engine (libsaa.so).

Argument marshalling only: every numerical step runs in the HIP kernels
behind the C ABI declared in include/saa.h.  PyTorch provides device memory
and the stream.  If the shared library is missing, importing still works
(so that the host-side tests can run) but every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsaa.so")

SAA_OK, SAA_W_FALLBACK = 0, 1
SAA_E_INVALID, SAA_E_NOCONV, SAA_E_DEVICE, SAA_E_OOM, SAA_E_MODEL, SAA_E_IO = -1, -2, -3, -4, -5, -6
FORM_PDE, FORM_MRDINO = 0, 1
FP64, FP32, FP32_DC64, BF16, FP8 = 0, 1, 2, 3, 4
WANT_Q, WANT_DQDZ, WANT_PHI, WANT_DPHIDZ = 1, 2, 4, 8
TARGET_CONST, TARGET_SIN, TARGET_QUAD = 0, 1, 2
RISK_CVAR, RISK_MEAN, RISK_MEAN_VAR, RISK_POF, RISK_BPOE = 0, 1, 2, 3, 4
JAC_AUTO, JAC_FORWARD, JAC_ADJOINT = 0, 1, 2
OUU_PGTOL, OUU_FTOL, OUU_MAXITER, OUU_MAXEVAL, OUU_LINESEARCH = 0, 1, 2, 3, 4


class SaaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class COuuOptions(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("max_eval", ctypes.c_int), ("memory", ctypes.c_int),
                ("joint_t", ctypes.c_int), ("pgtol", ctypes.c_double), ("ftol", ctypes.c_double)]


class COuuReport(ctypes.Structure):
    _fields_ = [("J", ctypes.c_double), ("pg_norm", ctypes.c_double), ("t", ctypes.c_double),
                ("seconds", ctypes.c_double), ("iterations", ctypes.c_int), ("evaluations", ctypes.c_int),
                ("status", ctypes.c_int), ("n_active", ctypes.c_int), ("n_fallback", ctypes.c_int),
                ("pad", ctypes.c_int)]


class CProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("n_src_per_dim", ctypes.c_int),
                ("src_sigma", ctypes.c_double), ("kl_per_dim", ctypes.c_int),
                ("kl_shift", ctypes.c_double), ("kl_exp", ctypes.c_double), ("kl_amp", ctypes.c_double),
                ("reaction", ctypes.c_double), ("u_target", ctypes.c_double), ("target", ctypes.c_int),
                ("pad_", ctypes.c_int)]


class COptions(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("eps", ctypes.c_double), ("alpha", ctypes.c_double),
                ("t_mode", ctypes.c_int), ("t_in", ctypes.c_double), ("prec", ctypes.c_int),
                ("newton_tol", ctypes.c_double), ("lin_rtol", ctypes.c_double),
                ("max_newton", ctypes.c_int), ("max_lin", ctypes.c_int), ("max_dc", ctypes.c_int),
                ("all_adjoints", ctypes.c_int), ("fallback_tol", ctypes.c_double), ("timing", ctypes.c_int),
                ("risk", ctypes.c_int), ("jac_mode", ctypes.c_int), ("risk_kappa", ctypes.c_double),
                ("risk_tau", ctypes.c_double)]


class CDims(ctypes.Structure):
    _fields_ = [("r_m", ctypes.c_int), ("d_z", ctypes.c_int), ("r_u", ctypes.c_int), ("width", ctypes.c_int),
                ("depth", ctypes.c_int)]


class CReport(ctypes.Structure):
    _fields_ = [("t_star", ctypes.c_double), ("dJ_dt", ctypes.c_double), ("err_estimate", ctypes.c_double),
                ("seconds", ctypes.c_double), ("newton_max", ctypes.c_int), ("n_unconverged", ctypes.c_int),
                ("n_adjoints", ctypes.c_int), ("fallback_used", ctypes.c_int), ("lin_total", ctypes.c_int64),
                ("newton_total", ctypes.c_int64), ("ms_state", ctypes.c_double), ("ms_adjoint", ctypes.c_double),
                ("ms_reduce", ctypes.c_double), ("graph", ctypes.c_int), ("pad", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = ctypes.c_void_p
_SIGS = {
    "saa_abi_version": (ctypes.c_int, []),
    "saa_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "saa_options_default": (ctypes.c_int, [ctypes.POINTER(COptions)]),
    "saa_ctx_create": (ctypes.c_int, [ctypes.POINTER(CProblem), ctypes.c_int64, _P, ctypes.POINTER(_P)]),
    "saa_ctx_destroy": (None, [_P]),
    "saa_ctx_dims": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int)]),
    "saa_set_samples": (ctypes.c_int, [_P, ctypes.c_int64, _P]),
    "saa_objective_grad": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, ctypes.POINTER(COptions), _P, _P,
                                          ctypes.POINTER(CReport)]),
    "saa_per_sample": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, ctypes.POINTER(COptions), _P, _P,
                                      ctypes.POINTER(CReport)]),
    "saa_solve_states": (ctypes.c_int, [_P, _P, ctypes.POINTER(COptions), _P, _P, _P, ctypes.POINTER(CReport)]),
    "saa_sample_status": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "saa_objective_grad_multi": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                                ctypes.POINTER(COptions), _P, ctypes.POINTER(_P),
                                                ctypes.POINTER(CReport)]),
    "saa_ctx_launch3": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       ctypes.c_int]),
    "mrdino_num_params": (ctypes.c_int, [ctypes.POINTER(None), ctypes.POINTER(ctypes.c_int64)]),
    "mrdino_create": (ctypes.c_int, [ctypes.POINTER(None), _P, ctypes.POINTER(_P)]),
    "mrdino_free": (None, [_P]),
    "mrdino_set_params": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "mrdino_get_params": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "mrdino_set_qoi": (ctypes.c_int, [_P, _P, ctypes.c_double]),
    "mrdino_eval": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P]),
    "mrdino_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "mrdino_get_dims": (ctypes.c_int, [_P, _P]),
    "mrdino_load": (ctypes.c_int, [ctypes.c_char_p, _P, ctypes.POINTER(_P)]),
    "saa_ouu_options_default": (ctypes.c_int, [ctypes.POINTER(None)]),
    "saa_ouu_solve": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.POINTER(COptions), _P, _P, _P, _P, _P]),
}

_lib = None
_lib_error = None


def _load():
    global _lib, _lib_error
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        _lib_error = f"{LIB_PATH} is not built; run __graft_entry__.build() or paper_2305_20053_amd/build.py"
        raise SaaError(SAA_E_DEVICE, _lib_error)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def lib():
    """The loaded ctypes library (raises SaaError if it is not built)."""
    return _load()


def exported_symbols() -> list[str]:
    return sorted(_SIGS)


def status_str(status: int) -> str:
    return _load().saa_status_str(status).decode()


def _check(status: int, allow=(SAA_OK,)):
    if status not in allow:
        raise SaaError(status, status_str(status))
    return status


def require_gpu():
    """Raise unless the HIP library is built and a GPU is visible."""
    _load()
    import torch
    if not torch.cuda.is_available():
        raise SaaError(SAA_E_DEVICE, "no HIP device is visible")


@dataclass
class Problem:
    """Semilinear elliptic source-control problem (paper Sec. 4.2)."""
    n: int = 32
    n_src_per_dim: int = 5
    src_sigma: float = 0.05
    kl_per_dim: int = 8
    kl_shift: float = 25.0
    kl_exp: float = 1.25
    kl_amp: float = 1.0
    reaction: float = 1.0
    u_target: float = 0.5
    dim: int = 2
    target: int = 0          # TARGET_CONST (u_target), TARGET_SIN or TARGET_QUAD

    def c_struct(self) -> CProblem:
        return CProblem(self.dim, self.n, self.n_src_per_dim, self.src_sigma, self.kl_per_dim,
                        self.kl_shift, self.kl_exp, self.kl_amp, self.reaction, self.u_target, self.target, 0)

    @property
    def d_z(self) -> int:
        return self.n_src_per_dim ** self.dim

    @property
    def d_u(self) -> int:
        return (self.n - 1) ** self.dim


def problem_small(target: int = None) -> Problem:
    """n = 32 (1089 nodes), 8 x 8 KL modes: the N = 64 correctness workload;
    q = int (u - 0.5)^2 (constant target) unless `target` selects the
    sinusoidal or quadratic target of Sec. 4.2."""
    return Problem(n=32, kl_per_dim=8, target=TARGET_CONST if target is None else target)


def problem_medium(target: int = None) -> Problem:
    """n = 128 (16641 nodes), 16 x 16 KL modes: the N = 1024 PDE workload;
    constant target 0.5 unless `target` says otherwise."""
    return Problem(n=128, kl_per_dim=16, target=TARGET_CONST if target is None else target)


def objective_grad_multi(contexts, zs, opt=None):
    """J and grad of several 2D PDE-form contexts (up to 4, any sizes, one
    stream) with one state launch and one adjoint launch for all of them.
    Returns a list of (J, grad, report dict), one per context."""
    import numpy as np
    opt = opt if opt is not None else options()
    k = len(contexts)
    zz = [np.ascontiguousarray(np.asarray(z, dtype=np.float64)) for z in zs]
    grads = [np.zeros(c.d_z) for c in contexts]
    J = np.zeros(k)
    reps = (CReport * k)()
    hs = (_P * k)(*[c._h for c in contexts])
    zp = (_P * k)(*[z.ctypes.data for z in zz])
    gp = (_P * k)(*[g.ctypes.data for g in grads])
    _check(lib().saa_objective_grad_multi(k, hs, zp, ctypes.byref(opt), J.ctypes.data, gp, reps))
    return [(float(J[i]), grads[i], {name: getattr(reps[i], name) for name, _ in reps[i]._fields_})
            for i in range(k)]


def problem_3d(target: int = None) -> Problem:
    """The same equation on the unit cube: trilinear elements on 48^3 cells
    (117649 nodes), 10^3 KL modes with amplitudes (pi^2 |k|^2 + 25)^(-1.5),
    64 sources of width 0.08 on a 4 x 4 x 4 lattice; constant target 0.5
    unless `target` says otherwise.  PDE form only."""
    return Problem(dim=3, n=48, n_src_per_dim=4, src_sigma=0.08, kl_per_dim=10, kl_shift=25.0, kl_exp=1.5,
                   target=TARGET_CONST if target is None else target)


def ouu_options(**kw) -> COuuOptions:
    o = COuuOptions()
    _check(_load().saa_ouu_options_default(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown OUU option {k}")
        setattr(o, k, v)
    return o


def options(**kw) -> COptions:
    o = COptions()
    _check(_load().saa_options_default(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ptr(t) -> int:
    return t.data_ptr()


def _stream_handle():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Context:
    """A sample set of one problem with its device workspaces."""

    def __init__(self, problem: Problem, n_max: int, stream=None):
        self._lib = _load()
        self.problem = problem
        self._stream = _stream_handle() if stream is None else stream
        h = _P()
        _check(self._lib.saa_ctx_create(ctypes.byref(problem.c_struct()), n_max, _P(self._stream),
                                        ctypes.byref(h)))
        self._h = h
        du, dz, nk = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.saa_ctx_dims(h, ctypes.byref(du), ctypes.byref(dz), ctypes.byref(nk)))
        self.d_u, self.d_z, self.n_kl = du.value, dz.value, nk.value
        self.n = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.saa_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_samples(self, xi):
        """xi: float64 CUDA tensor (N, K1, K1) of KL coefficients ((N, K1, K1, K1) in 3D)."""
        xi = xi.contiguous()
        _check(self._lib.saa_set_samples(self._h, xi.shape[0], _P(_ptr(xi))))
        self.n = xi.shape[0]

    def objective_grad(self, z, form=FORM_PDE, model=None, opt=None, allow_noconv=False):
        """Returns (J, grad (numpy d_Z), report dict)."""
        import numpy as np
        opt = opt if opt is not None else options()
        zz = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        J = ctypes.c_double()
        grad = np.zeros(self.d_z)
        rep = CReport()
        st = self._lib.saa_objective_grad(self._h, zz.ctypes.data, form, _P(model.handle if model else None),
                                          ctypes.byref(opt), ctypes.byref(J), grad.ctypes.data, ctypes.byref(rep))
        _check(st, (SAA_OK, SAA_W_FALLBACK) + ((SAA_E_NOCONV,) if allow_noconv else ()))
        out = rep.as_dict()
        out["status"] = st
        return J.value, grad, out

    def per_sample(self, z, form=FORM_PDE, model=None, opt=None, allow_noconv=False):
        """Returns (q (N,), g (N, d_Z)) float64 CUDA tensors and the report."""
        import numpy as np
        import torch
        opt = opt if opt is not None else options()
        zz = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        q = torch.empty(self.n, dtype=torch.float64, device="cuda")
        g = torch.empty(self.n, self.d_z, dtype=torch.float64, device="cuda")
        rep = CReport()
        st = self._lib.saa_per_sample(self._h, zz.ctypes.data, form, _P(model.handle if model else None),
                                      ctypes.byref(opt), _P(_ptr(q)), _P(_ptr(g)), ctypes.byref(rep))
        _check(st, (SAA_OK, SAA_W_FALLBACK) + ((SAA_E_NOCONV,) if allow_noconv else ()))
        out = rep.as_dict()
        out["status"] = st
        return q, g, out

    def ouu_solve(self, z0, lb=None, ub=None, form=FORM_PDE, model=None, opt=None, **ouu):
        """Bound-constrained L-BFGS over z in [lb, ub] (host solver, device
        evaluations).  ouu: fields of saa_ouu_options.  Returns (z*, report
        dict); an evaluation failure raises."""
        import numpy as np
        opt = opt if opt is not None else options()
        oo = ouu_options(**ouu)
        z = np.ascontiguousarray(np.array(z0, dtype=np.float64))
        lbp = None if lb is None else np.ascontiguousarray(np.broadcast_to(np.asarray(lb, np.float64), (self.d_z,)))
        ubp = None if ub is None else np.ascontiguousarray(np.broadcast_to(np.asarray(ub, np.float64), (self.d_z,)))
        rep = COuuReport()
        st = self._lib.saa_ouu_solve(self._h, form, _P(model.handle if model else None), ctypes.byref(opt),
                                     ctypes.byref(oo), None if lbp is None else lbp.ctypes.data,
                                     None if ubp is None else ubp.ctypes.data, z.ctypes.data, ctypes.byref(rep))
        _check(st)
        return z, {name: getattr(rep, name) for name, _ in rep._fields_}

    def sample_status(self):
        """Per-sample (flags, newton_iters, lin_iters, adj_lin_iters) of the last call (numpy int32)."""
        import numpy as np
        arrs = [np.zeros(self.n, dtype=np.int32) for _ in range(4)]
        _check(self._lib.saa_sample_status(self._h, *[a.ctypes.data for a in arrs]))
        return tuple(arrs)

    def launch3(self, prec=FP32_DC64, state=None, adjoint=None):
        """3D contexts: threads per sample of the state / adjoint kernels for
        `prec`.  With no sizes given returns the recorded (state, adjoint)
        pair (0: chosen by timing at the next call); otherwise installs them
        (256, 512, 1024, or 0 to time again)."""
        a, b = ctypes.c_int(state or 0), ctypes.c_int(adjoint or 0)
        setting = state is not None or adjoint is not None
        _check(self._lib.saa_ctx_launch3(self._h, prec, ctypes.byref(a), ctypes.byref(b), 1 if setting else 0))
        return a.value, b.value

    def solve_states(self, Z, want_dudz=False, opt=None):
        """Z: float64 CUDA tensor (N, d_Z).  Returns (u (N, d_U), q (N,),
        dudz (N, d_Z, d_U) or None, report)."""
        import torch
        opt = opt if opt is not None else options()
        Z = Z.contiguous()
        u = torch.empty(self.n, self.d_u, dtype=torch.float64, device="cuda")
        q = torch.empty(self.n, dtype=torch.float64, device="cuda")
        dudz = (torch.empty(self.n, self.d_z, self.d_u, dtype=torch.float64, device="cuda")
                if want_dudz else None)
        rep = CReport()
        _check(self._lib.saa_solve_states(self._h, _P(_ptr(Z)), ctypes.byref(opt), _P(_ptr(u)), _P(_ptr(q)),
                                          _P(_ptr(dudz)) if want_dudz else None, ctypes.byref(rep)))
        return u, q, dudz, rep.as_dict()


class Model:
    """MR-DINO network (Sec. 3.3): FP32 parameters on the device plus the
    reduced-QoI terms c, c0."""

    def __init__(self, r_m=100, d_z=25, r_u=200, width=256, depth=4, stream=None):
        self._lib = _load()
        self.dims = CDims(r_m, d_z, r_u, width, depth)
        n = ctypes.c_int64()
        _check(self._lib.mrdino_num_params(ctypes.byref(self.dims), ctypes.byref(n)))
        self.n_params = n.value
        h = _P()
        st = _stream_handle() if stream is None else stream
        _check(self._lib.mrdino_create(ctypes.byref(self.dims), _P(st), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h.value

    def widths(self):
        d = self.dims
        return [d.r_m + d.d_z] + [d.width] * d.depth + [d.r_u]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mrdino_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        """flat: float32-convertible vector in the packed order of include/saa.h."""
        import numpy as np
        p = np.ascontiguousarray(np.asarray(flat, dtype=np.float32))
        _check(self._lib.mrdino_set_params(self._h, p.ctypes.data, p.size))

    def get_params(self):
        import numpy as np
        p = np.zeros(self.n_params, dtype=np.float32)
        _check(self._lib.mrdino_get_params(self._h, p.ctypes.data, p.size))
        return p

    def set_qoi(self, c, c0):
        import numpy as np
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        _check(self._lib.mrdino_set_qoi(self._h, cc.ctypes.data, float(c0)))

    def save(self, path):
        _check(self._lib.mrdino_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path, stream=None):
        lib = _load()
        h = _P()
        st = _stream_handle() if stream is None else stream
        _check(lib.mrdino_load(os.fsencode(path), _P(st), ctypes.byref(h)))
        d = CDims()
        self = cls.__new__(cls)
        self._lib = lib
        self._h = h
        _check(lib.mrdino_get_dims(h, ctypes.byref(d)))
        self.dims = d
        n = ctypes.c_int64()
        _check(lib.mrdino_num_params(ctypes.byref(d), ctypes.byref(n)))
        self.n_params = n.value
        return self

    def eval(self, ctx, z, want=WANT_Q | WANT_DQDZ | WANT_PHI | WANT_DPHIDZ, prec=FP32):
        """mrdino_eval on ctx's samples: dict of CUDA tensors q (N,), dqdz
        (N, d_Z) float64, phi (N, r_u), dphidz (N, d_Z, r_u) float32."""
        import numpy as np
        import torch
        d, n = self.dims, ctx.n
        zz = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        out = {}
        if want & WANT_Q:
            out["q"] = torch.empty(n, dtype=torch.float64, device="cuda")
        if want & WANT_DQDZ:
            out["dqdz"] = torch.empty(n, d.d_z, dtype=torch.float64, device="cuda")
        if want & WANT_PHI:
            out["phi"] = torch.empty(n, d.r_u, dtype=torch.float32, device="cuda")
        if want & WANT_DPHIDZ:
            out["dphidz"] = torch.empty(n, d.d_z, d.r_u, dtype=torch.float32, device="cuda")
        ptr = [_P(_ptr(out[k])) if k in out else _P(None) for k in ("q", "dqdz", "phi", "dphidz")]
        _check(self._lib.mrdino_eval(self._h, ctx.handle, zz.ctypes.data, want, prec, *ptr))
        return out


class CTrainCfg(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int), ("epochs", ctypes.c_int), ("lr_drop_epoch", ctypes.c_int),
                ("lr", ctypes.c_double), ("lr_late", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("adam_eps", ctypes.c_double), ("dino", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("prec", ctypes.c_int), ("resume", ctypes.c_int)]


_SIGS.update({
    "mrdino_data_create": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(COptions), _P, ctypes.POINTER(_P), ctypes.POINTER(CReport)]),
    "mrdino_data_free": (None, [_P]),
    "mrdino_data_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), _P, ctypes.POINTER(ctypes.c_double), _P]),
    "mrdino_data_qoi": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_double)]),
    "mrdino_data_get": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int64]),
    "mrdino_loss_grad": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double), _P]),
    "mrdino_train": (ctypes.c_int, [_P, _P, ctypes.POINTER(CTrainCfg), _P, ctypes.POINTER(ctypes.c_double)]),
    "mrdino_data_errors": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "saa_sym_eig": (ctypes.c_int, [ctypes.c_int, _P, _P, _P]),
    "saa_sym_eig_gpu": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int)]),
    "saa_attach_holdout": (ctypes.c_int, [_P, _P]),
    "saa_tune_get": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]),
    "saa_tune_set": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int]),
    "saa_risk_reduce": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int, _P, ctypes.POINTER(COptions), _P, _P,
                                       _P]),
    "saa_risk_reduce_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int, _P, ctypes.POINTER(COptions),
                                               _P, _P, _P]),
})


def risk_reduce(q, g, z, opt=None, noalloc=False):
    """Risk reduction alone over per-sample values already on the device:
    q (N,) and g (N, d_Z) float64 CUDA tensors, z (d_Z) host array.  Returns
    (J, dJ/dt, grad (numpy d_Z), t) from saa_risk_reduce, or from
    saa_risk_reduce_noalloc (static workspace, no allocation) with noalloc."""
    import numpy as np
    import torch
    opt = opt if opt is not None else options()
    q = q.contiguous()
    g = g.contiguous()
    N, dz = g.shape
    zd = torch.as_tensor(np.asarray(z, dtype=np.float64)).to(q.device)
    out = torch.empty(2 + dz, dtype=torch.float64, device=q.device)
    t = torch.empty(1, dtype=torch.float64, device=q.device)
    fn = _load().saa_risk_reduce_noalloc if noalloc else _load().saa_risk_reduce
    _check(fn(_P(_ptr(q)), _P(_ptr(g)), N, dz, _P(_ptr(zd)), ctypes.byref(opt), _P(_ptr(out)), _P(_ptr(t)),
              _P(torch.cuda.current_stream().cuda_stream)))
    o = out.cpu().numpy()
    return float(o[0]), float(o[1]), o[2:].copy(), float(t.item())


def tune_get(key: str):
    """The autotuner's recorded choice for `key` on this device, or None."""
    v = ctypes.c_int()
    st = _load().saa_tune_get(key.encode(), ctypes.byref(v))
    return v.value if st == SAA_OK else None


def tune_set(key: str, value: int):
    """Record a launch-shape choice (see include/saa.h for the keys)."""
    _check(_load().saa_tune_set(key.encode(), int(value)))


def attach_holdout(ctx: Context, holdout):
    """Attach (or, with None, detach) held-out samples for the surrogate error
    estimate and PDE fallback of MR-DINO evaluations."""
    _check(_load().saa_attach_holdout(ctx.handle, holdout.handle if holdout is not None else None))


def sym_eig(A):
    """Eigenvalues (decreasing) and eigenvectors (columns) of a symmetric
    matrix by the library's host eigensolver (no GPU needed)."""
    import numpy as np
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n))
    _check(_load().saa_sym_eig(n, A.ctypes.data, w.ctypes.data, V.ctypes.data))
    return w, V


def sym_eig_gpu(A):
    """Eigenvalues (decreasing, numpy) and eigenvectors (columns, CUDA
    tensor) of a symmetric CUDA float64 tensor by the library's GPU Jacobi
    solver; also returns the number of sweeps."""
    import numpy as np
    import torch
    A = A.contiguous()
    n = A.shape[0]
    w = np.zeros(n)
    V = torch.empty(n, n, dtype=torch.float64, device=A.device)
    sw = ctypes.c_int()
    _check(_load().saa_sym_eig_gpu(n, _P(_ptr(A)), w.ctypes.data, _P(_ptr(V)),
                                   _P(torch.cuda.current_stream().cuda_stream), ctypes.byref(sw)))
    return w, V, sw.value


def init_params(layers, out_scale=1.0):
    """Packed FP32 parameters of a list of (W, b) layers with the output
    layer multiplied by out_scale (e.g. TrainData.output_scale())."""
    import numpy as np
    parts = []
    for k, (W, b) in enumerate(layers):
        f = out_scale if k == len(layers) - 1 else 1.0
        parts.append(np.concatenate([np.ravel(W) * f, np.asarray(b) * f]))
    return np.concatenate(parts).astype(np.float32)


def train_cfg(batch=256, epochs=1600, lr_drop_epoch=800, lr=1e-3, lr_late=2.5e-4, dino=1, seed=2305,
              beta1=0.9, beta2=0.999, adam_eps=1e-8, prec=None, resume=0) -> CTrainCfg:
    """Adam schedule of Sec. 4.2.1 (lr 1e-3, 2.5e-4 after 800 of 1600 epochs);
    products in BF16 with FP32 accumulation unless prec = FP32; resume = 1
    continues the model's optimiser state."""
    return CTrainCfg(batch, epochs, lr_drop_epoch, lr, lr_late, beta1, beta2, adam_eps, dino, seed,
                     BF16 if prec is None else prec, resume)


class TrainData:
    """Reduced training data built on the GPU from the PDE form (Sec. 3.3-3.4)."""

    def __init__(self, ctx: Context, Z, r_m=100, r_u=200, n_pod=512, opt=None, basis=None):
        """basis: another TrainData whose POD basis is reused (held-out data)."""
        self._lib = _load()
        opt = opt if opt is not None else options()
        Z = Z.contiguous()
        h = _P()
        rep = CReport()
        _check(self._lib.mrdino_data_create(ctx.handle, _P(_ptr(Z)), r_m, r_u, n_pod, ctypes.byref(opt),
                                            _P(basis.handle if basis is not None else None), ctypes.byref(h),
                                            ctypes.byref(rep)))
        if basis is not None:
            n_pod = basis.n_pod
        self._h = h
        self.report = rep.as_dict()
        self.r_m, self.r_u, self.n_pod, self.d_z, self.d_u = r_m, r_u, n_pod, ctx.d_z, ctx.d_u
        n = ctypes.c_int64()
        _check(self._lib.mrdino_data_info(h, ctypes.byref(n), None, None, None))
        self.n = n.value

    @property
    def handle(self):
        return self._h.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mrdino_data_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        """(c, c0, eigenvalues of the POD Gram matrix)."""
        import numpy as np
        c = np.zeros(self.r_u)
        lam = np.zeros(self.n_pod)
        c0 = ctypes.c_double()
        _check(self._lib.mrdino_data_info(self._h, None, c.ctypes.data, ctypes.byref(c0), lam.ctypes.data))
        return c, c0.value, lam

    def qoi(self, target: int, u_target: float = 0.5):
        """(c, c0) of the tracking QoI for another target with this POD basis."""
        import numpy as np
        c = np.zeros(self.r_u)
        c0 = ctypes.c_double()
        _check(self._lib.mrdino_data_qoi(self._h, target, u_target, c.ctypes.data, ctypes.byref(c0)))
        return c, c0.value

    def output_scale(self):
        """The output scale sigma of training on this data: the RMS of the
        reduced states rounded to a power of two (mrdino_train trains the
        output layer as phi = sigma phi').  A fresh network whose output
        layer is multiplied by sigma starts at the scale of the targets."""
        import numpy as np
        y = self.get("Y").astype(np.float64)
        rms = float(np.sqrt(np.mean(y * y)))
        return float(2.0 ** round(np.log2(rms))) if rms > 0 and np.isfinite(rms) else 1.0

    def get(self, which: str):
        """'X', 'Y', 'J' (float32) or 'PhiT', 'ubar' (float64) as numpy arrays."""
        import numpy as np
        shapes = {"X": ((self.n, self.r_m + self.d_z), np.float32, 0), "Y": ((self.n, self.r_u), np.float32, 1),
                  "J": ((self.n * self.d_z, self.r_u), np.float32, 2),
                  "PhiT": ((self.r_u, self.d_u), np.float64, 3), "ubar": ((self.d_u,), np.float64, 4)}
        shape, dt, code = shapes[which]
        a = np.zeros(shape, dtype=dt)
        _check(self._lib.mrdino_data_get(self._h, code, a.ctypes.data, a.size))
        return a


def loss_grad(model: Model, data: TrainData, idx, dino=True, want_grad=True, prec=None):
    """Batch loss and gradient (packed order) of the rows idx; products in
    FP32 (default) or BF16 (prec = BF16, the training precision)."""
    import numpy as np
    ii = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    loss = ctypes.c_double()
    g = np.zeros(model.n_params, dtype=np.float32) if want_grad else None
    _check(_load().mrdino_loss_grad(model._h, data.handle, ii.ctypes.data, ii.size, int(dino),
                                    FP32 if prec is None else prec, ctypes.byref(loss),
                                    g.ctypes.data if want_grad else None))
    return loss.value, g


def train(model: Model, data: TrainData, cfg: CTrainCfg):
    """Run Adam training; returns (per-epoch mean loss, device seconds)."""
    import numpy as np
    hist = np.zeros(max(1, cfg.epochs))
    sec = ctypes.c_double()
    _check(_load().mrdino_train(model._h, data.handle, ctypes.byref(cfg), hist.ctypes.data, ctypes.byref(sec)))
    return hist[:cfg.epochs], sec.value


def data_errors(model: Model, data: TrainData):
    """(relative reduced state error, relative reduced Jacobian error)."""
    es, ej = ctypes.c_double(), ctypes.c_double()
    _check(_load().mrdino_data_errors(model._h, data.handle, ctypes.byref(es), ctypes.byref(ej)))
    return es.value, ej.value


def _autograd_functions():
    """torch.autograd.Function wrappers (built lazily: importing the package
    must not require torch)."""
    import numpy as np
    import torch

    class Objective(torch.autograd.Function):
        """J(z) as a differentiable function of the host control z (float64
        CPU tensor); the backward is the library's gradient (Sec. 2.3)."""

        @staticmethod
        def forward(fctx, z, sctx, form, model, opt):
            J, g, _ = sctx.objective_grad(z.detach().cpu().numpy(), form=form, model=model, opt=opt)
            fctx.save_for_backward(torch.from_numpy(g))
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(fctx, gJ):
            (g,) = fctx.saved_tensors
            return gJ * g, None, None, None, None

    class DinoLoss(torch.autograd.Function):
        """Derivative-informed training loss (Sec. 3.4) of the rows idx of a
        TrainData as a function of the packed FP32 parameters (CPU tensor);
        the backward is the hand-written gradient kernel."""

        @staticmethod
        def forward(fctx, params, model, data, idx, dino):
            p = params.detach().cpu().numpy().astype(np.float32)
            model.set_params(p)
            loss, g = loss_grad(model, data, idx, dino=dino)
            fctx.save_for_backward(torch.from_numpy(g))
            return torch.tensor(loss, dtype=torch.float64)

        @staticmethod
        def backward(fctx, gL):
            (g,) = fctx.saved_tensors
            return (gL * g.double()).to(torch.float32), None, None, None, None

    return Objective, DinoLoss


def objective(z, ctx: Context, form=FORM_PDE, model=None, opt=None):
    """Differentiable J(z): z is a float64 CPU tensor of d_Z controls."""
    return _autograd_functions()[0].apply(z, ctx, form, model, opt)


def dino_loss(params, model: Model, data: TrainData, idx, dino=True):
    """Differentiable training loss of the rows idx at the packed FP32
    parameters `params` (CPU tensor); sets the model's parameters."""
    return _autograd_functions()[1].apply(params, model, data, idx, dino)
