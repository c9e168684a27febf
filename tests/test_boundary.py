"""Host-side checks of the C-ABI boundary (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2305_20053_amd as saa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, re.M):
            name = m.group(1)
            if name.startswith(("saa_", "mrdino_")):
                names.add(name)
    return names


def test_library_exports_every_declared_symbol():
    lib = saa.lib()
    declared = _declared_functions()
    assert len(declared) >= 9
    out = subprocess.run(["nm", "-D", "--defined-only", saa.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = declared - exported
    assert not missing, missing
    for name in declared:
        getattr(lib, name)
    assert set(saa.exported_symbols()) <= exported


def test_status_strings_and_version():
    lib = saa.lib()
    assert lib.saa_abi_version() == 3
    for st in (0, 1, -1, -2, -3, -4, -5, -6):
        assert saa.status_str(st) and saa.status_str(st) != "unknown status"
    assert saa.status_str(12345) == "unknown status"


def test_options_default():
    o = saa.options()
    assert o.beta == 0.95 and o.eps == 1e-4 and o.alpha == 1e-3 and o.prec == saa.FP32_DC64
    assert saa.lib().saa_options_default(None) == saa.SAA_E_INVALID


@pytest.mark.parametrize("field,value", [("n", 3), ("n", 80), ("n", 40), ("n", 0), ("dim", 3), ("n_src_per_dim", 0),
                                         ("src_sigma", 0.0), ("src_sigma", float("nan")), ("kl_per_dim", 0),
                                         ("kl_exp", -1.0), ("reaction", -1.0), ("u_target", float("inf")),
                                         ("kl_per_dim", 65), ("target", 3), ("target", -1)])
def test_ctx_create_rejects_bad_problem_before_device_work(field, value):
    p = saa.problem_small()
    setattr(p, field, value)
    h = ctypes.c_void_p()
    st = saa.lib().saa_ctx_create(ctypes.byref(p.c_struct()), 16, None, ctypes.byref(h))
    assert st == saa.SAA_E_INVALID and not h.value


@pytest.mark.parametrize("field,value", [("n", 47), ("n", 36), ("n", 98), ("n", 2), ("n_src_per_dim", 5),
                                         ("kl_per_dim", 17), ("kl_per_dim", 0), ("src_sigma", -0.1),
                                         ("target", 7), ("dim", 4)])
def test_ctx_create_rejects_bad_3d_problem_before_device_work(field, value):
    """3D: n even in [4, 96] halving to a coarsest grid of at most 7 cells
    (n = 36 stops at 9), at most 4 sources per dimension (64 controls), K1 in
    1..16."""
    p = saa.problem_3d()
    setattr(p, field, value)
    h = ctypes.c_void_p()
    st = saa.lib().saa_ctx_create(ctypes.byref(p.c_struct()), 16, None, ctypes.byref(h))
    assert st == saa.SAA_E_INVALID and not h.value
    st = saa.lib().saa_ctx_create(ctypes.byref(saa.problem_3d().c_struct()), (1 << 20) + 1, None, ctypes.byref(h))
    assert st == saa.SAA_E_INVALID and not h.value


@pytest.mark.parametrize("dim,n,n_max,ok", [(2, 32, 4194303, True), (2, 32, 4194304, False), (2, 4, 1 << 24, False),
                                            (3, 16, 986895, True), (3, 16, 986896, False), (3, 96, 172960, True),
                                            (3, 96, 172961, False), (3, 4, 1 << 20, True), (3, 4, (1 << 20) + 1, False)])
def test_sample_count_cap_fits_every_launch_grid(dim, n, n_max, ok):
    """N_max is capped so that every kernel's grid (2D: one 1024-thread
    workgroup per sample; 3D: N (n + 1) workgroups of 256 threads for the
    field) stays within 2^32 - 1 work-items.  Accepted counts are checked by
    the bound itself (creating such a context needs a GPU); refused ones must
    fail before any device work."""
    if dim == 2:
        bound = ((1 << 32) - 1) // 1024
        p = saa.Problem(n=n, kl_per_dim=4)
    else:
        bound = min(1 << 20, ((1 << 32) - 1) // (256 * (n + 1)))
        p = saa.Problem(dim=3, n=n, n_src_per_dim=2, src_sigma=0.08, kl_per_dim=3, kl_exp=1.5)
    assert (n_max <= bound) == ok
    if not ok:
        h = ctypes.c_void_p()
        st = saa.lib().saa_ctx_create(ctypes.byref(p.c_struct()), n_max, None, ctypes.byref(h))
        assert st == saa.SAA_E_INVALID and not h.value


def test_multi_rejects_bad_arguments_before_device_work():
    lib = saa.lib()
    J = (ctypes.c_double * 4)()
    o = saa.options()
    for count in (0, 5, -1):
        assert lib.saa_objective_grad_multi(count, None, None, ctypes.byref(o), ctypes.cast(J, ctypes.c_void_p),
                                            None, None) == saa.SAA_E_INVALID
    hs = (ctypes.c_void_p * 1)(None)
    zp = (ctypes.c_void_p * 1)(None)
    assert lib.saa_objective_grad_multi(1, hs, zp, ctypes.byref(o), ctypes.cast(J, ctypes.c_void_p), zp,
                                        None) == saa.SAA_E_INVALID


def test_launch3_rejects_without_context():
    a, b = ctypes.c_int(512), ctypes.c_int(512)
    assert saa.lib().saa_ctx_launch3(None, saa.FP32_DC64, ctypes.byref(a), ctypes.byref(b), 1) == saa.SAA_E_INVALID


def test_null_arguments_rejected():
    lib = saa.lib()
    p = saa.problem_small().c_struct()
    assert lib.saa_ctx_create(None, 4, None, ctypes.byref(ctypes.c_void_p())) == saa.SAA_E_INVALID
    assert lib.saa_ctx_create(ctypes.byref(p), 4, None, None) == saa.SAA_E_INVALID
    assert lib.saa_ctx_create(ctypes.byref(p), 0, None, ctypes.byref(ctypes.c_void_p())) == saa.SAA_E_INVALID
    assert lib.saa_set_samples(None, 4, None) == saa.SAA_E_INVALID
    o = saa.options()
    J = ctypes.c_double()
    assert lib.saa_objective_grad(None, None, 0, None, ctypes.byref(o), ctypes.byref(J), None,
                                  None) == saa.SAA_E_INVALID
    assert lib.saa_per_sample(None, None, 0, None, ctypes.byref(o), None, None, None) == saa.SAA_E_INVALID
    assert lib.saa_solve_states(None, None, ctypes.byref(o), None, None, None, None) == saa.SAA_E_INVALID
    assert lib.saa_sample_status(None, None, None, None, None) == saa.SAA_E_INVALID
    lib.saa_ctx_destroy(None)


def test_model_file_rejected_before_device_work(tmp_path):
    """mrdino_load validates the whole file (magic, version, dimensions, size,
    FNV-1a hash) before any device allocation."""
    lib = saa.lib()
    h = ctypes.c_void_p()
    missing = os.fsencode(str(tmp_path / "missing.bin"))
    assert lib.mrdino_load(missing, None, ctypes.byref(h)) == saa.SAA_E_IO and not h.value
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"SAADINO1" + b"\0" * 64)
    assert lib.mrdino_load(os.fsencode(str(bad)), None, ctypes.byref(h)) == saa.SAA_E_IO and not h.value
    bad.write_bytes(b"NOTAMODEL")
    assert lib.mrdino_load(os.fsencode(str(bad)), None, ctypes.byref(h)) == saa.SAA_E_IO and not h.value
    assert lib.mrdino_load(None, None, ctypes.byref(h)) == saa.SAA_E_INVALID
    assert lib.mrdino_save(None, os.fsencode(str(bad))) == saa.SAA_E_INVALID
    assert lib.mrdino_eval(None, None, None, 1, saa.FP32, None, None, None, None) == saa.SAA_E_INVALID
    assert lib.mrdino_get_dims(None, None) == saa.SAA_E_INVALID
