"""The library path has no CPU fallback and never reaches the oracle.

The package's sources (binding, HIP kernels, host runtime) must not import
or reference the oracle, and every entry point must raise when the shared
library is absent instead of computing anything on the host.
"""
import os
import re

import pytest

import paper_2305_20053_amd as saa

PKG = os.path.dirname(os.path.abspath(saa.__file__))


def _package_sources():
    for root, dirs, files in os.walk(PKG):
        dirs[:] = [d for d in dirs if d not in ("_build", "__pycache__")]
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                yield os.path.join(root, f)


def test_package_sources_do_not_reference_the_oracle():
    srcs = list(_package_sources())
    assert any(p.endswith("pde.hip") for p in srcs) and any(p.endswith("__init__.py") for p in srcs)
    pat = re.compile(r"\boracle\b")
    hits = [p for p in srcs if pat.search(open(p, encoding="utf-8").read())]
    assert not hits, hits


def test_entry_points_raise_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(saa, "_lib", None)
    monkeypatch.setattr(saa, "LIB_PATH", str(tmp_path / "libsaa.so"))
    with pytest.raises(saa.SaaError, match="not built"):
        saa.lib()
    with pytest.raises(saa.SaaError):
        saa.options()
    with pytest.raises(saa.SaaError):
        saa.require_gpu()
    with pytest.raises(saa.SaaError):
        saa.Context(saa.problem_small(), 4)
    with pytest.raises(saa.SaaError):
        saa.sym_eig([[2.0, 0.0], [0.0, 1.0]])
