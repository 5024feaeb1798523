"""The C-ABI library builds, loads and exports every symbol include/gf.h
declares; argument validation runs on the host and needs no GPU."""
import os
import re

import pytest

import paper_1205_0752_amd as gf
from paper_1205_0752_amd import build as gfbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "gf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gf.LIB_PATH):
        gfbuild.build()
    return gf.load()


def test_every_declared_symbol_is_exported(lib):
    decl = _declared()
    assert set(decl) == set(gf.EXPORTS)
    for name in decl:
        assert hasattr(lib, name), name


def test_version(lib):
    assert "gfx950" in gf.version()


@pytest.mark.parametrize("params, quad, msg", [
    (gf.Params(-1.0, 1.0, 1.0, 1e4), gf.Quadrature(), "m1^2"),
    (gf.Params(1.0, 0.0, 1.0, 1e4), gf.Quadrature(), "m2^2"),
    (gf.Params(1.0, 1.0, -1.0, 1e4), gf.Quadrature(), "mu2"),
    (gf.Params(1.0, 1.0, 1.0, 0.0), gf.Quadrature(), "lambda2"),
    (gf.Params(1.0, 1.0, 1.0, float("inf")), gf.Quadrature(), "finite"),
    (gf.Params(1.0, 1.0, 1.0, 1e4), gf.Quadrature(0, 32, 16), "n_radial"),
    (gf.Params(1.0, 1.0, 1.0, 1e4), gf.Quadrature(64, 9000, 16), "n_angular"),
    (gf.Params(1.0, 1.0, 1.0, 1e4), gf.Quadrature(64, 32, -1), "n_arc"),
    (gf.Params(1.0, 1.0, 1.0, 1e4), gf.Quadrature(64, 32, 0), "n_arc"),
    (gf.Params(1.0, 1.0, 1.0, 1e4), gf.Quadrature(64, 32, 16, 7), "precision"),
])
def test_plan_validation_before_any_device_call(lib, params, quad, msg):
    with pytest.raises(gf.GFError) as e:
        gf.Plan(params, quad)
    assert e.value.code == -1 and msg in str(e.value)


def test_one_call_scan_validates_first(lib):
    with pytest.raises(gf.GFError) as e:
        gf.scan(gf.Params(1.0, 1.0, 1.0, -5.0), gf.Grid(2, 2, -1, 1, -1, 1), gf.Quadrature(),
                out=_FakeTensor(), stream=0)
    assert e.value.code == -1


class _FakeTensor:
    def data_ptr(self):
        return 0


def test_workload_generators_are_seeded():
    from paper_1205_0752_amd.workloads import serving_trace, sample_points, CONFIGS
    a = serving_trace(50, 10.0, seed=3)
    b = serving_trace(50, 10.0, seed=3)
    assert a == b
    assert all(r.grid.n_re in range(16, 513, 16) for r in a)
    g = CONFIGS["c1_fp64_1024sq"][1]
    assert (sample_points(g, 100, 4) == sample_points(g, 100, 4)).all()
