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
    # straight through the C ABI: invalid parameters are rejected before the
    # output pointer or any device is looked at
    from paper_1205_0752_amd._binding import c_grid, c_params, c_quad
    import ctypes
    rc = lib.gf_scan(ctypes.byref(c_params(gf.Params(1.0, 1.0, 1.0, -5.0))),
                     ctypes.byref(c_grid(gf.Grid(2, 2, -1, 1, -1, 1))),
                     ctypes.byref(c_quad(gf.Quadrature())), None, None)
    assert rc == -1 and "lambda2" in lib.gf_last_error().decode()


# ---- output buffers are checked in Python before the library sees their address


class _FakePlan:
    device = 0
    handle = None  # never reached: the checks raise first


def _t(shape, dtype, **kw):
    import torch
    return torch.zeros(shape, dtype=dtype, **kw)


@pytest.mark.parametrize("make, msg", [
    (lambda torch: _t((4, 6), torch.complex64), "dtype"),
    (lambda torch: _t((4, 5), torch.complex128), "elements"),
    (lambda torch: _t((6, 4), torch.complex128).t(), "contiguous"),
    (lambda torch: _t((4, 6), torch.complex128), "GPU"),
    (lambda torch: "not a tensor", "torch tensor"),
])
def test_scan_output_checked_before_launch(make, msg):
    import torch
    with pytest.raises(ValueError, match=msg):
        gf.scan_plan(_FakePlan(), gf.Grid(6, 4, -1, 1, -1, 1), out=make(torch))
    with pytest.raises(ValueError, match=msg):
        gf.yscan_plan(_FakePlan(), 1.0 + 1.0j, gf.Grid(6, 4, -1, 1, -1, 1), out=make(torch))


def test_class_map_checked_before_launch():
    import torch
    out = _t((4, 6), torch.complex128, device="meta")
    # a meta tensor passes dtype, size and contiguity but not the device check
    with pytest.raises(ValueError, match="GPU"):
        gf.scan_plan(_FakePlan(), gf.Grid(6, 4, -1, 1, -1, 1), out=out)
    with pytest.raises(ValueError, match="cls must have dtype"):
        gf.scan_plan(_FakePlan(), gf.Grid(6, 4, -1, 1, -1, 1),
                     out=_t((4, 6), torch.complex128), cls=_t((4, 6), torch.uint8))


def test_one_call_scan_and_obstruction_map_check_outputs(monkeypatch):
    import torch
    from paper_1205_0752_amd import _binding
    monkeypatch.setattr(_binding, "_current_device", lambda: 0)
    g = gf.Grid(6, 4, -1, 1, -1, 1)
    with pytest.raises(ValueError, match="dtype"):
        gf.scan(gf.Params(1.0, 1.0, 1.0, 1e4), g, gf.Quadrature(), out=_t((4, 6), torch.float64))
    with pytest.raises(ValueError, match="GPU"):
        gf.obstruction_map(gf.Params(1.0, 1.0, 1.0, 1e4), g, out=_t((4, 6), torch.uint8))
    with pytest.raises(ValueError, match="dtype"):
        gf.obstruction_map(gf.Params(1.0, 1.0, 1.0, 1e4), g, out=_t((4, 6), torch.int8))


def test_workload_generators_are_seeded():
    from paper_1205_0752_amd.workloads import serving_trace, sample_points, CONFIGS
    a = serving_trace(50, 10.0, seed=3)
    b = serving_trace(50, 10.0, seed=3)
    assert a == b
    assert all(r.grid.n_re in range(16, 513, 16) for r in a)
    g = CONFIGS["c1_fp64_1024sq"][1]
    assert (sample_points(g, 100, 4) == sample_points(g, 100, 4)).all()
