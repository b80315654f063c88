"""C-ABI library: loads, exports every symbol the header declares, and
rejects bad arguments before touching the GPU (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lindblad.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"defined"})


@pytest.fixture(scope="module")
def L():
    from paper_2603_18052_amd import lindblad
    return lindblad.lib()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("lindblad_liouvillian", "lindblad_propagator", "lindblad_propagate", "grape_gradient",
              "lindblad_generators", "lindblad_propagate_baseline", "lindblad_batch_run",
              "lb_workspace_create", "lb_workspace_destroy", "lindblad_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2603_18052_amd import lindblad
    assert set(declared_functions()) <= set(lindblad.SYMBOLS)


def test_validation_errors_without_gpu(L):
    from paper_2603_18052_amd import lindblad as lb
    assert L.lindblad_liouvillian(0, None, 0, None, None, None) == lb.ESHAPE
    assert "d must be" in lb.last_error()
    assert L.lindblad_liouvillian(3, None, 0, None, None, None) == lb.EINVAL
    assert L.lindblad_liouvillian(3, 1, 70, 1, 1, None) == lb.ESHAPE
    assert L.lindblad_generators(0, 1, 1, 1, 1, 1, 1, None) == lb.ESHAPE
    assert L.lindblad_generators(9, -1, 1, 1, 1, 1, 1, None) == lb.ESHAPE
    dts = (ctypes.c_double * 1)(0.5)
    assert L.lindblad_propagator(0, 1, 1, dts, 0.25, 1, None, None, None) == lb.ESHAPE
    assert L.lindblad_propagator(9, 0, 1, dts, 0.25, 1, None, None, None) == lb.ESHAPE
    assert L.lindblad_propagator(9, 1, None, dts, 0.25, 1, None, None, None) == lb.EINVAL
    assert L.lindblad_propagator(9, 1, 1, dts, 0.0, 1, None, None, None) == lb.EINVAL
    bad = (ctypes.c_double * 1)(float("nan"))
    assert L.lindblad_propagator(9, 1, 1, bad, 0.25, 1, None, None, None) == lb.EINVAL
    assert L.lindblad_propagate(9, 1, 0, 0, 1, 1, None, None) == lb.ESHAPE
    assert L.lindblad_propagate(9, 1, 0, 1, 1, -1, None, None) == lb.EINVAL
    assert L.lindblad_propagate(9, 1, 9, 1, 1, 1, None, None) == lb.EINVAL
    assert L.lindblad_propagate(9, None, 0, 1, 1, 1, None, None) == lb.EINVAL
    assert L.lindblad_propagate_baseline(5000, 1, 1, 1, 1, None, None) == lb.ESHAPE


def test_workspace_lifecycle(L):
    h = ctypes.c_void_p()
    assert L.lb_workspace_create(1 << 20, ctypes.byref(h)) == 0
    assert L.lb_workspace_bytes(h) == 0
    assert L.lb_workspace_destroy(h) == 0
    assert L.lb_workspace_create(1 << 20, None) == -1
