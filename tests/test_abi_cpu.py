"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point declared in include/gravity.h, and rejects malformed
descriptors with the documented status codes before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "gravity.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gravity_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def gl():
    import paper_2001_02765_amd as m
    return m


def test_exports_every_declared_symbol(gl):
    names = _header_functions()
    assert len(names) >= 9
    lib = ctypes.CDLL(gl.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(gl.SYMBOLS)


def test_descriptor_validation_without_device(gl):
    cases = [
        (dict(n0=48), gl.EUNSUPPORTED),                                     # not a power of two
        (dict(n0=8192), gl.EUNSUPPORTED),                                   # finest lattice too large
        (dict(n0=8), gl.EUNSUPPORTED),                                      # too small
        (dict(n0=32, nlevels=2, patches=[(1, 1, 0, 4, 4)]), gl.EINVAL),     # odd corner
        (dict(n0=32, nlevels=2, patches=[(2, 0, 0, 4, 4)]), gl.EINVAL),     # level out of range
        (dict(n0=32, nlevels=2, patches=[(1, 60, 0, 8, 8)]), gl.EINVAL),    # outside the domain
        (dict(n0=32, nlevels=3, patches=[(2, 0, 0, 8, 8)]), gl.EINVAL),     # not nested
        (dict(n0=32, nlevels=2, patches=[(1, 0, 0, 8, 8), (1, 4, 4, 8, 8)]), gl.EINVAL),  # overlap
        (dict(n0=32, nlevels=1, patches=[(1, 0, 0, 8, 8)]), gl.EINVAL),     # patches on a uniform grid
        (dict(n0=32, h0=-1.0), gl.EINVAL),                                  # bad geometry
    ]
    for kw, st in cases:
        with pytest.raises(gl.GravityError) as e:
            gl.Plan(**kw)
        assert e.value.status == st, (kw, e.value)
        assert len(gl._lib.gravity_last_error()) > 0


def test_null_arguments(gl):
    b = ctypes.c_size_t()
    assert gl._lib.gravity_plan_workspace_bytes(None, ctypes.byref(b)) == gl.EINVAL
    assert gl._lib.gravity_plan(None, None) == gl.EINVAL
    assert gl._lib.gravity_batch_workspace_bytes(-1, None, ctypes.byref(b)) == gl.EINVAL
    u = ctypes.c_uint32(7)
    assert gl._lib.gravity_batch_persistent_abandoned(0, None, None, None, None) == gl.EINVAL
    assert gl._lib.gravity_batch_persistent_abandoned(1, None, None, None, ctypes.byref(u)) == gl.EINVAL
    assert gl._lib.gravity_batch_persistent_abandoned(0, None, None, None, ctypes.byref(u)) == gl.OK
    assert u.value == 0
    gl._lib.gravity_plan_destroy(None)


def test_binding_checks_sizes_before_calling_the_library():
    """The C ABI takes plain pointers, so the binding checks every array it
    hands over: dtype, device, contiguity and length (CPU tensors here are
    rejected before any device call)."""
    import torch
    import paper_2001_02765_amd as gl
    with pytest.raises(ValueError, match="CUDA"):
        gl._check_cells(torch.zeros(16), torch.float32, 16, "fx")
    with pytest.raises(ValueError, match="required"):
        gl._check_cells(None, torch.float32, 16, "fx")
    gl._check_cells(None, torch.float32, 16, "dsx", required=False)
    with pytest.raises(ValueError, match="workspace"):
        gl._check_workspace(torch.zeros(16, dtype=torch.uint8), 8)
