"""C-ABI checks that need no GPU: the library loads, exports every function
include/sfo.h declares, and rejects invalid descriptors before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sfo.h")).read()
    return sorted(set(re.findall(r"^\s*(?:sfo_status|const char \*)\s*(sfo_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1012_3911_amd import sfo

    if not os.path.exists(sfo.LIB_PATH):
        pytest.skip("libsfo.so not built")
    return sfo.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header(lib):
    from paper_1012_3911_amd import sfo

    assert set(declared_functions()) == set(sfo.EXPORTS)


def _desc(**kw):
    from paper_1012_3911_amd import sfo

    d = sfo.GridDesc()
    d.ndim = kw.get("ndim", 2)
    n = kw.get("n", (64, 64, 1))
    for a in range(3):
        d.n[a] = n[a]
        d.xmin[a] = -1.0
        d.xmax[a] = kw.get("xmax", 1.0)
    d.equation = kw.get("equation", 0)
    d.dtype = kw.get("dtype", 1)
    d.dt = kw.get("dt", 0.01)
    d.mass = 1.0
    d.charge = -1.0
    d.c = 137.036
    d.hbar = 1.0
    d.flags = 0
    return d


@pytest.mark.parametrize("kw,status", [
    (dict(ndim=0), -1), (dict(ndim=4), -1), (dict(n=(96, 64, 1)), -1), (dict(n=(64, 0, 1)), -1),
    (dict(xmax=-2.0), -1), (dict(dt=0.0), -1), (dict(dt=float("nan")), -1), (dict(dtype=7), -1),
    (dict(equation=3), -1), (dict(equation=1, ndim=3, n=(64, 64, 64)), -1),
    (dict(n=(32, 64, 1)), -2), (dict(n=(8192, 64, 1)), -2), (dict(ndim=1, n=(16384, 1, 1)), -2),
    # beyond the 32-bit offsets of the passes: 2^36 bytes of complex64, 2^36 of complex128
    (dict(ndim=3, n=(4096, 4096, 512), dtype=0), -2), (dict(ndim=3, n=(4096, 4096, 256), dtype=1), -2),
])
def test_invalid_descriptors(lib, kw, status):
    d = _desc(**kw)
    h = ctypes.c_void_p()
    rc = lib.sfo_create_grid(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == status
    assert h.value is None
    assert lib.sfo_last_error().decode()


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.sfo_create_grid(None, None, ctypes.byref(h)) == -1
    assert lib.sfo_destroy_grid(None) == -1
    assert lib.sfo_propagate(None, None, 0, 1) == -1
    assert lib.sfo_norm(None, None, None) == -1
    assert lib.sfo_create_batch(None, 0, None, ctypes.byref(h)) == -1
    assert lib.sfo_destroy_batch(None) == -1
    assert lib.sfo_propagate_batch(None, None, 0, 1) == -1
    assert lib.sfo_adjoint_batch(None, None, None, 0, 1, None, None) == -1
    assert lib.sfo_batch_set_graph(None, 1) == -1
    assert lib.sfo_batch_check(None) == -1
    assert lib.sfo_time_pass(None, 0, 10, None) == -1
    assert lib.sfo_autocorrelation(None, None, 4, None) == -1
    assert lib.sfo_spectrum(None, None, 4, None, 1, None) == -1
    assert lib.sfo_eigenfunction(None, None, 4, ctypes.c_double(0.0), None) == -1
    assert lib.sfo_set_vector_field(None, None, None, 4) == -1
    assert lib.sfo_adjoint_noalloc(None, None, None, 0, 1, None, None) == -1
    assert lib.sfo_set_norm_watch(None, 1.0, 1e-6) == -1
    assert lib.sfo_adjoint_velocity(None, None, None, 0, 1, None, None, None) == -1
    assert lib.sfo_version().decode().startswith("sfo")
