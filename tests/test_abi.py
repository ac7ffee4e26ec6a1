"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/smg.h declares, and sizes/validates descriptors."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "smg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(smg_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2302_13680_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2302_13680_amd import build
        build.build()
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    from paper_2302_13680_amd import binding
    assert sorted(binding.EXPORTED) == names


def test_workspace_bytes_validation(lib):
    from paper_2302_13680_amd.binding import Desc
    ok = Desc(255, 64, 7, 2, 2, 1.0, 0, 30, 0)
    nb = lib.smg_workspace_bytes(C.byref(ok))
    # at least the Krylov basis: 61 vectors of (2N+1) n^2 doubles
    assert nb >= 61 * (2 * 64 + 1) * 255 * 255 * 8
    f32 = Desc(255, 64, 7, 2, 2, 1.0, 1, 30, 0)
    assert lib.smg_workspace_bytes(C.byref(f32)) > 0
    for bad in [Desc(254, 64, 7, 2, 2, 1.0, 0, 30, 0),   # n not (nc+1)2^k - 1
                Desc(255, 0, 7, 2, 2, 1.0, 0, 30, 0),    # no samples
                Desc(255, 2049, 7, 2, 2, 1.0, 0, 30, 0),  # too many samples
                Desc(255, 64, 6, 2, 2, 1.0, 0, 30, 0),   # even coarsest grid
                Desc(255, 64, 7, 2, 2, 2.5, 0, 30, 0),   # theta out of range
                Desc(255, 64, 7, 2, 2, 1.0, 2, 30, 0),   # unknown precision
                Desc(255, 64, 7, 2, 2, 1.0, 0, 40, 0),   # restart too long
                Desc(255, 64, 7, 2, 2, 1.0, 0, 30, 64),  # unknown flags
                Desc(255, 64, 7, 2, 2, 1.0, 1, 30, 16),  # risk-averse buffers in an FP32 context
                Desc(255, 64, 7, 2, 2, 1.0, 0, 30, 0, 33),   # odd strip width
                Desc(255, 64, 7, 2, 2, 1.0, 0, 30, 0, -2),   # negative strip width
                Desc(255, 64, 7, 2, 2, 1.0, 0, 30, 0, 0, -1)]:  # negative sweep segment
        assert lib.smg_workspace_bytes(C.byref(bad)) == 0
    # every defined flag is accepted (eager, unfused, Jacobi smoother, Newton and risk-averse
    # buffers, half-sweeps only)
    assert lib.smg_workspace_bytes(C.byref(Desc(255, 64, 7, 2, 2, 0.5, 0, 30, 63))) > 0
    # the Newton buffers: two more vectors and six node arrays at least
    ssn = lib.smg_workspace_bytes(C.byref(Desc(255, 64, 7, 2, 2, 1.0, 0, 30, 8)))
    assert ssn - nb >= (2 * (2 * 64 + 1) + 4) * 255 * 255 * 8
    # defaults: coarsest_n 0 -> 7, theta 0 -> 1
    assert lib.smg_workspace_bytes(C.byref(Desc(31, 8, 0, 2, 2, 0.0, 0, 0, 0))) > 0


def test_strerror_covers_codes(lib):
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert lib.smg_strerror(code).decode() != "unknown error"


def test_setup_rejects_bad_arguments_before_any_launch(lib):
    from paper_2302_13680_amd.binding import Blocks, Desc
    out = C.c_void_p()
    d = Desc(31, 8, 7, 2, 2, 1.0, 0, 0, 0)
    assert lib.smg_setup(C.byref(d), None, None, 0, None, C.byref(out)) == -1
    c = (C.c_double * 8)(*([1.0] * 8))
    dd = (C.c_double * 8)(*([-1.0] * 8))
    b = Blocks(C.c_void_p(256), C.c_void_p(256), c, dd, dd, -1.0)   # g < 0: rejected on the host
    assert lib.smg_setup(C.byref(d), C.byref(b), C.c_void_p(256), 1 << 30, None, C.byref(out)) == -2
    b = Blocks(C.c_void_p(256), C.c_void_p(256), c, dd, dd, 1.0, None, None, -2.0)   # control growth <= 0
    assert lib.smg_setup(C.byref(d), C.byref(b), C.c_void_p(256), 1 << 30, None, C.byref(out)) == -1
    b = Blocks(C.c_void_p(256), C.c_void_p(256), c, dd, dd, 1.0)
    assert lib.smg_setup(C.byref(d), C.byref(b), None, 0, None, C.byref(out)) == -5
