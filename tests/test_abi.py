"""The C-ABI library loads on the CPU and exports every declared symbol.

No compute call is made here (there is no GPU); the GPU tests call the same
entry points through the binding.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2604_12083_amd", "libmrs.so")
HEADERS = [os.path.join(ROOT, "include", h) for h in os.listdir(os.path.join(ROOT, "include")) if h.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        names |= set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(mrs_[a-z0-9_]+)\s*\(", text, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2604_12083_amd import build as b

        b.build()
    import torch  # noqa: F401  (same HIP runtime as the package uses)

    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mrs_context_create", "mrs_eval_host", "mrs_eval_device", "mrs_rod_forces_device",
                 "mrs_rotsqrt_device", "mrs_ensemble_create", "mrs_ensemble_step", "mrs_batch_step"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    import paper_2604_12083_amd as mrs

    missing = [n for n in _declared() if not callable(getattr(mrs, n, None))]
    assert not missing, missing


def test_invalid_arguments_without_device(lib):
    """Argument checks fire before any device work: a null out pointer."""
    lib.mrs_context_create.argtypes = [ctypes.c_int, ctypes.c_void_p]
    lib.mrs_context_create.restype = ctypes.c_int
    assert lib.mrs_context_create(0, None) == -1  # MRS_EINVAL
    lib.mrs_last_error.restype = ctypes.c_char_p
    lib.mrs_last_error.argtypes = [ctypes.c_void_p]
    assert lib.mrs_last_error(None) == b"null context"


def test_kernels_built_for_gfx950():
    data = open(LIB, "rb").read()
    assert b"gfx950" in data
