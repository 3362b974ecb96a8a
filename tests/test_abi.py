"""The C-ABI library loads and exports every entry point that include/shot.h declares (CPU only)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shot.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(shot_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2605_18389_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2605_18389_amd.build import build
        build()
    return binding.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("shot_sht_plan", "shot_heat_apply", "shot_sinkhorn_solve",
                     "shot_sinkhorn_divergence", "shot_sinkhorn_divergence_grad"):
        assert required in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2605_18389_amd import binding
    assert sorted(binding.EXPORTS) == _declared()


def test_status_strings(lib_path):
    from paper_2605_18389_amd import binding
    lib = binding.load_library(lib_path)
    assert lib.shot_status_string(0) == b"ok"
    assert b"breakdown" in lib.shot_status_string(17)


def test_argument_errors_need_no_gpu(lib_path):
    # invalid plans are rejected before any HIP call
    from paper_2605_18389_amd import binding
    lib = binding.load_library(lib_path)
    h = ctypes.c_void_p()
    bad = (binding.GridDesc * 1)(binding.GridDesc(0, 32, 40, 32))  # nlon < 2L-1
    assert lib.shot_sht_plan(ctypes.byref(h), bad, 1, 1, 0, None) == binding.E_INVALID
    bad = (binding.GridDesc * 1)(binding.GridDesc(0, 32, 4096, 32))  # nlon > 2048
    assert lib.shot_sht_plan(ctypes.byref(h), bad, 1, 1, 0, None) == binding.E_UNSUPPORTED
    assert lib.shot_sht_plan(ctypes.byref(h), bad, 0, 1, 0, None) == binding.E_INVALID
    # degenerate grids: one row, one column
    for desc in ((0, 1, 4, 1), (0, 2, 1, 1), (1, 1, 4, 1)):
        bad = (binding.GridDesc * 1)(binding.GridDesc(*desc))
        assert lib.shot_sht_plan(ctypes.byref(h), bad, 1, 1, 0, None) == binding.E_INVALID
    assert lib.shot_plan_destroy(None) == 0


def test_library_was_built_from_these_sources(lib_path):
    """The build id stored in libshot.so is the hash of the sources next to it
    (the loader refuses a library whose id differs)."""
    from paper_2605_18389_amd.build import source_hash
    lib = ctypes.CDLL(lib_path)
    lib.shot_build_id.restype = ctypes.c_char_p
    assert lib.shot_build_id().decode() == source_hash()
