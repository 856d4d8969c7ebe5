"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and its host-only entry points behave (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pd.h")


@pytest.fixture(scope="module")
def pd():
    from paper_1806_06917_amd import pd as mod
    return mod


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    syms = declared_symbols()
    for name in ("pd_build_neighbors", "pd_internal_force", "pd_verlet_step",
                 "pd_apply_tangent", "pd_solve_implicit"):
        assert name in syms


def test_library_exports_every_declared_symbol(pd):
    missing = [s for s in declared_symbols() if not hasattr(pd.lib, s)]
    assert not missing, missing


def test_status_strings_and_version(pd):
    assert pd.lib.pd_version() >= 10000
    for st in range(0, -7, -1):
        assert pd.lib.pd_status_string(st)
    assert pd.lib.pd_status_string(-99) == b"unknown status"


def test_micromodulus_matches_oracle(pd, orc):
    for dim in (2, 3):
        for d in (0.03, 3 / 32, 0.1, 0.05):
            for E in (1.0, 4000.0):
                assert pd.micromodulus(dim, E, d) == orc.micromodulus(dim, E, d)
    assert pd.micromodulus(4, 1.0, 0.1) != pd.micromodulus(4, 1.0, 0.1)   # NaN


def test_null_handles_rejected_without_gpu(pd):
    L = pd.lib
    assert L.pd_ctx_destroy(None) == pd.PD_EINVAL
    assert L.pd_nbr_destroy(None) == pd.PD_EINVAL
    assert L.pd_sim_destroy(None) == pd.PD_EINVAL
    assert L.pd_verlet_step(None, 1, 0.1) == pd.PD_EINVAL
    assert L.pd_nbr_info(None, None, None) == pd.PD_EINVAL
    assert L.pd_build_neighbors(None, 2, 4, None, 0.1, None) == pd.PD_EINVAL
    assert L.pd_last_error(None) == b"null context"


def test_context_without_gpu_reports_device_error(pd):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert pd.lib.pd_ctx_create(0, None, C.byref(h)) == pd.PD_EDEVICE
    assert not h.value
