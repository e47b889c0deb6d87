"""C ABI contract on the CPU: the library loads, exports every symbol the header
declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "rbc.h")).read()
    return sorted(set(re.findall(r"\b(rbc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1701_02059_amd import rbc
    return rbc.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n


def test_binding_names_match_header():
    from paper_1701_02059_amd import rbc
    assert sorted(rbc.FUNCTIONS) == _declared()


def test_status_strings(L):
    for s in range(9):
        assert L.rbc_status_string(s)
    assert L.rbc_status_string(0) == b"ok"
    assert L.rbc_status_string(99) == b"unknown status"


def test_null_handles_and_bad_params(L):
    from paper_1701_02059_amd import rbc
    from paper_1701_02059_amd.inputs import ModelParams
    assert L.rbc_step(None, 1, 0.01) == rbc.RBC_ERR_INVALID_ARG
    assert L.rbc_destroy(None) == rbc.RBC_ERR_INVALID_ARG
    assert L.rbc_sync(None) == rbc.RBC_ERR_INVALID_ARG
    assert L.rbc_last_error(None) == b"null handle"
    h = C.c_void_p()
    p = rbc.make_params(ModelParams(zeta=2.5))
    assert L.rbc_create(C.byref(p), None, C.byref(h)) == rbc.RBC_ERR_INVALID_ARG
    p = rbc.make_params(ModelParams(cell_target=0))
    assert L.rbc_create(C.byref(p), None, C.byref(h)) == rbc.RBC_ERR_INVALID_ARG
    assert L.rbc_create(None, None, C.byref(h)) == rbc.RBC_ERR_INVALID_ARG


def test_create_without_device_reports_hip_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_1701_02059_amd import rbc
    from paper_1701_02059_amd.inputs import ModelParams
    h = C.c_void_p()
    p = rbc.make_params(ModelParams())
    assert L.rbc_create(C.byref(p), None, C.byref(h)) == rbc.RBC_ERR_HIP
