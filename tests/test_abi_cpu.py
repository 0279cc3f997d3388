"""The C-ABI library loads, exports every symbol include/ns.h declares, and
rejects bad arguments before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ns.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ns_status|const char\*)\s+(ns_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def capi():
    from paper_2509_13307_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        from paper_2509_13307_amd.build import build
        build()
    return _capi


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("ns_loglike_batch", "ns_loglike_grad_batch", "ns_theory_batch", "ns_slice_step", "ns_run", "ns_hmc",
                 "ns_model_create", "ns_model_free", "ns_last_error", "ns_prior_transform"):
        assert name in fns


def test_every_declared_symbol_is_exported(capi):
    lib = capi.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert {n for n, _, _ in capi.SIGNATURES} == set(declared_functions())


def test_argument_validation_without_device(capi):
    lib = capi.lib()
    out = ctypes.c_void_p()
    assert lib.ns_model_create(None, 0, ctypes.byref(out)) == capi.NS_E_INVALID
    assert b"desc" in lib.ns_last_error()
    assert lib.ns_loglike_batch(None, None, 6, 10, None, 0, None) == capi.NS_E_INVALID
    assert lib.ns_theory_batch(None, None, 6, 10, None, 100, 0, None) == capi.NS_E_INVALID
    assert lib.ns_loglike_batch_noalloc(None, None, 6, 10, None, 3, None) == capi.NS_E_INVALID
    assert lib.ns_model_free(None) == capi.NS_OK
    assert lib.ns_last_error() == b""
    assert lib.ns_run(None, None, None, None, None, None, 0, None) == capi.NS_E_INVALID
    assert lib.ns_slice_step(None, None, None, None, None, 4, 0.0, None, 1, 0, 0, 0, None) == capi.NS_E_INVALID
    res = capi.HmcResult()
    opts = capi.HmcOpts(4, 10, 5, 0, 0.1, 1)
    assert lib.ns_hmc(None, ctypes.byref(opts), None, None, None, None, ctypes.byref(res), None) == capi.NS_E_INVALID
    assert b"model" in lib.ns_last_error()


def test_module_refuses_to_run_without_library(tmp_path, monkeypatch):
    from paper_2509_13307_amd import _capi
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_capi, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _capi.lib()


def test_binding_rejects_bad_tensors():
    """The binding refuses host, wrong-dtype, mis-shaped and strided tensors
    before any pointer reaches the library (no device needed: every tensor
    here is a host tensor or fails a shape check first)."""
    import torch
    from paper_2509_13307_amd.model import check_rows, check_vector
    with pytest.raises(TypeError, match="float64"):
        check_rows(torch.zeros(4, 6, dtype=torch.float32), 6, 0, "u")
    with pytest.raises(TypeError, match="device"):
        check_rows(torch.zeros(4, 6, dtype=torch.float64), 6, 0, "u")
    with pytest.raises(TypeError, match="float64"):
        check_rows([[0.0] * 6], 6, 0, "u")
    with pytest.raises(TypeError, match="float64"):
        check_vector(torch.zeros(4, dtype=torch.float32), 4, torch.float64, torch.device("cpu"), "logl")
    with pytest.raises(TypeError, match="live on"):
        check_vector(torch.zeros(4, dtype=torch.float64), 4, torch.float64, torch.device("cuda", 0), "logl")
    with pytest.raises(ValueError, match="length 5"):
        check_vector(torch.zeros(4, dtype=torch.float64), 5, torch.float64, torch.device("cpu"), "logl")
    with pytest.raises(ValueError, match="contiguous"):
        check_vector(torch.zeros(8, dtype=torch.float64)[::2], 4, torch.float64, torch.device("cpu"), "logl")
