"""The C-ABI library loads and exports every entry point its header declares
(no device calls)."""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sp_[a-z_0-9]+)\s*\(", text)))


def test_header_declarations_are_exported():
    import paper_2311_03906_amd as sp
    L = sp.lib()
    declared = _declared("symphase.h")
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(sp.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", sp._capi.LIB_PATH], capture_output=True, text=True).stdout
    syms = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert set(declared) <= syms


def test_library_has_gfx950_code_object():
    import paper_2311_03906_amd as sp
    data = open(sp._capi.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_errors_cross_the_boundary_as_codes():
    import paper_2311_03906_amd as sp
    L = sp.lib()
    import ctypes
    assert L.sp_symbolize(None, None) == sp._capi.SP_E_INVALID
    assert b"null" in L.sp_last_error()
    assert L.sp_sample(None, 0, 0, 10, None, 1, None) == sp._capi.SP_E_INVALID
    h = ctypes.c_void_p()
    assert L.sp_circuit_parse(b"FOO 1\n", 6, ctypes.byref(h)) == sp._capi.SP_E_UNSUPPORTED
    assert h.value is None
    L.sp_circuit_free(None)
    L.sp_model_free(None)
    L.sp_dmodel_free(None)


def test_sampling_requires_a_gpu_and_has_no_fallback():
    import torch
    import paper_2311_03906_amd as sp
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    m = sp.Model("X_ERROR(0.1) 0\nM 0\n")
    with pytest.raises(sp.SymphaseError):
        sp.DeviceModel(m)


def test_device_initialization_checks_arguments_before_device_work():
    """sp_symbolize_device rejects what it cannot do before it touches the
    device: the pointer below is never dereferenced."""
    import ctypes
    import paper_2311_03906_amd as sp
    L, E = sp.lib(), sp._capi
    fake = ctypes.c_void_p(1 << 20)   # 256-byte aligned, never used
    h = ctypes.c_void_p()
    c = sp.Circuit("H 0\nCX 0 1\nX_ERROR(0.1) 1\nM 0 1\n")
    need = ctypes.c_size_t()
    assert L.sp_symbolize_device_work_bytes(c.handle, ctypes.byref(need)) == 0 and need.value > 0
    assert L.sp_symbolize_device(None, 0, fake, need.value, None, ctypes.byref(h)) == E.SP_E_INVALID
    assert L.sp_symbolize_device(c.handle, 0, None, need.value, None, ctypes.byref(h)) == E.SP_E_INVALID
    assert L.sp_symbolize_device(c.handle, 7, fake, need.value, None, ctypes.byref(h)) == E.SP_E_INVALID
    assert L.sp_symbolize_device(c.handle, 0, ctypes.c_void_p((1 << 20) + 8), need.value, None,
                                 ctypes.byref(h)) == E.SP_E_INVALID
    assert b"aligned" in L.sp_last_error()
    assert L.sp_symbolize_device(c.handle, 0, fake, 256, None, ctypes.byref(h)) == E.SP_E_INVALID
    assert b"need at least" in L.sp_last_error()
    big = sp.Circuit("M 1024\n")   # 1025 qubits
    assert L.sp_symbolize_device_work_bytes(big.handle, ctypes.byref(need)) == E.SP_E_LIMIT
    assert L.sp_symbolize_device(big.handle, 0, fake, 1 << 30, None, ctypes.byref(h)) == E.SP_E_LIMIT
    assert b"1024 qubits" in L.sp_last_error()
    assert h.value is None


def test_device_initialization_modes_checked_before_device_work():
    import ctypes
    import paper_2311_03906_amd as sp
    L, E = sp.lib(), sp._capi
    fake = ctypes.c_void_p(1 << 20)
    h = ctypes.c_void_p()
    c = sp.Circuit("H 0\nCX 0 1\nX_ERROR(0.1) 1\nM 0 1\n")
    sizes = []
    for mode in (E.SP_INIT_AUTO, E.SP_INIT_ONE_PASS, E.SP_INIT_TWO_PASS):
        need = ctypes.c_size_t()
        assert L.sp_symbolize_device_work_bytes_mode(c.handle, mode, ctypes.byref(need)) == 0
        sizes.append(need.value)
    assert sizes[0] == sizes[1]   # a tiny circuit runs in one pass
    need = ctypes.c_size_t()
    assert L.sp_symbolize_device_work_bytes_mode(c.handle, 3, ctypes.byref(need)) == E.SP_E_INVALID
    got = ctypes.c_size_t(7)
    assert L.sp_symbolize_device_mode(c.handle, 0, 3, fake, 1 << 30, None, ctypes.byref(h),
                                      ctypes.byref(got)) == E.SP_E_INVALID
    assert got.value == 0   # not a size error
    assert L.sp_symbolize_device_mode(c.handle, 0, E.SP_INIT_TWO_PASS, fake, 256, None,
                                      ctypes.byref(h), ctypes.byref(got)) == E.SP_E_INVALID
    # the size that suffices comes back in the out-parameter (and the message)
    assert 256 < got.value <= sizes[2]
    assert b"need at least %d" % got.value in L.sp_last_error()
    assert L.sp_symbolize_device_mode(c.handle, 0, E.SP_INIT_TWO_PASS, fake, 256, None,
                                      ctypes.byref(h), None) == E.SP_E_INVALID
    assert h.value is None
