"""The C-ABI library loads, exports every symbol that include/cyclo.h declares,
and rejects bad arguments before touching the device (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2405_16911_amd import cyclo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            src = open(os.path.join(inc, fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(cyc_\w+)\s*\(", src, flags=re.M))
    return names


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(cyclo.LIB_PATH):
        from paper_2405_16911_amd.build import build_library
        build_library()
    return cyclo.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert {"cyc_create", "cyc_push", "cyc_read", "cyc_reset", "cyc_destroy", "cyc_status_str",
            "cyc_query"} <= names
    out = subprocess.run(["nm", "-D", "--defined-only", cyclo.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (cyc_\w+)", out))
    assert names <= exported, names - exported
    assert set(cyclo.SIGNATURES) == names
    for n in names:
        getattr(L, n)


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5):
        assert cyclo.status_str(code)
    assert "unknown" in cyclo.status_str(42)


def test_invalid_arguments_rejected_on_host(L):
    out = ctypes.c_void_p()
    a = (ctypes.c_double * 3)(0.0, 0.1, 0.2)
    assert L.cyc_create(None, a, 3, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create(ctypes.byref(out), None, 3, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create(ctypes.byref(out), a, 0, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create(ctypes.byref(out), a, 3, 0, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create(ctypes.byref(out), a, 3, 5000, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create(ctypes.byref(out), a, 3, 4097, 0, None) == cyclo.CYC_EINVAL  # T <= 4096
    assert L.cyc_create(ctypes.byref(out), a, 3, 4, 0x100, None) == cyclo.CYC_EINVAL
    assert L.cyc_create(ctypes.byref(out), a, 3, 4, 0x3, None) == cyclo.CYC_EINVAL
    assert L.cyc_create(ctypes.byref(out), a, 3, 4, cyclo.CYC_TW_SPLIT, None) == cyclo.CYC_EUNSUPPORTED
    bad = (ctypes.c_double * 2)(0.0, float("nan"))
    assert L.cyc_create(ctypes.byref(out), bad, 2, 4, 0, None) == cyclo.CYC_EINVAL
    inf = (ctypes.c_double * 1)(float("inf"))
    assert L.cyc_create(ctypes.byref(out), inf, 1, 4, 0, None) == cyclo.CYC_EINVAL
    assert out.value is None
    assert L.cyc_push(None, None, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_read(None, None, None, None, None) == cyclo.CYC_EINVAL
    assert L.cyc_reset(None) == cyclo.CYC_EINVAL
    assert L.cyc_query(None, None, None, None, None) == cyclo.CYC_EINVAL
    assert L.cyc_profile(None, 1) == cyclo.CYC_EINVAL
    assert L.cyc_profile_read(None, None, None, None) == cyclo.CYC_EINVAL
    L.cyc_destroy(None)


def test_kernel_configurations_enumerate(L):
    n = cyclo.cyc_kernel_cfg_count()
    assert n > 0
    infos = [cyclo.cyc_kernel_cfg_info(i) for i in range(n)]
    names = [i["name"] for i in infos]
    assert len(set(names)) == n
    modes = {(i["flags"]) for i in infos}
    # every precision / split mode the ABI accepts has at least one configuration
    assert {0x0, 0x1, 0x2, 0x1 | 0x4, 0x2 | 0x4} <= modes
    for i in infos:
        assert i["lag_tile"] % 16 == 0 and i["alpha_tile"] > 0 and i["threads"] % 64 == 0
    with pytest.raises(cyclo.CycloError):
        cyclo.cyc_kernel_cfg_info(n)
    assert L.cyc_kernel_cfg_info(-1, None, None, None, None, None) == cyclo.CYC_EINVAL
    assert L.cyc_set_kernel_cfg(None, 0) == cyclo.CYC_EINVAL
    assert L.cyc_autotune(0, 4, 0, None, None, None) == cyclo.CYC_EINVAL


def test_batch_invalid_arguments(L):
    out = ctypes.c_void_p()
    a = (ctypes.c_double * 3)(0.0, 0.1, 0.2)
    offs = (ctypes.c_int64 * 3)(0, 2, 3)
    bad_offs = (ctypes.c_int64 * 3)(0, 0, 3)
    assert L.cyc_batch_create(None, 2, offs, a, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_batch_create(ctypes.byref(out), 0, offs, a, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_batch_create(ctypes.byref(out), 2, bad_offs, a, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_batch_create(ctypes.byref(out), 2, offs, a, 0, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_batch_create(ctypes.byref(out), 2, offs, a, 4, cyclo.CYC_TW_SPLIT, None) == cyclo.CYC_EUNSUPPORTED
    nan = (ctypes.c_double * 3)(0.0, float("nan"), 0.2)
    assert L.cyc_batch_create(ctypes.byref(out), 2, offs, nan, 4, 0, None) == cyclo.CYC_EINVAL
    assert out.value is None
    assert L.cyc_batch_push(None, None, None, None) == cyclo.CYC_EINVAL
    assert L.cyc_batch_read(None, None, None, None, None) == cyclo.CYC_EINVAL
    assert L.cyc_batch_reset(None) == cyclo.CYC_EINVAL
    assert L.cyc_batch_query(None, None, None, None) == cyclo.CYC_EINVAL
    L.cyc_batch_destroy(None)


def test_proposal_invalid_arguments(L):
    out = ctypes.c_void_p()
    assert L.cyc_model_create(None, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_model_create(ctypes.byref(out), 0, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_model_create(ctypes.byref(out), 4, 0x2, None) == cyclo.CYC_EUNSUPPORTED
    assert out.value is None
    assert L.cyc_model_num_params() == 67197568
    assert L.cyc_propose(None, None, 1, 16, 2, 512, 0.0, None, None, None, None, None) == cyclo.CYC_EINVAL
    assert L.cyc_select(None, 1, 16, 2, 512, None, None, None) == cyclo.CYC_EINVAL
    assert L.cyc_peak_labels(None, None, 1, 64, 8, 0, 7.0, None, None) == cyclo.CYC_EINVAL
    L.cyc_model_destroy(None)


def test_parameter_file_round_trip(tmp_path):
    v = np.arange(cyclo.ProposalModel.num_params(), dtype=np.float32) * np.float32(1e-3)
    cyclo.ProposalModel.save(str(tmp_path / "p.npy"), v)
    assert np.array_equal(cyclo.ProposalModel.load(str(tmp_path / "p.npy")), v)
    np.save(tmp_path / "bad.npy", v[:10])
    with pytest.raises(ValueError):
        cyclo.ProposalModel.load(str(tmp_path / "bad.npy"))


def test_grid_invalid_arguments(L):
    out = ctypes.c_void_p()
    assert L.cyc_grid_create(None, 0.0, 64, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_grid_create(ctypes.byref(out), float("nan"), 64, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_grid_create(ctypes.byref(out), 0.0, 64, 0, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_grid_create(ctypes.byref(out), 0.0, 64, 4, cyclo.CYC_OP_BF16, None) == cyclo.CYC_EINVAL
    assert L.cyc_grid_create(ctypes.byref(out), 0.0, 100, 4, 0, None) == cyclo.CYC_EUNSUPPORTED
    assert L.cyc_grid_create(ctypes.byref(out), 0.0, 1 << 17, 4, 0, None) == cyclo.CYC_EUNSUPPORTED
    assert L.cyc_grid_create(ctypes.byref(out), 0.0, 1, 4, 0, None) == cyclo.CYC_EUNSUPPORTED
    assert out.value is None
    assert L.cyc_grid_push(None, None, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_grid_read(None, None, None, None, None) == cyclo.CYC_EINVAL
    assert L.cyc_grid_reset(None) == cyclo.CYC_EINVAL
    L.cyc_grid_destroy(None)


def test_two_input_invalid_arguments(L):
    out = ctypes.c_void_p()
    a = (ctypes.c_double * 3)(0.0, 0.1, 0.2)
    assert L.cyc_create2(None, a, 3, -5, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create2(ctypes.byref(out), a, 3, -(1 << 21), 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create2(ctypes.byref(out), a, 3, 1 << 21, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create2(ctypes.byref(out), a, 3, -5, 0, 0, None) == cyclo.CYC_EINVAL
    assert out.value is None
    assert L.cyc_push2(None, None, None, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_grid_create2(None, 0.0, 64, -3, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_grid_create2(ctypes.byref(out), 0.0, 64, 1 << 21, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_grid_create2(ctypes.byref(out), 0.0, 100, -3, 4, 0, None) == cyclo.CYC_EUNSUPPORTED
    assert L.cyc_grid_push2(None, None, None, 0, None) == cyclo.CYC_EINVAL


def test_scf_invalid_arguments(L):
    assert L.cyc_scf(None, None, 4, 0, 4, 16, 0, None, None) == cyclo.CYC_EINVAL


def test_window_invalid_arguments(L):
    out = ctypes.c_void_p()
    a = (ctypes.c_double * 3)(0.0, 0.1, 0.2)
    assert L.cyc_create_window(ctypes.byref(out), a, 3, 4, 64, 0, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create_window(ctypes.byref(out), a, 3, 4, 48, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create_window(ctypes.byref(out), a, 3, 4, 0, 4, 0, None) == cyclo.CYC_EINVAL
    assert L.cyc_create_window(ctypes.byref(out), a, 3, 4, 64, 5000, 0, None) == cyclo.CYC_EINVAL
    assert out.value is None
