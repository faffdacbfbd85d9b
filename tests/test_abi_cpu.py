"""The C ABI on the host: every declared symbol is exported, and argument
validation rejects bad input before any device call (runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2412_14775_amd import rfi

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rfi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rfi_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = rfi.load_library()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), f"{n} declared in rfi.h but not exported"
    assert sorted(rfi.EXPORTS) == names


def test_params_struct_layout_matches_header():
    # 16 4-byte fields, no padding
    assert ctypes.sizeof(rfi.rfi_params) == 64
    p = rfi.rfi_params_default()
    assert p.eps == pytest.approx(2.0 ** -23) and p.block_f == 1 and p.block_m == 64


GOOD = dict(n_stations=4, n_baselines=10, n_channels=16, n_samples=256, block_m=16)

BAD = [
    (dict(n_stations=0, n_baselines=0), "n_stations"),
    (dict(n_baselines=9), "n_baselines"),
    (dict(n_channels=0), "n_channels"),
    (dict(block_m=1), "block_m"),
    (dict(n_samples=250), "multiple of block_m"),
    (dict(n_samples=0), "multiple of block_m"),
    (dict(vis_format=7), "vis_format"),
    (dict(sk_d=0.0), "sk_d"),
    (dict(sk_d=float("nan")), "sk_d"),
    (dict(sk_low=2.0, sk_high=2.0), "sk_low < sk_high"),
    (dict(sk_low=float("nan")), "sk_low < sk_high"),
    (dict(ds_gamma=1.5), "ds_gamma"),
    (dict(ds_gamma=-0.1), "ds_gamma"),
    (dict(eps=-1.0), "eps"),
    (dict(eps=float("inf")), "eps"),
    (dict(options=64), "option"),
    (dict(options=4, kappa_sk=-1.0), "kappa"),
    (dict(options=4, n_warm=-3), "n_warm"),
    (dict(block_f=3), "block_f"),
    (dict(n_samples=1 << 26, block_m=16), "2^31"),
]


@pytest.mark.parametrize("bad,msg", BAD)
def test_plan_validation_rejects(bad, msg):
    p = rfi.rfi_params_default(**{**GOOD, **bad})
    with pytest.raises(rfi.RfiError) as ei:
        rfi.rfi_plan_create(p)
    assert ei.value.code == rfi.RFI_ERR_INVALID_ARGUMENT
    assert msg in str(ei.value)


def test_null_arguments():
    lib = rfi.load_library()
    out = ctypes.c_void_p()
    assert lib.rfi_plan_create(None, 0, ctypes.byref(out)) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert out.value is None
    p = rfi.rfi_params_default(**GOOD)
    assert lib.rfi_plan_create(ctypes.byref(p), 0, None) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert lib.rfi_plan_create(ctypes.byref(p), -1, ctypes.byref(out)) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert lib.rfi_screen(None, 16, 16, 16, None, None, None) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert "plan is NULL" in rfi.rfi_last_error()
    assert lib.rfi_destroy(None) == rfi.RFI_OK
    n = ctypes.c_size_t()
    assert lib.rfi_plan_footprint(None, ctypes.byref(n)) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert lib.rfi_state_bytes(None) == 0
    assert lib.rfi_state_get(None, None, 0) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert lib.rfi_state_set(None, None, 0) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert lib.rfi_state_reset(None, None) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert lib.rfi_probe_read(None, 16, None, None) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert lib.rfi_probe_copy(None, None, 16, None) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert lib.rfi_probe_read(32, 17, 64, None) == rfi.RFI_ERR_INVALID_ARGUMENT
    assert lib.rfi_probe_half_sums(None, None) == rfi.RFI_ERR_INVALID_ARGUMENT


def test_unsupported_block_f_reports_unsupported():
    p = rfi.rfi_params_default(**{**GOOD, "block_f": 8})
    with pytest.raises(rfi.RfiError) as ei:
        rfi.rfi_plan_create(p)
    assert ei.value.code == rfi.RFI_ERR_UNSUPPORTED


def test_missing_library_fails_loudly(tmp_path):
    saved = rfi._lib
    rfi._lib = None
    try:
        with pytest.raises(rfi.RfiError):
            rfi.load_library(str(tmp_path / "nope.so"))
    finally:
        rfi._lib = saved


def test_single_hip_runtime_in_process():
    rfi.load_library()
    assert len(rfi.hip_runtimes_loaded()) <= 1
