"""The C ABI (include/gsb.h) on the host: the library loads, exports every declared entry
point, and its host-side checks reject what eq. (1) excludes.  No device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2508_17655_amd import gsb, instances

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header="gsb.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsb_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(gsb.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(gsb.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert gsb.gsb_version().startswith("gsb-mi355x")


def test_probe_library_is_separate_and_exports_its_header():
    from paper_2508_17655_amd import probe

    assert declared_symbols("gsb_probe.h") == sorted(probe.SYMBOLS)
    plib = ctypes.CDLL(probe.LIB_PATH)
    for name in probe.SYMBOLS:
        assert hasattr(plib, name), name
    # the product library carries no measurement code
    assert not hasattr(ctypes.CDLL(gsb.LIB_PATH), "gsb_probe_ceilings")


def _status(fn, *args):
    try:
        fn(*args)
    except gsb.GsbError as e:
        return e.status
    return gsb.GSB_OK


def test_create_rejects_invalid_instances():
    J = instances.dense_pm1(6, 1)
    bad = J.copy(); bad[0, 1] = 5.0
    assert _status(gsb.gsb_create, bad) == gsb.GSB_ENOTSYM
    bad = J.copy(); bad[2, 2] = 1.0
    assert _status(gsb.gsb_create, bad) == gsb.GSB_EDIAG
    bad = J.copy(); bad[0, 1] = bad[1, 0] = np.nan
    assert _status(gsb.gsb_create, bad) == gsb.GSB_ENONFINITE
    assert _status(gsb.gsb_create, J, np.array([0, 0, np.inf, 0, 0, 0], np.float32)) == gsb.GSB_ENONFINITE
    assert _status(gsb.gsb_create, np.zeros((0, 0), np.float32)) == gsb.GSB_EINVAL
    assert "J_ij != J_ji" in (gsb.gsb_create.__doc__ or "J_ij != J_ji")


def test_options_and_errors_without_device():
    ctx = gsb.gsb_create(instances.dense_pm1(10, 2))
    try:
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_PRECISION) == gsb.GSB_PREC_FP8  # J in {0, +-1}
        assert _status(gsb.gsb_set, ctx, gsb.GSB_OPT_C, -1.0) == gsb.GSB_EINVAL
        assert _status(gsb.gsb_set, ctx, gsb.GSB_OPT_PRECISION, 7) == gsb.GSB_EINVAL
        assert _status(gsb.gsb_set, ctx, gsb.GSB_OPT_LAMBDA_MAX, 1.0) == gsb.GSB_EINVAL
        assert _status(gsb.gsb_step, ctx, 1) == gsb.GSB_ESTATE
        assert _status(gsb.gsb_energy, ctx) in (gsb.GSB_ESTATE, gsb.GSB_EINVAL)
        assert _status(gsb.gsb_init, ctx, 9, 0, 0.0, 1.0, 4, 10, 1) == gsb.GSB_EINVAL
        assert _status(gsb.gsb_init, ctx, 0, 0, -1.0, 1.0, 4, 10, 1) == gsb.GSB_EINVAL
        assert _status(gsb.gsb_init, ctx, 0, 0, 0.0, 0.0, 4, 10, 1) == gsb.GSB_EINVAL
        assert _status(gsb.gsb_init, ctx, 0, 0, 0.0, 1.0, 0, 10, 1) == gsb.GSB_EINVAL
        assert _status(gsb.gsb_init, ctx, 0, 0, 0.0, 1.0, 4, 0, 1) == gsb.GSB_EINVAL
        gsb.gsb_set(ctx, gsb.GSB_OPT_C, 0.25)
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_C) == 0.25
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_STEP_KERNEL) == 0
        for bad in (-1, 3, 1.5, float("nan"), float("inf"), 1e300):
            assert _status(gsb.gsb_set, ctx, gsb.GSB_OPT_STEP_KERNEL, bad) == gsb.GSB_EINVAL
            assert _status(gsb.gsb_set, ctx, gsb.GSB_OPT_PRECISION, bad if bad != 3 else 9) == gsb.GSB_EINVAL
            assert _status(gsb.gsb_set, ctx, gsb.GSB_OPT_INIT_MODE, bad if bad != 3 else 9) == gsb.GSB_EINVAL
        gsb.gsb_set(ctx, gsb.GSB_OPT_STEP_KERNEL, 2)
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_STEP_KERNEL) == 2
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_GRID_PAD) == 1
        for bad in (-1, 2, 0.5, float("nan"), float("inf")):
            assert _status(gsb.gsb_set, ctx, gsb.GSB_OPT_GRID_PAD, bad) == gsb.GSB_EINVAL
        gsb.gsb_set(ctx, gsb.GSB_OPT_GRID_PAD, 0)
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_GRID_PAD) == 0
        # the LLE window start: an integer step >= 0 (gsb_lle checks it against its steps)
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_LLE_FROM) == 0
        for bad in (-1, 0.5, float("nan"), float("inf"), 2.0**25):
            assert _status(gsb.gsb_set, ctx, gsb.GSB_OPT_LLE_FROM, bad) == gsb.GSB_EINVAL
        gsb.gsb_set(ctx, gsb.GSB_OPT_LLE_FROM, 400)
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_LLE_FROM) == 400
        # the device-memory state and reverse-pass calls need a run first (no device work)
        lib = gsb.load_library()
        m = ctypes.c_int32()
        assert lib.gsb_state_device(ctx, None, None, None, ctypes.byref(m)) == gsb.GSB_ESTATE
        assert lib.gsb_set_state_device(ctx, None, None, None, 0) == gsb.GSB_ESTATE
        assert lib.gsb_vjp_device(ctx, 1, None, None, None) == gsb.GSB_EINVAL  # NULL cotangents
    finally:
        gsb.gsb_destroy(ctx)
    ctx = gsb.gsb_create(instances.dense_gaussian(10, 2))
    try:
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_PRECISION) == gsb.GSB_PREC_BF16X2
        assert _status(gsb.gsb_set, ctx, gsb.GSB_OPT_PRECISION, gsb.GSB_PREC_FP8) == gsb.GSB_EUNSUPPORTED
    finally:
        gsb.gsb_destroy(ctx)


def test_encode_operand_arguments_are_checked_before_any_device_work():
    enc = gsb.gsb_encode_operand
    assert _status(enc, 7, 0, 0x1000, 4, 0x2000, None) == gsb.GSB_EINVAL      # precision
    assert _status(enc, gsb.GSB_PREC_FP8, 0, 0x1000, -1, 0x2000, None) == gsb.GSB_EINVAL
    assert _status(enc, gsb.GSB_PREC_FP8, 0, None, 4, 0x2000, None) == gsb.GSB_EINVAL
    assert _status(enc, gsb.GSB_PREC_FP8, 0, 0x1000, 4, None, None) == gsb.GSB_EINVAL
    assert _status(enc, gsb.GSB_PREC_FP8, 0, 0x1002, 4, 0x2000, None) == gsb.GSB_EINVAL  # misaligned
    assert _status(enc, gsb.GSB_PREC_FP8, 0, 0x1000, 4, 0x2001, None) == gsb.GSB_EINVAL
    # out overlapping x: FP8 needs count bytes, FP32 4 count bytes
    assert _status(enc, gsb.GSB_PREC_FP32, 0, 0x1000, 16, 0x1020, None) == gsb.GSB_EINVAL
    assert _status(enc, gsb.GSB_PREC_FP8, 0, 0x1000, 16, 0x0ff4, None) == gsb.GSB_EINVAL
    # count 0 is a no-op that never touches the device
    enc(gsb.GSB_PREC_FIX16, 0, None, 0, None, None)


@pytest.mark.parametrize("n", [2, 9, 64])
def test_eigenvalues_and_default_c(n):
    # App. A: c = 1/lambda_max; eq. (13) dt = 1.25 sqrt(2/(1 - lambda_min/lambda_max)).
    # Ferromagnet J = 1 - I has lambda_max = n - 1 and lambda_min = -1.
    ctx = gsb.gsb_create((np.ones((n, n)) - np.eye(n)).astype(np.float32))
    try:
        lmax = gsb.gsb_get(ctx, gsb.GSB_OPT_LAMBDA_MAX)
        lmin = gsb.gsb_get(ctx, gsb.GSB_OPT_LAMBDA_MIN)
        assert abs(lmax - (n - 1)) < 1e-9 and abs(lmin + 1) < 1e-9
        assert abs(gsb.gsb_get(ctx, gsb.GSB_OPT_C) - 1 / (n - 1)) < 1e-12
        dt = gsb.gsb_get(ctx, gsb.GSB_OPT_DT_STABLE)
        assert abs(dt - 1.25 * math.sqrt(2 / (1 + 1 / (n - 1)))) < 1e-9
    finally:
        gsb.gsb_destroy(ctx)


def test_eigenvalues_random_matrix():
    J = instances.dense_gaussian(300, 4)
    lam = np.linalg.eigvalsh(J.astype(np.float64))
    ctx = gsb.gsb_create(J)
    try:
        assert abs(gsb.gsb_get(ctx, gsb.GSB_OPT_LAMBDA_MAX) - lam[-1]) < 1e-8
        assert abs(gsb.gsb_get(ctx, gsb.GSB_OPT_LAMBDA_MIN) - lam[0]) < 1e-8
    finally:
        gsb.gsb_destroy(ctx)


def test_field_becomes_ancilla():
    n = 7
    ctx = gsb.gsb_create(instances.dense_pm1(n, 3), np.linspace(-1, 1, n).astype(np.float32))
    try:
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_N) == n
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_N_DYN) == n + 1
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_PRECISION) == gsb.GSB_PREC_BF16X2  # h not in {0, +-1}
    finally:
        gsb.gsb_destroy(ctx)
    ctx = gsb.gsb_create(instances.dense_pm1(n, 3), np.zeros(n, np.float32))
    try:
        assert gsb.gsb_get(ctx, gsb.GSB_OPT_N_DYN) == n  # zero field: no ancilla
    finally:
        gsb.gsb_destroy(ctx)
