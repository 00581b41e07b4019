"""The operand encodings of the coupling product (eq. (3)) on the GPU against the oracle's
number formats, over EVERY binary32 value in [-1, 1] (the wall of eq. (5) keeps x there):
the hardware E4M3 conversion, the bf16 hi/lo split and the 16-bit fixed-point hi/lo split
are the encoders the step kernels' operand stores use (gsb_encode_operand shares them).
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ONE = 0x3F800000        # bit pattern of 1.0f
CHUNK = 1 << 25         # values per device round trip


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _chunks():
    """Every binary32 x with |x| <= 1, as (sign, float32 host array) chunks."""
    for sign in (0, 0x80000000):
        for lo in range(0, ONE + 1, CHUNK):
            hi = min(lo + CHUNK, ONE + 1)
            bits = np.arange(lo, hi, dtype=np.uint32) | np.uint32(sign)
            yield sign, bits.view(np.float32)


def _gsb():
    from paper_2508_17655_amd import gsb
    return gsb


def test_fp8_every_value_in_unit_interval(orc):
    import torch
    gsb = _gsb()
    say("case encode fp8 exhaustive |x| <= 1")
    total = signed_zero = 0
    for sign, xh in _chunks():
        x = torch.from_numpy(xh).cuda()
        got = gsb.encode_operand(x, gsb.GSB_PREC_FP8).cpu().numpy()
        ref = orc.e4m3_encode(xh)
        bad = got != ref
        if bad.any():
            # a zero result may carry either sign (-0 and +0 are the same operand value)
            zero = ((got & 0x7F) == 0) & ((ref & 0x7F) == 0)
            signed_zero += int(np.count_nonzero(bad & zero))
            real = np.flatnonzero(bad & ~zero)
            assert real.size == 0, (f"x = {xh[real[0]]!r} ({xh[real[0]:real[0]+1].view(np.uint32)[0]:#010x}): "
                                    f"device {got[real[0]]:#04x}, oracle {ref[real[0]]:#04x}; {real.size} in chunk")
        total += xh.size
    say(f"fp8: {total} values equal to the oracle's E4M3 codes ({signed_zero} zeros differ only in sign)")
    assert total == 2 * (ONE + 1)


def test_sign_operand_every_value_in_unit_interval(orc):
    """The sign operand of dSB/GdSB (+1 or -1 in E4M3, s(x) = +1 for x >= 0, -0.0 included,
    reading R2) for every binary32 |x| <= 1: every negative denormal must give -1 and -0.0
    must give +1, whatever the encoder computes the sign bit from."""
    import torch
    gsb = _gsb()
    say("case encode sign operand exhaustive |x| <= 1")
    total = 0
    for sign, xh in _chunks():
        x = torch.from_numpy(xh).cuda()
        got = gsb.encode_operand(x, gsb.GSB_PREC_FP8, discrete=True).cpu().numpy()
        s = orc.operand(xh, orc.FORM_EXACT, discrete=True)
        ref = np.where(s > 0, 0x38, 0xB8).astype(np.uint8)
        bad = np.flatnonzero(got != ref)
        assert bad.size == 0, (f"x = {xh[bad[0]]!r} ({xh[bad[0]:bad[0]+1].view(np.uint32)[0]:#010x}): "
                               f"device {got[bad[0]]:#04x}, oracle {ref[bad[0]]:#04x}; {bad.size} in chunk")
        total += xh.size
    say(f"sign operand: {total} values equal to the oracle's s(x)")
    assert total == 2 * (ONE + 1)


def test_fix16_every_value_in_unit_interval(orc):
    import torch
    gsb = _gsb()
    say("case encode fix16 exhaustive |x| <= 1")
    total = 0
    for sign, xh in _chunks():
        x = torch.from_numpy(xh).cuda()
        hi, lo = gsb.encode_operand(x, gsb.GSB_PREC_FIX16)
        hi = hi.cpu().numpy().astype(np.int64)
        lo = lo.cpu().numpy().astype(np.int64)
        assert hi.min() >= -64 and hi.max() <= 64
        got = (256 * hi + lo).astype(np.float64) * 2.0**-14
        ref = orc.operand(xh, orc.FORM_FIX16)
        bad = np.flatnonzero(got != ref)
        assert bad.size == 0, f"x = {xh[bad[0]]!r}: device {got[bad[0]]!r}, oracle {ref[bad[0]]!r}"
        total += xh.size
    say(f"fix16: {total} values equal to the oracle's rint(x 2^14) 2^-14")


def test_bf16x2_every_value_in_unit_interval(orc):
    import torch
    gsb = _gsb()
    say("case encode bf16x2 exhaustive |x| <= 1")
    total = 0
    for sign, xh in _chunks():
        x = torch.from_numpy(xh).cuda()
        hi, lo = gsb.encode_operand(x, gsb.GSB_PREC_BF16X2)
        got = hi.float().cpu().numpy().astype(np.float64) + lo.float().cpu().numpy().astype(np.float64)
        ref = orc.operand(xh, orc.FORM_BF16X2)
        bad = np.flatnonzero(got != ref)
        assert bad.size == 0, f"x = {xh[bad[0]]!r}: device {got[bad[0]]!r}, oracle {ref[bad[0]]!r}"
        total += xh.size
    say(f"bf16x2: {total} values equal to the oracle's bf16(x) + bf16(x - bf16(x))")


def test_sign_and_fp32_forms(orc):
    import torch
    gsb = _gsb()
    say("case encode sign forms and fp32")
    rng = np.random.default_rng(5)
    xh = np.concatenate([rng.uniform(-1, 1, 100003), [0.0, -0.0, 1.0, -1.0, 1e-30, -1e-30, 2.0**-149, -2.0**-149]])
    xh = xh.astype(np.float32)
    x = torch.from_numpy(xh).cuda()
    s = orc.operand(xh, orc.FORM_EXACT, discrete=True)
    np.testing.assert_array_equal(np.where(s > 0, 0x38, 0xB8).astype(np.uint8),
                                  gsb.encode_operand(x, gsb.GSB_PREC_FP8, discrete=True).cpu().numpy())
    hi, lo = gsb.encode_operand(x, gsb.GSB_PREC_BF16X2, discrete=True)
    np.testing.assert_array_equal(hi.float().cpu().numpy(), s)
    assert not lo.float().cpu().numpy().any()
    hi, lo = gsb.encode_operand(x, gsb.GSB_PREC_FIX16, discrete=True)
    np.testing.assert_array_equal((256 * hi.cpu().numpy().astype(np.int64) + lo.cpu().numpy()) * 2.0**-14, s)
    np.testing.assert_array_equal(gsb.encode_operand(x, gsb.GSB_PREC_FP32, discrete=True).cpu().numpy(), s)
    out = gsb.encode_operand(x, gsb.GSB_PREC_FP32).cpu().numpy()
    np.testing.assert_array_equal(out.view(np.uint32), xh.view(np.uint32))  # bit for bit, -0.0 included


@pytest.mark.parametrize("count", [1, 2, 3, 5, 4097])
def test_ragged_counts_write_only_their_values(orc, count):
    import torch
    gsb = _gsb()
    say(f"case encode ragged count={count}")
    xh = np.random.default_rng(count).uniform(-1, 1, count).astype(np.float32)
    x = torch.from_numpy(xh).cuda()
    for prec, width in ((gsb.GSB_PREC_FP8, 1), (gsb.GSB_PREC_FIX16, 2), (gsb.GSB_PREC_BF16X2, 4),
                        (gsb.GSB_PREC_FP32, 4)):
        buf = torch.full((width * count + 64,), 0xAB, dtype=torch.uint8, device="cuda")
        gsb.gsb_encode_operand(prec, 0, x.data_ptr(), count, buf.data_ptr(), torch.cuda.current_stream().cuda_stream)
        b = buf.cpu().numpy()
        assert np.all(b[width * count:] == 0xAB), f"precision {prec} wrote past its output"
        if prec == gsb.GSB_PREC_FP8:
            np.testing.assert_array_equal(b[:count], orc.e4m3_encode(xh))
        elif prec == gsb.GSB_PREC_FIX16:
            hi = b[:count].view(np.int8).astype(np.int64)
            lo = b[count:2 * count].view(np.int8).astype(np.int64)
            np.testing.assert_array_equal((256 * hi + lo) * 2.0**-14, orc.operand(xh, orc.FORM_FIX16))
        elif prec == gsb.GSB_PREC_BF16X2:
            u = b[:4 * count].view(np.uint16).astype(np.uint32) << 16
            v = u.view(np.float32).astype(np.float64)
            np.testing.assert_array_equal(v[:count] + v[count:], orc.operand(xh, orc.FORM_BF16X2))
        else:
            np.testing.assert_array_equal(b[:4 * count].view(np.float32), xh)
