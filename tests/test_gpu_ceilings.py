"""The device-ceiling probes (libgsb_probe.so, gsb_probe_ceilings) return rates in the range
an MI355X can reach: at most the published dense peaks plus a clock margin, and well above
zero; and the MFMA/VALU sharing probe's times are consistent."""
import pytest

pytestmark = pytest.mark.gpu


def test_ceilings_are_plausible():
    from paper_2508_17655_amd import probe

    c = probe.device_ceilings()
    print(c, flush=True)
    # published dense peaks at 2.4 GHz: FP8 5.0 PFLOP/s, int8 5.0 POP/s, BF16 2.5, FP32 MFMA 0.157
    assert 1.0e15 < c["mfma_fp8_flops"] <= 5.5e15
    assert 1.0e15 < c["mfma_fp4xfp8_flops"] <= 11.0e15
    assert 1.0e15 < c["mfma_int8_ops"] <= 5.5e15
    assert 0.5e15 < c["mfma_bf16_flops"] <= 2.8e15
    assert 3.0e13 < c["mfma_fp32_flops"] <= 1.8e14
    # HBM3E 8 TB/s; caches faster than HBM
    assert 1.0e12 < c["read_hbm_2GiB_Bps"] <= 8.5e12
    assert 1.0e12 < c["write_hbm_2GiB_Bps"] <= 8.5e12
    assert c["read_l2_2MiB_Bps"] > c["read_hbm_2GiB_Bps"]
    assert 1.0e9 < c["shader_clock_hz"] < 3.0e9
    # both kinds of waves together take at least as long as either alone and at most the sum
    # (with a margin for the clock)
    m, v, b = c["coissue_mfma_only_ms"], c["coissue_valu_only_ms"], c["coissue_both_ms"]
    assert 0.0 < m and 0.0 < v
    assert 0.95 * max(m, v) <= b <= 1.1 * (m + v)
