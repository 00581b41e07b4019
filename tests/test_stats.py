"""Host statistics of a launch (Sec. VI): P_S, its error, TTS99 and the TTS error, with the
batch semantics (one launch of R replicas is one run; it succeeds when any replica does)."""
import math

import pytest

from paper_2508_17655_amd import stats


def test_dps_definition():
    # sqrt((P - P^2) / N_rep): 0 at P = 0 and 1, largest at 1/2
    assert stats.dp_s(0.0, 100) == 0.0 and stats.dp_s(1.0, 100) == 0.0
    assert stats.dp_s(0.5, 100) == pytest.approx(0.05, rel=1e-15)
    assert stats.dp_s(0.2, 1024) == pytest.approx(math.sqrt(0.16 / 1024), rel=1e-15)


def test_dtts_paper_expression_and_edges():
    # Sec. VI: dTTS = TTS dP_S / ((1 - P_S)|ln(1 - P_S)|); at P_S = 1/2 that is TTS dP/(ln 2 / 2)
    t = stats.tts99(1.0, 0.5)
    assert stats.dtts(t, 0.5, 0.05) == pytest.approx(t * 0.05 / (0.5 * math.log(2.0)), rel=1e-15)
    assert stats.dtts(1.0, 0.995, 0.01) == 0.0  # TTS = T_com: no statistical error
    assert stats.dtts(math.inf, 0.0, 0.0) == math.inf


@pytest.mark.parametrize("p", [1e-4, 3e-3, 0.05, 0.3])
@pytest.mark.parametrize("R", [16, 128, 1024])
def test_dtts_is_the_propagated_error(p, R):
    """dTTS equals |d TTS / d p_hat| dp_hat, the derivative taken numerically on
    TTS(p) = T ln 0.01 / ln(1 - P_run(p)), wherever P_run stays below 0.99."""
    T = 2.5e-3
    pr = stats.p_run(p, R)
    if pr > 0.98:
        pytest.skip("launch succeeds almost surely: TTS = T_com")
    h = p * 1e-6
    deriv = (stats.tts99(T, stats.p_run(p + h, R)) - stats.tts99(T, stats.p_run(p - h, R))) / (2 * h)
    dp = stats.dp_s(p, R)
    got = stats.dtts(stats.tts99(T, pr), p, dp)
    assert got == pytest.approx(abs(deriv) * dp, rel=1e-6)
    # the same through the launch-level quantities: the paper's expression at P_S = P_run
    # with dP_run = R (1 - p)^(R-1) dp
    dpr = R * (1 - p) ** (R - 1) * dp
    assert stats.dtts(stats.tts99(T, pr), pr, dpr) == pytest.approx(got, rel=1e-9)


def test_batch_tts():
    # 1 hit in 1024: p = 1/1024, P_run = 1 - (1 - p)^1024 = 0.6323...
    d = stats.batch_tts(7.5e-3, 1, 1024)
    assert d["p_hat"] == 1 / 1024
    assert d["p_run"] == pytest.approx(1 - (1 - 1 / 1024) ** 1024, rel=1e-15)
    assert d["tts99_s"] == pytest.approx(7.5e-3 * math.log(0.01) / math.log(1 - d["p_run"]), rel=1e-12)
    assert d["dtts99_s"] > 0
    # no hit: the TTS is unbounded; enough hits: one launch
    assert stats.batch_tts(1.0, 0, 1024)["tts99_s"] == math.inf
    d = stats.batch_tts(1.0, 10, 1024)
    assert d["tts99_s"] == 1.0 and d["dtts99_s"] == 0.0
    with pytest.raises(ValueError):
        stats.p_hat(5, 4)
