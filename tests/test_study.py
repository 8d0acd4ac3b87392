"""The study logic of sections 5.2 and 6.4 (threshold, rectangle choice, smallest
predicting height, fixed-height regret) on synthetic timings with known answers."""
import pytest

from paper_2306_10016_amd import study


def _rect(m_best, ms=(64, 128, 256, 512)):
    return {m: (1.0 if m == m_best else 2.0 + m * 1e-3) for m in ms}


def test_gamma_and_choice():
    ts = {64: 1.0, 128: 3.0, 256: 2.0}
    assert study.gamma(ts, 0.0) == 1.0
    assert study.gamma(ts, 0.1) == pytest.approx(1.2)
    assert study.gamma(ts, 1.0) == 3.0
    assert study.choice({64: 2.0, 128: 1.0, 256: 1.0}) == 128  # ties: the smaller m


def test_smallest_predicting_height():
    ts = {64: 1.0, 128: 1.05, 256: 1.5, 512: 2.0}
    rects = [(16, _rect(64)), (2, _rect(512)), (8, _rect(128)), (4, _rect(256))]
    assert study.smallest_predicting_height(ts, rects, 0.0) == 16
    assert study.smallest_predicting_height(ts, rects, 0.05) == 8
    assert study.smallest_predicting_height(ts, rects, 0.5) == 4
    assert study.smallest_predicting_height(ts, rects, 1.0) == 2
    assert study.smallest_predicting_height(ts, [(2, _rect(512)), (4, _rect(256))], 0.0) is None


def test_height_regret():
    ts = {64: 1.0, 128: 1.25, 256: 1.5}
    assert study.height_regret(ts, _rect(64, ts)) == 0.0
    assert study.height_regret(ts, _rect(128, ts)) == pytest.approx(0.25)
