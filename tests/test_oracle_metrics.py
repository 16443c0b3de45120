"""Pins for the quality indicators of Sec. 5 on hand-built confusion matrices."""
import math

import numpy as np

from oracle.metrics import confusion, indicators, score


def test_hand_built_counts():
    r = indicators(tp=5, tn=80, fp=10, fn=5)
    assert r["PWC"] == 15.0
    assert r["FNR"] == 0.5
    assert math.isclose(r["FPR"], 10 / 90)
    assert r["Si"] == 0.25


def test_confusion_from_masks():
    gt = np.array([[255, 255, 0, 0], [0, 0, 0, 255]], np.uint8)
    m = np.array([[255, 0, 255, 0], [0, 0, 0, 255]], np.uint8)
    assert confusion(m, gt) == (2, 4, 1, 1)
    r = score(m, gt)
    assert r["PWC"] == 25.0 and r["Si"] == 0.5


def test_perfect_and_empty():
    gt = np.zeros((3, 3), np.uint8)
    r = score(gt, gt)
    assert r["PWC"] == 0.0 and r["FPR"] == 0.0 and math.isnan(r["FNR"])
