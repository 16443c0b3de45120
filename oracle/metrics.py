"""Segmentation quality indicators (Sec. 5).  Oracle (test infrastructure only).

From the confusion counts of a binary mask against ground truth (foreground =
positive): PWC = 100 (FN + FP) / (TP + FN + FP + TN), FNR = FN / (TP + FN),
FPR = FP / (FP + TN), Si = TP / (TP + FP + FN).
"""
from __future__ import annotations

import numpy as np


def confusion(mask, gt):
    """(TP, TN, FP, FN) of a mask against ground truth, foreground = positive (Sec. 5)."""
    m = np.asarray(mask) != 0
    g = np.asarray(gt) != 0
    tp = int(np.count_nonzero(m & g))
    tn = int(np.count_nonzero(~m & ~g))
    fp = int(np.count_nonzero(m & ~g))
    fn = int(np.count_nonzero(~m & g))
    return tp, tn, fp, fn


def _div(a, b):
    return float(a) / float(b) if b else float("nan")


def indicators(tp: int, tn: int, fp: int, fn: int) -> dict:
    """The Sec. 5 indicators from the counts: PWC, FNR, FPR and the similarity Si."""
    return dict(PWC=100.0 * _div(fn + fp, tp + fn + fp + tn), FNR=_div(fn, tp + fn),
                FPR=_div(fp, fp + tn), Si=_div(tp, tp + fp + fn))


def score(mask, gt) -> dict:
    """The Sec. 5 indicators of one mask."""
    return indicators(*confusion(mask, gt))
