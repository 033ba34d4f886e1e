"""Differential metrics of Sec. IV-B (Eqs. 14-16) and the critical values of
the NPCR / UACI randomness tests (the ideal-cipher closed forms of the
reference the paper cites for its 512x512 thresholds)."""
from __future__ import annotations

import math

import numpy as np
from scipy.stats import norm

F = 255  # largest pixel value


def npcr_uaci(c1: np.ndarray, c2: np.ndarray):
    """Per-channel NPCR and UACI in percent (Eqs. 14-16) of two (h, w, 3)
    uint8 frames."""
    a = c1.astype(np.int32)
    b = c2.astype(np.int32)
    npcr = (a != b).mean(axis=(0, 1)) * 100.0
    uaci = (np.abs(a - b) / F).mean(axis=(0, 1)) * 100.0
    return npcr, uaci


def npcr_mean_sigma(M: int):
    mu = F / (F + 1)
    sigma = math.sqrt(F / ((F + 1) ** 2 * M))
    return 100 * mu, 100 * sigma


def uaci_mean_sigma(M: int):
    mu = (F + 2) / (3 * F + 3)
    var = (F + 2) * (F * F + 2 * F + 3) / (18 * (F + 1) ** 2 * F * M)
    return 100 * mu, 100 * math.sqrt(var)


def npcr_critical(M: int, alpha: float = 0.05) -> float:
    """One-sided lower critical NPCR (percent) for M pixels per channel."""
    mu, s = npcr_mean_sigma(M)
    return mu - norm.ppf(1 - alpha) * s


def uaci_interval(M: int, alpha: float = 0.05):
    """Two-sided UACI acceptance interval (percent)."""
    mu, s = uaci_mean_sigma(M)
    z = norm.ppf(1 - alpha / 2)
    return mu - z * s, mu + z * s
