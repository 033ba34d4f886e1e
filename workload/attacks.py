"""Seeded damage to ciphertext frames, standing in for the cropping attacks
and channel noise of Sec. IV-C: a cropped region is set to zero; salt-and-
pepper noise of density d sets each byte, with probability d, to 0 or 255
(equally likely); Gaussian noise of variance v (on the 0..1 intensity
scale) adds N(0, v) * 255 to each byte, rounded and clipped to 0..255.
Frames are numpy uint8 arrays (h, w, 3).

Nothing here implements any part of the cipher.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

# crop patterns: name -> list of (top, left, bottom, right) as fractions of
# the frame; each removes the stated share of the frame's area
CROPS: Dict[str, List[Tuple[float, float, float, float]]] = {
    "corner_1/16": [(0.0, 0.0, 0.25, 0.25)],
    "centre_1/16": [(0.375, 0.375, 0.625, 0.625)],
    "band_1/8": [(0.4375, 0.0, 0.5625, 1.0)],
    "half_column_1/4": [(0.0, 0.0, 1.0, 0.25)],
    "two_blocks_3/8": [(0.0, 0.0, 0.5, 0.5), (0.5, 0.5, 1.0, 0.75)],
}
SALT_PEPPER = (0.01, 0.05, 0.1, 0.2, 0.3)
GAUSSIAN_VAR = (0.0001, 0.0005, 0.001, 0.005, 0.01)


def crop_rects(h: int, w: int, pattern: str) -> List[Tuple[int, int, int, int]]:
    return [(round(t * h), round(l * w), round(b * h), round(r * w)) for t, l, b, r in CROPS[pattern]]


def crop(frame: np.ndarray, pattern: str) -> np.ndarray:
    out = frame.copy()
    h, w, _ = frame.shape
    for t, l, b, r in crop_rects(h, w, pattern):
        out[t:b, l:r] = 0
    return out


def crop_fraction(h: int, w: int, pattern: str) -> float:
    m = np.zeros((h, w), dtype=bool)
    for t, l, b, r in crop_rects(h, w, pattern):
        m[t:b, l:r] = True
    return float(m.mean())


def salt_pepper(rng: np.random.Generator, frame: np.ndarray, density: float) -> np.ndarray:
    hit = rng.random(frame.shape) < density
    val = np.where(rng.random(frame.shape) < 0.5, 0, 255).astype(np.uint8)
    return np.where(hit, val, frame)


def gaussian(rng: np.random.Generator, frame: np.ndarray, var: float) -> np.ndarray:
    noisy = frame.astype(np.float64) + rng.normal(0.0, np.sqrt(var) * 255.0, frame.shape)
    return np.clip(np.rint(noisy), 0, 255).astype(np.uint8)
