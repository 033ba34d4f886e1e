"""Seeded synthetic workloads standing in for the paper's test videos.

The paper measures on six real videos (Akiyo, Coastguard, Hall, Rhinos,
Train, Waterfall) re-encoded to several resolutions; they are not available
here.  The cipher's work and memory traffic depend only on (w, h, n) and on
the pseudorandom shift distances, never on pixel values, so content only
matters for the statistical checks.  The generator below produces
natural-looking frames: a smooth per-channel gradient field (optionally
panning), eight moving discs of constant colour, and Gaussian noise with
sigma 4, clipped to 0..255.

Nothing here implements any part of the cipher.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np


def key_bytes(seed: int = 0) -> bytes:
    """32 key bytes from PCG64(seed)."""
    return np.random.default_rng(seed).bytes(32)


def random_frame(h: int, w: int, seed: int) -> np.ndarray:
    """i.i.d. uniform bytes, shape (h, w, 3)."""
    return np.random.default_rng(seed).integers(0, 256, (h, w, 3), dtype=np.uint8)


def config_seed(config: int, stream: int = 0) -> int:
    return 1000 * config + stream


@dataclass
class _Disc:
    cx: float
    cy: float
    vx: float
    vy: float
    r: float
    colour: np.ndarray


class SynthVideo:
    """Deterministic synthetic video: ``frame(t)`` is reproducible for any t."""

    def __init__(self, w: int, h: int, seed: int, pan: Tuple[float, float] = (0.0, 0.0), discs: int = 8):
        self.w, self.h, self.seed, self.pan = w, h, seed, pan
        rng = np.random.default_rng(seed)
        a = rng.uniform(70, 130, 3)
        b = rng.uniform(-40, 40, 3)
        c = rng.uniform(-40, 40, 3)
        d = rng.uniform(10, 40, 3)
        x = np.arange(w, dtype=np.float32) / w
        y = np.arange(h, dtype=np.float32) / h
        sx = np.sin(2 * np.pi * x)
        cy = np.cos(2 * np.pi * y)
        field = np.empty((h, w, 3), np.float32)
        for ch in range(3):
            field[:, :, ch] = (a[ch] + b[ch] * x[None, :] + c[ch] * y[:, None]
                               + d[ch] * cy[:, None] * sx[None, :])
        self._field = field
        m = min(w, h)
        self._discs: List[_Disc] = []
        for _ in range(discs):
            speed = rng.uniform(1, 6)
            ang = rng.uniform(0, 2 * np.pi)
            self._discs.append(_Disc(rng.uniform(0, w), rng.uniform(0, h), speed * math.cos(ang),
                                     speed * math.sin(ang), rng.uniform(0.03, 0.12) * m,
                                     rng.integers(0, 256, 3).astype(np.float32)))
        self._noise_seed = int(rng.integers(0, 2**63 - 1))
        self._field_i16 = np.rint(field).astype(np.int16)
        self._bank = None

    # Gaussian noise (sigma 4) comes from a bank of NOISE_BANK pre-drawn
    # fields, frame t using field t mod NOISE_BANK.
    NOISE_BANK = 8

    def _noise(self, t: int) -> np.ndarray:
        if self._bank is None:
            g = np.random.default_rng(self._noise_seed)
            self._bank = [np.clip(np.rint(4.0 * g.standard_normal((self.h, self.w, 3), dtype=np.float32)),
                                  -127, 127).astype(np.int16) for _ in range(self.NOISE_BANK)]
        return self._bank[t % self.NOISE_BANK]

    def frame(self, t: int) -> np.ndarray:
        w, h = self.w, self.h
        px = int(round(self.pan[0] * t)) % w
        py = int(round(self.pan[1] * t)) % h
        img = np.roll(self._field_i16, (py, px), axis=(0, 1))
        for dsc in self._discs:
            cx = (dsc.cx + dsc.vx * t) % w
            cy = (dsc.cy + dsc.vy * t) % h
            r = dsc.r
            x0, x1 = int(math.floor(cx - r)), int(math.ceil(cx + r)) + 1
            y0, y1 = int(math.floor(cy - r)), int(math.ceil(cy + r)) + 1
            xs = np.arange(x0, x1)
            ys = np.arange(y0, y1)
            mask = ((xs[None, :] - cx) ** 2 + (ys[:, None] - cy) ** 2) <= r * r
            yy = (ys % h)[:, None]
            xx = (xs % w)[None, :]
            yi, xi = np.broadcast_arrays(yy, xx)
            img[yi[mask], xi[mask]] = dsc.colour.astype(np.int16)
        img += self._noise(t)
        np.clip(img, 0, 255, out=img)
        return img.astype(np.uint8)

    def frames(self, T: int, start: int = 0) -> np.ndarray:
        out = np.empty((T, self.h, self.w, 3), np.uint8)
        for k in range(T):
            out[k] = self.frame(start + k)
        return out


# The workloads of the evaluation (sizes from the paper's Tab. IX resolutions
# and the benchmark plan).
CONFIG1 = dict(w=64, h=64, frames=1)            # one random 64x64 frame
CONFIG2 = dict(w=640, h=480, frames=24)         # VGA, 24 frames, one stream
CONFIG3 = dict(w=1920, h=1080, frames=300, pan=(3.0, 1.0))   # 1080p, 10 s at 30 FPS


def config1_frame() -> np.ndarray:
    return random_frame(64, 64, seed=1)


def config2_video() -> SynthVideo:
    return SynthVideo(640, 480, seed=config_seed(2))


def config3_video() -> SynthVideo:
    return SynthVideo(1920, 1080, seed=config_seed(3), pan=CONFIG3["pan"])
