"""Statistical tests of Sec. III and the difference measures of Sec. IV of
arXiv 2505.07158, written out plainly
(numpy, fp64) from their definitions.  TEST INFRASTRUCTURE ONLY: the
library computes the same quantities from integer reductions on the GPU;
this module is what its tests compare against.

Frames are uint8 arrays of shape (h, w, 3), channels interleaved.
"""
from __future__ import annotations

import numpy as np

LEVELS = 256


def histogram(channel: np.ndarray) -> np.ndarray:
    """z_i = number of pixels of intensity i (Sec. III-A)."""
    z = np.zeros(LEVELS, dtype=np.int64)
    for v, cnt in zip(*np.unique(channel.ravel(), return_counts=True)):
        z[int(v)] = int(cnt)
    return z


def frame_histograms(frame: np.ndarray) -> np.ndarray:
    """(3, 256) histograms, one per channel."""
    return np.stack([histogram(frame[..., c]) for c in range(3)])


def histogram_variance(z: np.ndarray) -> float:
    """Eq. 4: var(Z) = (1/256^2) sum_i sum_j (z_i - z_j)^2 / 2, the double sum as written."""
    z = z.astype(np.float64)
    return float(np.sum(0.5 * (z[:, None] - z[None, :]) ** 2) / LEVELS ** 2)


def chi_square(z: np.ndarray) -> float:
    """Eq. 5: sum_i (z_i - N/256)^2 / (N/256), N = number of pixels."""
    z = z.astype(np.float64)
    e = z.sum() / LEVELS
    return float(np.sum((z - e) ** 2 / e))


def entropy(z: np.ndarray) -> float:
    """Eq. 10: H = sum p_i log2(1/p_i) over the symbols that occur (log base 2:
    a source of 2^n equiprobable symbols has entropy n)."""
    p = z.astype(np.float64) / z.sum()
    p = p[p > 0]
    return float(np.sum(p * np.log2(1.0 / p)))


def local_entropy(frame: np.ndarray, channel: int, origins: np.ndarray, bw: int, bh: int) -> float:
    """Eq. 11: mean of the entropies of the blocks of bh x bw pixels at the
    given (row, col) origins, one channel."""
    hs = [entropy(histogram(frame[r:r + bh, c:c + bw, channel])) for r, c in origins]
    return float(np.sum(hs) / len(hs))


NEIGHBOUR = {0: (0, 1), 1: (1, 0), 2: (1, 1)}   # horizontal, vertical, diagonal


def pairs(frame: np.ndarray, channel: int, direction: int, positions=None):
    """x = pixels at the positions, y = their neighbours in the direction.
    positions: (npairs, 2) of (row, col), or None for every pixel that has
    all three neighbours."""
    h, w, _ = frame.shape
    if positions is None:
        rr, cc = np.meshgrid(np.arange(h - 1), np.arange(w - 1), indexing="ij")
        positions = np.stack([rr.ravel(), cc.ravel()], axis=1)
    dr, dc = NEIGHBOUR[direction]
    r, c = positions[:, 0], positions[:, 1]
    return frame[r, c, channel].astype(np.int64), frame[r + dr, c + dc, channel].astype(np.int64)


def pair_moments(frame: np.ndarray, positions=None) -> np.ndarray:
    """(3 directions, 3 channels, 5) integer sums of x, y, x^2, y^2, xy."""
    out = np.zeros((3, 3, 5), dtype=np.int64)
    for d in range(3):
        for ch in range(3):
            x, y = pairs(frame, ch, d, positions)
            out[d, ch] = [x.sum(), y.sum(), (x * x).sum(), (y * y).sum(), (x * y).sum()]
    return out


def correlation(frame: np.ndarray, channel: int, direction: int, positions=None) -> float:
    """Eqs. 6-9: r = cov(x, y) / sqrt(D(x) D(y)) with E, D and cov as 1/N sums."""
    x, y = pairs(frame, channel, direction, positions)
    x = x.astype(np.float64)
    y = y.astype(np.float64)
    n = len(x)
    ex, ey = np.sum(x) / n, np.sum(y) / n
    cov = np.sum((x - ex) * (y - ey)) / n
    dx = np.sum((x - ex) ** 2) / n
    dy = np.sum((y - ey) ** 2) / n
    return float(cov / np.sqrt(dx * dy))


# ---------------------------------------------------------------------------
# differences between two frames (Sec. IV)
# ---------------------------------------------------------------------------

def frame_diff(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """(3, 4) per channel: differing bytes, sum |a-b|, sum (a-b)^2, differing bits."""
    out = np.zeros((3, 4), dtype=np.int64)
    for c in range(3):
        x = a[..., c].astype(np.int64).ravel()
        y = b[..., c].astype(np.int64).ravel()
        d = x - y
        out[c, 0] = np.count_nonzero(d)
        out[c, 1] = np.abs(d).sum()
        out[c, 2] = (d * d).sum()
        out[c, 3] = np.unpackbits((x ^ y).astype(np.uint8)).sum()
    return out


def npcr(a: np.ndarray, b: np.ndarray, c: int) -> float:
    """Eqs. 14 and 16: percentage of positions whose values differ, one channel."""
    return 100.0 * float(np.mean(a[..., c] != b[..., c]))


def uaci(a: np.ndarray, b: np.ndarray, c: int) -> float:
    """Eq. 15: mean absolute difference over the largest value 255, in percent."""
    d = np.abs(a[..., c].astype(np.float64) - b[..., c].astype(np.float64))
    return 100.0 * float(np.mean(d / 255.0))


def psnr(a: np.ndarray, b: np.ndarray, c=None) -> float:
    """Peak signal-to-noise ratio 10 log10(255^2 / MSE) in dB, over one channel
    or (c = None) over all three; infinite for identical data."""
    x = a.astype(np.float64) if c is None else a[..., c].astype(np.float64)
    y = b.astype(np.float64) if c is None else b[..., c].astype(np.float64)
    mse = float(np.mean((x - y) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)
