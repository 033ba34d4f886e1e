"""Statistical evaluation of frames (Sec. III of arXiv 2505.07158).

The counting runs on the GPU through the C ABI (``vc_frame_histograms``,
``vc_block_histograms``, ``vc_pair_moments``: integer histograms and exact
integer moments, see ``vcipher.py``); this module turns those counts into the
paper's statistics on the host, where each is a handful of operations per
frame and channel:

* histogram variance (Eq. 4) and chi-square (Eq. 5), from the 256-level
  histogram of each channel, with integer numerators:
  sum_i sum_j (z_i - z_j)^2 / 2 = 256 sum z^2 - N^2, so
  var = (256 sum z^2 - N^2) / 256^2 and chi^2 = (256 sum z^2 - N^2) / N;
* the correlation coefficient of adjacent pixels (Eqs. 6-9) from the sums
  of x, y, x^2, y^2 and xy: r = (N Sxy - Sx Sy) / sqrt((N Sxx - Sx^2)(N Syy - Sy^2))
  (the 1/N factors of cov and D cancel);
* information entropy (Eq. 10, base-2 logarithm, so 256 equiprobable levels
  give 8) and local Shannon entropy (Eq. 11: the mean entropy of k blocks of
  T_B pixels).

Random choices (pixel pairs, block origins) come from seeded generators
here and are passed to the kernels as inputs.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import vcipher as V

LEVELS = 256
# Sec. III-A: critical chi-square value, 255 degrees of freedom, alpha = 0.05
CHI2_CRITICAL = 293.25
# Sec. III-B: adjacent pairs drawn per frame for the correlation coefficients
CORR_PAIRS = 10000
# Sec. III-C: k blocks of T_B = 44 x 44 pixels, and the acceptance interval
# of the local Shannon entropy at alpha = 0.001 (ideal value 7.902469317)
LSE_BLOCKS = 30
LSE_SIDE = 44
LSE_IDEAL = 7.902469317
LSE_INTERVAL = (7.901515798, 7.903422936)
DIRECTIONS = ("horizontal", "vertical", "diagonal")


# ---------------------------------------------------------------------------
# seeded sampling
# ---------------------------------------------------------------------------

def sample_pair_positions(rng: np.random.Generator, h: int, w: int, npairs: int = CORR_PAIRS) -> np.ndarray:
    """(npairs, 2) uint32 (row, col), uniform over the pixels that have a
    right, a lower and a lower-right neighbour (rows < h-1, cols < w-1); the
    same positions serve the three directions."""
    if h < 2 or w < 2:
        raise ValueError("adjacent pairs need a frame of at least 2 x 2 pixels")
    idx = rng.integers(0, (h - 1) * (w - 1), npairs)
    return np.stack([idx // (w - 1), idx % (w - 1)], axis=1).astype(np.uint32)


def sample_block_origins(rng: np.random.Generator, h: int, w: int, k: int = LSE_BLOCKS,
                         side: int = LSE_SIDE) -> np.ndarray:
    """(k, 2) uint32 top-left corners of k distinct, non-overlapping side x side
    blocks: k cells drawn without replacement from the grid of side x side
    cells that tile the frame from its top-left corner."""
    gr, gc = h // side, w // side
    if gr * gc < k:
        raise ValueError(f"a {h}x{w} frame holds fewer than {k} blocks of {side}x{side}")
    cells = rng.choice(gr * gc, size=k, replace=False)
    return np.stack([(cells // gc) * side, (cells % gc) * side], axis=1).astype(np.uint32)


# ---------------------------------------------------------------------------
# statistics from counts (host, exact integer numerators)
# ---------------------------------------------------------------------------

def _sums(z: Sequence[int]):
    n = sum(int(v) for v in z)
    s2 = sum(int(v) * int(v) for v in z)
    return n, s2


def histogram_variance(z: Sequence[int]) -> float:
    """Eq. 4 for one 256-level histogram."""
    n, s2 = _sums(z)
    return (LEVELS * s2 - n * n) / LEVELS ** 2


def chi_square(z: Sequence[int]) -> float:
    """Eq. 5 for one 256-level histogram of N = sum z pixels."""
    n, s2 = _sums(z)
    return (LEVELS * s2 - n * n) / n


def entropy(z: Sequence[int]) -> float:
    """Eq. 10 in bits over the levels that occur."""
    z = np.asarray(z, dtype=np.float64)
    n = z.sum()
    p = z[z > 0] / n
    return float(-(p * np.log2(p)).sum())


def correlation(m: Sequence[int], npairs: int) -> float:
    """Eqs. 6-9 from (Sx, Sy, Sxx, Syy, Sxy) over npairs pairs; NaN when
    either variable is constant (the coefficient is then undefined)."""
    sx, sy, sxx, syy, sxy = (int(v) for v in m)
    num = npairs * sxy - sx * sy
    dx = npairs * sxx - sx * sx
    dy = npairs * syy - sy * sy
    if dx == 0 or dy == 0:
        return float("nan")
    return num / math.sqrt(dx * dy)


# ---------------------------------------------------------------------------
# frames in, statistics out
# ---------------------------------------------------------------------------

def frame_statistics(frames, seed: int = 0, pairs: Optional[int] = CORR_PAIRS, lse_blocks: int = LSE_BLOCKS,
                     lse_side: int = LSE_SIDE, stream=None) -> List[Dict[str, list]]:
    """Sec. III statistics of each frame (device uint8 tensors (h, w, 3)).

    Per frame, each a list over the three channels (in memory order):
    ``variance``, ``chi2``, ``entropy``, ``lse`` (None when the frame holds
    fewer than ``lse_blocks`` blocks) and ``corr`` (three directions, each
    a list over channels).  ``pairs`` = None correlates every pixel with its
    neighbours instead of a sample.  Random positions come from
    ``numpy.random.default_rng(seed)``, frame after frame."""
    frames = list(frames)
    if not frames:
        return []
    rng = np.random.default_rng(seed)
    hist = V.vc_frame_histograms(frames, stream=stream).cpu().numpy()
    out = [{"variance": [histogram_variance(hist[f, c]) for c in range(3)],
            "chi2": [chi_square(hist[f, c]) for c in range(3)],
            "entropy": [entropy(hist[f, c]) for c in range(3)]} for f in range(len(frames))]
    # block histograms and pair moments, one launch per frame shape
    by_shape: Dict[tuple, List[int]] = {}
    for f, t in enumerate(frames):
        by_shape.setdefault(tuple(t.shape[:2]), []).append(f)
    for (h, w), idx in by_shape.items():
        group = [frames[f] for f in idx]
        if (h // lse_side) * (w // lse_side) >= lse_blocks:
            origins = np.stack([sample_block_origins(rng, h, w, lse_blocks, lse_side) for _ in idx])
            bh = V.vc_block_histograms(group, origins, lse_side, lse_side, stream=stream).cpu().numpy()
            for j, f in enumerate(idx):
                out[f]["lse"] = [sum(entropy(bh[j, m, c]) for m in range(lse_blocks)) / lse_blocks
                                 for c in range(3)]
        else:
            for f in idx:
                out[f]["lse"] = [None, None, None]
        if h < 2 or w < 2:
            for f in idx:
                out[f]["corr"] = [[float("nan")] * 3 for _ in range(3)]
            continue
        if pairs:
            pos = np.stack([sample_pair_positions(rng, h, w, pairs) for _ in idx])
            npairs = pairs
        else:
            pos, npairs = None, (h - 1) * (w - 1)
        mom = V.vc_pair_moments(group, pos, stream=stream).cpu().numpy()
        for j, f in enumerate(idx):
            out[f]["corr"] = [[correlation(mom[j, d, c], npairs) for c in range(3)] for d in range(3)]
    return out


def summarize(stats: List[Dict[str, list]]) -> Dict[str, float]:
    """Means over frames and channels, as the paper's tables report them:
    variance, chi-square (and the fraction below the critical value),
    entropy, local Shannon entropy (and the fraction inside the interval),
    and the mean absolute correlation per direction."""
    def flat(key):
        return [v for s in stats for v in s[key] if v is not None]

    chi = flat("chi2")
    lse = flat("lse")
    res = {
        "frames": len(stats),
        "variance": float(np.mean(flat("variance"))),
        "chi2": float(np.mean(chi)),
        "chi2_pass": float(np.mean([c < CHI2_CRITICAL for c in chi])),
        "entropy": float(np.mean(flat("entropy"))),
    }
    if lse:
        res["lse"] = float(np.mean(lse))
        res["lse_pass"] = float(np.mean([LSE_INTERVAL[0] < v < LSE_INTERVAL[1] for v in lse]))
    for d, name in enumerate(DIRECTIONS):
        vals = [abs(v) for s in stats for v in s["corr"][d] if not math.isnan(v)]
        res[f"corr_{name}"] = float(np.mean(vals)) if vals else float("nan")
    return res
