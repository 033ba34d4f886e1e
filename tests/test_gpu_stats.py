"""GPU parity of the statistics reductions (Sec. III) against the oracle:
histograms, block histograms and adjacent-pair moments are integer counts
and must match exactly; the statistics computed from them on the host must
match the oracle's floating-point definitions to rounding."""
import math

import numpy as np
import pytest
import torch

from oracle import stats as O
from gpu_util import require_gpu, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 7), (9, 1), (2, 3), (17, 5), (64, 64), (100, 33), (481, 643), (1080, 1920)]


def frames_for(rng, shapes):
    out = []
    for k, (h, w) in enumerate(shapes):
        if k % 3 == 2:    # a smooth frame with few levels (heavy atomic contention in the histogram)
            yy, xx = np.mgrid[0:h, 0:w]
            f = np.stack([(yy // 7) % 4 * 60, (xx // 5) % 3 * 80, np.full((h, w), 255)], axis=2).astype(np.uint8)
        else:
            f = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
        out.append(f)
    return out


def test_frame_histograms_exact():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    rng = np.random.default_rng(100)
    fs = frames_for(rng, SHAPES)
    got = V.vc_frame_histograms([to_dev(f, dev) for f in fs]).cpu().numpy()
    for k, f in enumerate(fs):
        assert np.array_equal(got[k], O.frame_histograms(f)), SHAPES[k]


def test_constant_4k_frame_histogram():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    f = torch.full((2160, 3840, 3), 200, dtype=torch.uint8, device=dev)
    got = V.vc_frame_histograms([f]).cpu().numpy()
    want = np.zeros((1, 3, 256), dtype=np.int64)
    want[0, :, 200] = 2160 * 3840
    assert np.array_equal(got, want)


def test_block_histograms_exact_including_edge_blocks():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    from paper_2505_07158_amd import stats as S
    rng = np.random.default_rng(101)
    for (h, w) in [(1080, 1920), (481, 643), (264, 352)]:
        fs = [rng.integers(0, 256, (h, w, 3), dtype=np.uint8) for _ in range(3)]
        org = np.stack([S.sample_block_origins(rng, h, w) for _ in fs])
        org[1, 0] = (h - 44, w - 44)     # flush with the bottom-right corner
        got = V.vc_block_histograms([to_dev(f, dev) for f in fs], org, 44, 44).cpu().numpy()
        for k, f in enumerate(fs):
            for m, (r, c) in enumerate(org[k]):
                blk = f[r:r + 44, c:c + 44]
                assert np.array_equal(got[k, m], O.frame_histograms(blk)), ((h, w), k, m)
    # 1 x 1 blocks, and a block that is the whole frame
    f = rng.integers(0, 256, (5, 8, 3), dtype=np.uint8)
    org = np.array([[[4, 7], [0, 0], [2, 3]]], dtype=np.uint32)
    got = V.vc_block_histograms([to_dev(f, dev)], org, 1, 1).cpu().numpy()
    for m, (r, c) in enumerate(org[0]):
        assert np.array_equal(got[0, m], O.frame_histograms(f[r:r + 1, c:c + 1]))
    got = V.vc_block_histograms([to_dev(f, dev)], np.zeros((1, 1, 2), np.uint32), 8, 5).cpu().numpy()
    assert np.array_equal(got[0, 0], O.frame_histograms(f))


def test_pair_moments_exact_all_pixels_and_sampled():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    from paper_2505_07158_amd import stats as S
    rng = np.random.default_rng(102)
    fs = frames_for(rng, SHAPES)
    got = V.vc_pair_moments([to_dev(f, dev) for f in fs]).cpu().numpy()
    for k, f in enumerate(fs):
        h, w, _ = f.shape
        want = O.pair_moments(f) if h > 1 and w > 1 else np.zeros((3, 3, 5), np.int64)
        assert np.array_equal(got[k], want), SHAPES[k]
    for (h, w) in [(1080, 1920), (2, 2), (17, 5)]:
        fs = [rng.integers(0, 256, (h, w, 3), dtype=np.uint8) for _ in range(2)]
        pos = np.stack([S.sample_pair_positions(rng, h, w, 10000) for _ in fs])
        got = V.vc_pair_moments([to_dev(f, dev) for f in fs], pos).cpu().numpy()
        for k, f in enumerate(fs):
            assert np.array_equal(got[k], O.pair_moments(f, pos[k].astype(np.int64))), (h, w, k)


def test_invalid_origins_and_positions_are_rejected():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    f = torch.zeros((50, 60, 3), dtype=torch.uint8, device=dev)
    with pytest.raises(V.VcError):
        V.vc_block_histograms([f], np.array([[[7, 17]]], np.uint32), 44, 44)     # past the right edge
    with pytest.raises(V.VcError):
        V.vc_block_histograms([f], np.array([[[0, 0]]], np.uint32), 0, 4)
    with pytest.raises(V.VcError):
        V.vc_pair_moments([f], np.array([[[49, 0]]], np.uint32))                 # last row has no lower neighbour
    with pytest.raises(V.VcError):
        V.vc_pair_moments([f], np.array([[[0, 59]]], np.uint32))


def test_statistics_match_the_oracle():
    dev = require_gpu()
    from paper_2505_07158_amd import stats as S
    rng = np.random.default_rng(103)
    shapes = [(1080, 1920), (288, 352), (1080, 1920), (40, 50)]
    fs = frames_for(rng, shapes)
    st = S.frame_statistics([to_dev(f, dev) for f in fs], seed=7)
    # replay the sampler in the same order: by shape, origins then positions
    rng2 = np.random.default_rng(7)
    draws = {}
    by_shape = {}
    for k, (h, w) in enumerate(shapes):
        by_shape.setdefault((h, w), []).append(k)
    for (h, w), idx in by_shape.items():
        org = [S.sample_block_origins(rng2, h, w) for _ in idx] if (h // 44) * (w // 44) >= 30 else None
        pos = [S.sample_pair_positions(rng2, h, w) for _ in idx]
        for j, k in enumerate(idx):
            draws[k] = (None if org is None else org[j], pos[j])
    for k, f in enumerate(fs):
        org, pos = draws[k]
        H = O.frame_histograms(f)
        for c in range(3):
            assert st[k]["variance"][c] == pytest.approx(O.histogram_variance(H[c]), rel=1e-12)
            assert st[k]["chi2"][c] == pytest.approx(O.chi_square(H[c]), rel=1e-12)
            assert st[k]["entropy"][c] == pytest.approx(O.entropy(H[c]), rel=1e-12, abs=1e-15)
            if org is None:
                assert st[k]["lse"][c] is None
            else:
                assert st[k]["lse"][c] == pytest.approx(O.local_entropy(f, c, org, 44, 44), rel=1e-12, abs=1e-15)
            for d in range(3):
                want = O.correlation(f, c, d, pos.astype(np.int64))
                got = st[k]["corr"][d][c]
                if math.isnan(want):
                    assert math.isnan(got)
                else:
                    assert got == pytest.approx(want, rel=1e-9, abs=1e-12)


def test_ciphertext_statistics_are_uniform():
    """Encrypted smooth 1080p frames: mean chi-square under the critical
    value, entropy near 8, mean local entropy inside the paper's interval
    band, and no adjacent-pixel correlation (Sec. III's claims)."""
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    from paper_2505_07158_amd import stats as S
    rng = np.random.default_rng(104)
    h, w = 1080, 1920
    yy, xx = np.mgrid[0:h, 0:w]
    base = np.stack([(yy * 255) // h, (xx * 255) // w, ((yy + xx) * 255) // (h + w)], axis=2)
    P = torch.stack([to_dev((base + rng.integers(-4, 5, base.shape)).clip(0, 255).astype(np.uint8), dev)
                     for _ in range(8)])
    c = V.Cipher.from_bytes(bytes(range(32)), -1.0, 32)
    try:
        C, _ = c.encrypt(P)
    finally:
        torch.cuda.synchronize()
        c.close()
    plain = S.summarize(S.frame_statistics(list(P), seed=1))
    enc = S.summarize(S.frame_statistics(list(C), seed=1))
    assert plain["chi2"] > 10 * S.CHI2_CRITICAL and plain["corr_horizontal"] > 0.9
    assert enc["chi2"] < S.CHI2_CRITICAL
    assert enc["entropy"] > 7.9999
    assert abs(enc["lse"] - S.LSE_IDEAL) < 0.002
    for d in S.DIRECTIONS:
        assert enc[f"corr_{d}"] < 0.03


def test_bandwidth_probe_copies_and_xors():
    """The streaming reference kernel (vc_bandwidth_probe): out = a and
    out = a ^ b over a buffer that spans many workgroups and a ragged last
    one; misaligned or non-multiple-of-16 sizes are rejected."""
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    n = 16 * (256 * 1000 + 37)
    a = torch.randint(0, 256, (n,), dtype=torch.uint8, device=dev, generator=g)
    b = torch.randint(0, 256, (n,), dtype=torch.uint8, device=dev, generator=g)
    out = torch.zeros(n, dtype=torch.uint8, device=dev)
    V.vc_bandwidth_probe(0, a, b, out)
    torch.cuda.synchronize()
    assert torch.equal(out, a)
    V.vc_bandwidth_probe(1, a, b, out)
    torch.cuda.synchronize()
    assert torch.equal(out, a ^ b)
    with pytest.raises(V.VcError):
        V.vc_bandwidth_probe(1, a[1:], b[1:], out[:n - 16])      # misaligned
    with pytest.raises(V.VcError):
        V.vc_bandwidth_probe(0, a, b, out[:n - 8])               # not a multiple of 16 bytes
