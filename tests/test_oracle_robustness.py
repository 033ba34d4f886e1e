"""Pins of the oracle's difference measures (Sec. IV: NPCR Eqs. 14 and 16,
UACI Eq. 15, PSNR) and of the robustness property the experiments of
Sec. IV-C rest on, plus checks of the seeded attack generators.

* Closed forms: all-0 vs all-255 gives NPCR = UACI = 100; a least
  significant bit flip everywhere gives NPCR 100, UACI 100/255 and one
  differing bit per byte; a constant offset k gives PSNR 10 log10(255^2/k^2);
  identical frames give no difference and infinite PSNR; a brute-force loop
  on a tiny pair.
* Error locality (no diffusion, Sec. VI): decrypting damaged ciphertext with
  the sender's hash damages exactly as many plaintext bits as ciphertext
  bits were damaged, for crops and noise alike; for random plaintext the MSE
  is the bit-error rate times sum 4^k = 21845 (each damaged bit moves its
  byte by 2^k up or down).
* The library's host formulas from counts equal the oracle's measures."""
import math

import numpy as np
import pytest

import oracle
from oracle import stats as O
from workload import attacks as A


def test_diff_closed_forms():
    z = np.zeros((6, 7, 3), np.uint8)
    f = np.full((6, 7, 3), 255, np.uint8)
    for c in range(3):
        assert O.npcr(z, f, c) == 100.0 and O.uaci(z, f, c) == 100.0
    assert np.array_equal(O.frame_diff(z, f), np.array([[42, 42 * 255, 42 * 255 ** 2, 42 * 8]] * 3))
    rng = np.random.default_rng(1)
    a = rng.integers(0, 256, (9, 11, 3), dtype=np.uint8)
    b = a ^ 1
    for c in range(3):
        assert O.npcr(a, b, c) == 100.0
        assert O.uaci(a, b, c) == pytest.approx(100.0 / 255.0, rel=1e-14)
    assert (O.frame_diff(a, b)[:, 3] == 99).all()
    a = rng.integers(0, 200, (9, 11, 3), dtype=np.uint8)
    assert O.psnr(a, a + 7) == pytest.approx(10 * math.log10(255 ** 2 / 49), rel=1e-14)
    assert O.psnr(a, a) == math.inf and not O.frame_diff(a, a).any()


def test_diff_brute_force():
    rng = np.random.default_rng(2)
    a = rng.integers(0, 256, (3, 4, 3), dtype=np.uint8)
    b = a.copy()
    b[rng.random(a.shape) < 0.5] = rng.integers(0, 256, 1)[0]
    want = np.zeros((3, 4), np.int64)
    for r in range(3):
        for x in range(4):
            for c in range(3):
                p, q = int(a[r, x, c]), int(b[r, x, c])
                want[c] += [p != q, abs(p - q), (p - q) ** 2, bin(p ^ q).count("1")]
    assert np.array_equal(O.frame_diff(a, b), want)


def test_attack_generators():
    for name in A.CROPS:
        share = float(name.split("_")[-1].split("/")[0]) / float(name.split("/")[-1])
        assert A.crop_fraction(1080, 1920, name) == pytest.approx(share, abs=1e-3), name
    rng = np.random.default_rng(3)
    f = rng.integers(1, 255, (200, 300, 3), dtype=np.uint8)
    cr = A.crop(f, "two_blocks_3/8")
    assert (cr == 0).mean() == pytest.approx(0.375, abs=1e-3) and np.array_equal(cr[cr != 0], f[cr != 0])
    sp = A.salt_pepper(rng, f, 0.1)
    hit = sp != f
    assert hit.mean() == pytest.approx(0.1, abs=0.005)
    assert set(np.unique(sp[hit])) <= {0, 255} and (sp[hit] == 0).mean() == pytest.approx(0.5, abs=0.02)
    g = A.gaussian(rng, np.full((300, 300, 3), 128, np.uint8), 0.001)
    assert (g.astype(float) - 128).std() == pytest.approx(math.sqrt(0.001) * 255, rel=0.02)


@pytest.mark.parametrize("attack", ["crop", "salt_pepper", "gaussian"])
def test_oracle_decryption_damage_is_local(attack):
    rng = np.random.default_rng(4)
    h, w, n = 96, 128, 8
    P = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    key = oracle.key_from_bytes(bytes(range(32)))
    C, H, _ = oracle.encrypt_frame(key, -1.0, n, P)
    if attack == "crop":
        Cd = A.crop(C, "two_blocks_3/8")
    elif attack == "salt_pepper":
        Cd = A.salt_pepper(rng, C, 0.1)
    else:
        Cd = A.gaussian(rng, C, 0.001)
    Pd, _ = oracle.decrypt_frame(key, -1.0, n, Cd, H)
    dc = O.frame_diff(C, Cd)[:, 3].sum()
    dp = O.frame_diff(P, Pd)
    assert dp[:, 3].sum() == dc > 0
    # random plaintext: MSE = bit-error rate x 21845
    q = dc / (8 * 3 * h * w)
    mse = dp[:, 2].sum() / (3 * h * w)
    assert mse == pytest.approx(q * 21845, rel=0.1)


def test_library_diff_formulas_match_the_oracle():
    from paper_2505_07158_amd import robustness as R
    rng = np.random.default_rng(5)
    a = rng.integers(0, 256, (40, 50, 3), dtype=np.uint8)
    b = A.salt_pepper(rng, a, 0.2)
    cnt = O.frame_diff(a, b)
    m = 40 * 50
    for c in range(3):
        assert 100.0 * cnt[c, 0] / m == pytest.approx(O.npcr(a, b, c), rel=1e-14)
        assert 100.0 * cnt[c, 1] / (255.0 * m) == pytest.approx(O.uaci(a, b, c), rel=1e-12)
        assert R.psnr_from_mse(cnt[c, 2] / m) == pytest.approx(O.psnr(a, b, c), rel=1e-12)
    assert R.psnr_from_mse(cnt[:, 2].sum() / (3 * m)) == pytest.approx(O.psnr(a, b), rel=1e-12)
    assert R.psnr_from_mse(0) == math.inf
    k = R.perturbed_key(R.V.vc_key_from_bytes(bytes(range(32)), -1.0, 4), "z0", 1e-14)
    base = R.V.vc_key_from_bytes(bytes(range(32)), -1.0, 4)
    assert k.z0 == base.z0 + 1e-14 and k.z0 != base.z0 and (k.x0, k.y0, k.w0, k.n) == (base.x0, base.y0, base.w0, 4)
