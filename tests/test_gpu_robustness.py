"""GPU parity of the Sec. IV experiments against the oracle: the difference
counts of vc_frame_diff exactly; decryption of cropped and noisy 1080p
ciphertext byte for byte (with the damage staying local: as many plaintext
bits differ as ciphertext bits were damaged); decryption under keys moved
by 1e-14 byte for byte."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import stats as O
from gpu_util import require_gpu, to_dev, to_np
from workload import attacks as A
from workload.synth import SynthVideo

pytestmark = pytest.mark.gpu


def test_frame_diff_exact():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    rng = np.random.default_rng(200)
    shapes = [(1, 1), (2, 3), (17, 5), (64, 64), (481, 643), (1080, 1920), (2160, 3840)]
    a, b = [], []
    for k, (h, w) in enumerate(shapes):
        x = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
        y = x.copy() if k == 3 else A.salt_pepper(rng, x, 0.3) if k % 2 else rng.integers(0, 256, (h, w, 3),
                                                                                           dtype=np.uint8)
        a.append(x)
        b.append(y)
    da = [to_dev(x, dev) for x in a]
    # odd byte offsets for the second operand
    db = []
    for y in b:
        buf = torch.zeros(y.size + 1, dtype=torch.uint8, device=dev)
        t = buf[1:].view(*y.shape)
        t.copy_(to_dev(y, dev))
        db.append(t)
    got = V.vc_frame_diff(da, db).cpu().numpy()
    for k in range(len(shapes)):
        assert np.array_equal(got[k], O.frame_diff(a[k], b[k])), shapes[k]
    with pytest.raises(ValueError):
        V.vc_frame_diff(da[:2], [db[0], db[0]])


ATTACKS = [("crop", p) for p in A.CROPS] + [("salt_pepper", d) for d in (0.05, 0.3)] + \
          [("gaussian", v) for v in (0.0005, 0.01)]


@pytest.fixture(scope="module")
def encrypted_1080p():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    video = SynthVideo(1920, 1080, seed=77, pan=(3.0, 1.0))
    P = video.frames(2)
    kb = bytes(range(32, 64))
    enc = V.Cipher.from_bytes(kb, -1.0, 32)
    try:
        C, H = enc.encrypt(to_dev(P, dev))
        torch.cuda.synchronize()
    finally:
        enc.close()
    return kb, P, to_np(C), to_np(H)


@pytest.mark.parametrize("kind,level", ATTACKS)
def test_damaged_ciphertext_decrypts_like_the_oracle(encrypted_1080p, kind, level):
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    from paper_2505_07158_amd import robustness as R
    kb, P, C, H = encrypted_1080p
    rng = np.random.default_rng(300 + ATTACKS.index((kind, level)))
    Cd = np.stack([A.crop(c, level) if kind == "crop" else
                   A.salt_pepper(rng, c, level) if kind == "salt_pepper" else A.gaussian(rng, c, level) for c in C])
    dec = V.Cipher.from_bytes(kb, -1.0, 32)
    try:
        Pd = dec.decrypt(to_dev(Cd, dev), to_dev(H, dev))
        torch.cuda.synchronize()
    finally:
        dec.close()
    got = to_np(Pd)
    # frame 0 against the oracle, byte for byte
    want0, _ = oracle.decrypt_frame(oracle.key_from_bytes(kb), -1.0, 32, Cd[0], H[0].tobytes())
    assert np.array_equal(got[0], want0)
    # damage stays local, in both frames; PSNR from the GPU counts equals the oracle's
    dc = V.vc_frame_diff(list(to_dev(C, dev)), list(to_dev(Cd, dev))).cpu().numpy()
    res = R.frame_diff(list(Pd), list(to_dev(P, dev)))
    for t in range(2):
        assert res[t]["bits"] == int(dc[t, :, 3].sum()) > 0
        assert res[t]["psnr_all"] == pytest.approx(O.psnr(got[t], P[t]), rel=1e-12)


def test_key_sensitivity_decrypts_like_the_oracle():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    from paper_2505_07158_amd import robustness as R
    rng = np.random.default_rng(201)
    frames = rng.integers(0, 256, (3, 128, 160, 3), dtype=np.uint8)
    kb = bytes(range(7, 39))
    key = V.vc_key_from_bytes(kb, -1.0, 16)
    res = R.key_sensitivity(key, to_dev(frames, dev), delta=1e-14)
    assert all(r["bits"] == 0 for r in res["correct"])
    # the first frame decrypted under x0 + 1e-14, against the oracle
    enc_c, enc_h, _ = oracle.encrypt_frame(oracle.key_from_bytes(kb), -1.0, 16, frames[0])
    base = oracle.key_from_bytes(kb)
    for j, var in enumerate(R.VARIABLES):
        moved = base.copy()
        moved[j] = moved[j] + 1e-14
        Pw, _ = oracle.decrypt_frame(moved, -1.0, 16, enc_c, enc_h)
        d = O.frame_diff(Pw, frames[0])
        assert res[var][0]["bits"] == int(d[:, 3].sum()), var
        for c in range(3):
            assert res[var][0]["npcr"][c] == pytest.approx(O.npcr(Pw, frames[0], c), rel=1e-12)
        assert not math.isnan(res[var][0]["psnr_all"])
