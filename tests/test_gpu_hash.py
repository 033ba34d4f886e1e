"""GPU parity of the frame hash (Sec. II-A: xor of sub-frame SHA-256
digests) against the oracle and, for one sub-frame, against hashlib."""
import hashlib

import numpy as np
import pytest
import torch

import oracle
from gpu_util import require_gpu, to_dev, to_np
from workload.synth import random_frame

pytestmark = pytest.mark.gpu


def cipher(n):
    from paper_2505_07158_amd import vcipher as V
    return V.Cipher(V.vc_key_from_bytes(bytes(32), -1.0, n))


@pytest.mark.parametrize("n", [1, 2, 3, 6, 32, 64, 65, 100, 256, 1000, 1024])
def test_hash_parity(n):
    dev = require_gpu()
    c = cipher(n)
    shapes = [(64, 64), (1, 1000), (480, 640), (7, 9), (31, 33)]
    frames = [random_frame(h, w, seed=h * w + n) for h, w in shapes]
    frames = [f for f in frames if f.size >= n]
    H = to_np(c.hash([to_dev(f, dev) for f in frames]))
    for k, f in enumerate(frames):
        assert H[k].tobytes() == oracle.frame_hash(f, n), (n, f.shape)
        if n == 1:
            assert H[k].tobytes() == hashlib.sha256(f.tobytes()).digest()
    c.close()


def test_hash_unaligned_and_batched():
    dev = require_gpu()
    c = cipher(6)
    rng = np.random.default_rng(4)
    frames, ts = [], []
    for k in range(40):
        h, w = int(rng.integers(1, 60)), int(rng.integers(1, 60))
        f = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
        if f.size < 6:
            continue
        off = int(rng.integers(0, 4))
        buf = torch.zeros(f.size + off + 5, dtype=torch.uint8, device=dev)
        t = buf[off:off + f.size].view(h, w, 3)
        t.copy_(to_dev(f, dev))
        frames.append(f)
        ts.append(t)
    H = to_np(c.hash(ts))
    for k, f in enumerate(frames):
        assert H[k].tobytes() == oracle.frame_hash(f, 6)
    c.close()
