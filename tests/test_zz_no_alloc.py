"""The allocation-free entry point (encrypt_frames_noalloc) gives the bytes,
hashes and chain states of encrypt_frames, through the C ABI, on two calls
in a row (the second smaller), with the context's regular calls before and
after it; oversized frames are rejected before anything runs."""
import numpy as np
import pytest
import torch

from gpu_util import require_gpu
from workload.synth import key_bytes

pytestmark = pytest.mark.gpu


def _frames(rng, t, h, w, dev):
    return torch.from_numpy(rng.integers(0, 256, (t, h, w, 3), dtype=np.uint8)).to(dev)


def test_noalloc_matches_encrypt_frames():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    kb, gamma, n = key_bytes(11), -1.0, 32
    ref = V.Cipher.from_bytes(kb, gamma, n, max_streams=2)
    na = V.Cipher.from_bytes(kb, gamma, n, max_streams=2)
    rng = np.random.default_rng(2024)
    # a regular call first, so that the no-alloc call follows chain work of
    # the context's own chain stream
    warm = _frames(rng, 1, 64, 64, dev)
    ref.encrypt(warm, streams=[1])
    na.encrypt(warm, streams=[1])
    # call 1: six 1080p frames need two spans of the fixed array (about
    # 12.5 MB each); call 2: three 640x480 frames of both streams
    calls = [(_frames(rng, 6, 1080, 1920, dev), [0] * 6), (_frames(rng, 3, 480, 640, dev), [0, 1, 1])]
    for frames, streams in calls:
        C1, H1 = ref.encrypt(frames, streams=streams)
        C2 = torch.empty_like(frames)
        H2 = torch.empty((frames.shape[0], 32), dtype=torch.uint8, device=dev)
        na.encrypt_noalloc(frames, C2, H2, streams=streams)
        torch.cuda.synchronize()
        assert torch.equal(H1, H2)
        assert torch.equal(C1, C2), int((C1 != C2).sum())
    # a regular call after the no-alloc ones continues the same chains
    tail = _frames(rng, 2, 120, 160, dev)
    C1, H1 = ref.encrypt(tail, streams=[0, 1])
    C2, H2 = na.encrypt(tail, streams=[0, 1])
    assert torch.equal(C1, C2) and torch.equal(H1, H2)
    for s in (0, 1):
        assert ref.get_state(s) == na.get_state(s)
    assert ref.status() == 0 and na.status() == 0
    # a frame larger than the array's data area: rejected, nothing changes
    big = torch.zeros((1, 4320, 7680, 3), dtype=torch.uint8, device=dev)
    hb = torch.empty((1, 32), dtype=torch.uint8, device=dev)
    before = na.get_state(0)
    with pytest.raises(V.VcError) as e:
        na.encrypt_noalloc(big, torch.empty_like(big), hb, streams=[0])
    assert e.value.status == V.VC_ENOMEM
    assert na.get_state(0) == before
    ref.close()
    na.close()
