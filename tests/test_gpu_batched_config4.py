"""The benchmark's batched workload of uneven shapes -- 48 streams, 16 each
of 640x480, 1280x720 and 1920x1080, 8 frames per stream, n = 32 -- in one
encrypt_frames and one decrypt_frames call after the autotuner has picked
the column-pass tiling of every shape and direction, checked against the
oracle: the first frame of every stream, and all 8 frames of one stream per
shape; every frame must decrypt back."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import require_gpu, to_np
from workload.synth import key_bytes

pytestmark = pytest.mark.gpu

RES = [(640, 480)] * 16 + [(1280, 720)] * 16 + [(1920, 1080)] * 16
F = 8


def test_config4_autotuned_batch_matches_oracle():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    kb, gamma, n = key_bytes(0), -1.0, 32
    gen = torch.Generator(device=dev)
    gen.manual_seed(4000)
    pool = [torch.randint(0, 256, (F, h, w, 3), dtype=torch.uint8, device=dev, generator=gen) for (w, h) in RES]
    frames = [pool[s][t] for s in range(len(RES)) for t in range(F)]
    sids = [s for s in range(len(RES)) for _ in range(F)]
    seqs = [t for _ in range(len(RES)) for t in range(F)]
    per_batch = sum(V.vc_scratch_per_frame(w, h, n) for (w, h) in RES) * F + (64 << 20)
    enc = V.Cipher.from_bytes(kb, gamma, n, max_streams=len(RES), scratch_bytes=per_batch)
    dec = V.Cipher.from_bytes(kb, gamma, n, max_streams=len(RES), scratch_bytes=per_batch)
    picks = {}
    for (w, h) in sorted(set(RES)):
        picks[(w, h)] = (enc.autotune(w, h, frames=F * 16, decrypt=False), dec.autotune(w, h, frames=F * 16,
                                                                                       decrypt=True))
    C = [torch.empty_like(x) for x in frames]
    P = [torch.empty_like(x) for x in frames]
    H = torch.empty((len(frames), 32), dtype=torch.uint8, device=dev)
    V.encrypt_frames(enc.ctx, frames, sids, seqs, H, C)
    V.decrypt_frames(dec.ctx, C, sids, seqs, H, P)
    torch.cuda.synchronize()
    assert all(torch.equal(p, f) for p, f in zip(P, frames))
    Hn = to_np(H)
    base = oracle.key_from_bytes(kb)
    for s in range(len(RES)):
        full = s in (0, 16, 32)                   # one stream per shape: all 8 frames
        ts = range(F) if full else range(1)
        host = [to_np(pool[s][t]) for t in ts]
        Cs, Hs, _ = oracle.encrypt_stream(base, gamma, n, host)
        for t in ts:
            k = s * F + t
            assert Hn[k].tobytes() == Hs[t], (RES[s], s, t)
            assert np.array_equal(to_np(C[k]), Cs[t]), (RES[s], s, t, picks[RES[s]])
    assert enc.status() == 0 and dec.status() == 0
    enc.close(); dec.close()
