"""The continuous-batching loop on the GPU: each stream's result is the same
alone and in the mix (mixed resolutions, encrypt and decrypt requests,
out-of-order arrivals, batches of several streams in flight at once), and
every served frame equals the oracle's encryption or the plaintext."""
import random

import numpy as np
import pytest
import torch

import oracle
from gpu_util import require_gpu, to_dev, to_np
from workload.synth import SynthVideo, key_bytes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("per_class,hash_first", [(False, False), (True, False), (True, True)])
def test_results_alone_equal_results_in_the_mix(per_class, hash_first):
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    from paper_2505_07158_amd.serving import GpuBackend, Request, Scheduler

    kb, gamma, n, T = key_bytes(21), -1.0, 8, 5
    enc_shapes = [(48, 64), (64, 96), (96, 128), (48, 64)]   # (h, w)
    dec_shapes = [(64, 96), (32, 40)]
    vids = {("enc", s): SynthVideo(w, h, seed=2100 + s).frames(T) for s, (h, w) in enumerate(enc_shapes)}
    vids.update({("dec", s): SynthVideo(w, h, seed=2200 + s).frames(T) for s, (h, w) in enumerate(dec_shapes)})

    # alone: every encrypt stream on a fresh context of its own
    alone = {}
    for s in range(len(enc_shapes)):
        c = V.Cipher.from_bytes(kb, gamma, n)
        C, H = c.encrypt(to_dev(vids[("enc", s)], dev))
        alone[s] = (to_np(C), to_np(H))
        c.close()
    # ciphertext for the decrypt streams from a separate sender context
    sender = V.Cipher.from_bytes(kb, gamma, n, max_streams=len(dec_shapes))
    dec_in = {}
    for s in range(len(dec_shapes)):
        C, H = sender.encrypt(to_dev(vids[("dec", s)], dev), streams=[s] * T)
        dec_in[s] = (C, H)
    sender.close()
    torch.cuda.synchronize()

    shape_of = {("enc", s): sh for s, sh in enumerate(enc_shapes)}
    shape_of.update({("dec", s): sh for s, sh in enumerate(dec_shapes)})
    cls = (lambda r: shape_of[(r.kind, r.stream)]) if per_class else None
    be = GpuBackend(kb, gamma, n, max_streams=8, scratch_bytes=64 << 20, batch_class=cls,
                    classes=sorted(set(shape_of.values())) if per_class else None, hash_first=hash_first)
    sched = Scheduler(be.launch, hbm_budget=1 << 30, max_inflight=2, max_batch=5, batch_class=cls,
                      hash_first=hash_first)
    reqs = []
    for (kind, s), v in vids.items():
        for t in range(T):
            if kind == "enc":
                frame = to_dev(v[t], dev)
                hashes = torch.empty(32, dtype=torch.uint8, device=dev)
            else:
                frame = dec_in[s][0][t]
                hashes = dec_in[s][1][t]
            reqs.append(Request(stream=s, seq=t, kind=kind, frame=frame, out=torch.empty_like(frame), hashes=hashes,
                                nbytes=be.footprint(frame.shape[1], frame.shape[0])))
    order = list(reqs)
    random.Random(5).shuffle(order)     # arrivals out of order, also within a stream
    torch.cuda.synchronize()
    for r in order:
        sched.submit(r)
        sched.pump()
    while not sched.idle():
        sched.pump()
    torch.cuda.synchronize()
    assert len(sched.completed) == len(reqs)
    assert any(k == "enc" and size > 1 for k, size in sched.batches), sched.batches
    assert any(k == "hash" for k, _ in sched.batches) == hash_first
    base = oracle.key_from_bytes(kb)
    ref = {}
    for (kind, s), v in vids.items():
        Cs, Hs, _ = oracle.encrypt_stream(base, gamma, n, list(v))
        ref[(kind, s)] = (Cs, Hs)
    for s in range(len(dec_shapes)):          # the sender's ciphertext is the oracle's
        Cs, Hs = ref[("dec", s)]
        for t in range(T):
            assert np.array_equal(to_np(dec_in[s][0][t]), Cs[t]) and to_np(dec_in[s][1][t]).tobytes() == Hs[t]
    for r in reqs:
        if r.kind == "enc":
            C, H = alone[r.stream]
            Cs, Hs = ref[("enc", r.stream)]
            assert np.array_equal(to_np(r.out), C[r.seq]), (r.stream, r.seq)
            assert np.array_equal(to_np(r.out), Cs[r.seq]), (r.stream, r.seq)
            assert to_np(r.hashes).tobytes() == H[r.seq].tobytes() == Hs[r.seq]
        else:
            assert np.array_equal(to_np(r.out), vids[("dec", r.stream)][r.seq]), (r.stream, r.seq)
    assert be.status_ok()
    be.close()
