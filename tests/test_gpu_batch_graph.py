"""Prepared batches (vc_batch_prepare / vc_batch_launch) against the oracle:
a mixed batch of several streams and shapes, launched once eagerly and
then captured with its receiver's batch in a HIP graph and replayed; every
replay must give the oracle's bytes for the next frames of each stream, and
decrypt back to the plaintext.  Between replays the program does eager work
of its own (another context's encrypt_frames, a torch reduction) and
synchronises, and every replay is checked."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import require_gpu, to_np
from workload.synth import key_bytes

pytestmark = pytest.mark.gpu

# (h, w) per stream: 16-byte rows, 4-byte rows and unaligned rows
SHAPES = {0: (48, 64), 1: (30, 44), 2: (48, 64), 3: (17, 23), 4: (64, 80)}
F = 2          # frames per stream per batch
REPLAYS = 3


def test_prepared_batch_eager_and_graph_replays():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    kb, gamma, n = key_bytes(12), -1.0, 6
    rng = np.random.default_rng(31)
    host = {s: rng.integers(0, 256, (F, h, w, 3), dtype=np.uint8) for s, (h, w) in SHAPES.items()}
    order = [(s, t) for t in range(F) for s in (3, 0, 4, 2, 1)]   # streams interleaved
    frames = [torch.from_numpy(host[s][t]).to(dev) for s, t in order]
    streams = [s for s, _ in order]
    seqs = [t for _, t in order]
    cbuf = [torch.empty_like(x) for x in frames]
    pbuf = [torch.empty_like(x) for x in frames]
    H = torch.empty((len(frames), 32), dtype=torch.uint8, device=dev)
    enc = V.Cipher.from_bytes(kb, gamma, n, max_streams=len(SHAPES))
    dec = V.Cipher.from_bytes(kb, gamma, n, max_streams=len(SHAPES))
    eb = V.Batch(enc.ctx, False, frames, streams, seqs, H, cbuf)
    db = V.Batch(dec.ctx, True, cbuf, streams, seqs, H, pbuf)

    # the oracle: each stream's F frames, repeated once per launch
    runs = 1 + REPLAYS
    ref = {}
    for s in SHAPES:
        Cs, Hs, _ = oracle.encrypt_stream(oracle.key_from_bytes(kb), gamma, n, [host[s][t] for _ in range(runs)
                                                                                 for t in range(F)])
        ref[s] = (Cs, Hs)

    def check(run):
        torch.cuda.synchronize()
        Hn = to_np(H)
        for k, (s, t) in enumerate(order):
            Cs, Hs = ref[s]
            assert Hn[k].tobytes() == Hs[run * F + t], (run, s, t)
            assert np.array_equal(to_np(cbuf[k]), Cs[run * F + t]), (run, s, t)
            assert torch.equal(pbuf[k], frames[k]), (run, s, t)

    # eager launch: frames 0..F-1 of every stream
    eb.launch()
    db.launch()
    check(0)
    assert enc.get_state(0)[1] == F   # a direct launch advances the host sequence numbers

    s_cap = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s_cap):
        eb.launch()
        db.launch()
    other = V.Cipher.from_bytes(kb, gamma, n)
    x = torch.from_numpy(host[0][0]).to(dev)
    for r in range(1, runs):
        for b in cbuf + pbuf:
            b.zero_()
        g.replay()
        check(r)
        # eager work of the program between replays
        Co, Ho = other.encrypt(x[None])
        assert int(Co.sum()) >= 0 and int(torch.count_nonzero(Ho)) > 0
        torch.cuda.synchronize()
    Cs, Hs, _ = oracle.encrypt_stream(oracle.key_from_bytes(kb), gamma, n, [host[0][0]] * (runs - 1))
    assert np.array_equal(to_np(Co)[0], Cs[-1])
    assert enc.status() == 0 and dec.status() == 0
    del g
    eb.close(); db.close()
    enc.close(); dec.close(); other.close()


def test_prepare_rejects_bad_batches():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    c = V.Cipher.from_bytes(key_bytes(1), -1.0, 4, max_streams=2)
    f = [torch.zeros((8, 8, 3), dtype=torch.uint8, device=dev) for _ in range(2)]
    o = [torch.empty_like(x) for x in f]
    H = torch.empty((2, 32), dtype=torch.uint8, device=dev)
    with pytest.raises(V.VcError) as e:
        V.Batch(c.ctx, False, f, [0, 0], [3, 3], H, o)     # seq not increasing within a stream
    assert e.value.status == V.VC_EORDER
    with pytest.raises(V.VcError) as e:
        V.Batch(c.ctx, False, f, [0, 2], [0, 0], H, o)     # stream out of range
    assert e.value.status == V.VC_EINVAL
    with pytest.raises(V.VcError) as e:
        V.Batch(c.ctx, False, f, [0, 1], [0, 0], H, f)     # output aliases input
    assert e.value.status == V.VC_EINVAL
    c.close()
