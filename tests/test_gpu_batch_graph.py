"""Prepared batches (vc_batch_prepare / vc_batch_launch) against the oracle:
a mixed batch of several streams and shapes, launched once eagerly and
then captured with its receiver's batch in a HIP graph and replayed; every
replay must give the oracle's bytes for the next frames of each stream, and
decrypt back to the plaintext.  Between replays the program does eager
work of its own (another context's encrypt_frames, a torch reduction) and
synchronises, and every replay is checked.  The staged form (hash-only and
encrypt-from-hashes batches) runs in graphs over three buffer sets."""
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
    import ctypes as C
    for mode in (4, -1):                                    # not a mode
        h = C.c_void_p()
        rc = V.lib.vc_batch_prepare(C.c_void_p(c.ctx), mode, 2, V._ptrs(f), V._shapes(f, [0, 1], [0, 0]),
                                    C.c_void_p(H.data_ptr()), V._ptrs(o), C.byref(h))
        assert rc == V.VC_EINVAL and not h.value
    with pytest.raises(V.VcError) as e:
        V.Batch(c.ctx, "encrypt", f, [0, 1], [0, 0], H, None)   # only a hash batch may omit out
    assert e.value.status == V.VC_EINVAL
    c.close()


def test_staged_batches_in_three_set_graphs():
    """Hash-only and encrypt-from-hashes batches (VC_PREP_HASH,
    VC_PREP_ENCRYPT_HASHED) over three buffer sets: replay r hashes block
    r + 2, encrypts block r + 1 from its stored hashes and decrypts block r,
    each on its own forked capture stream (three graphs, one per rotation of
    the sets).  Every replay is checked against the oracle: the hashes, the
    ciphertext and the decrypted plaintext; a hash batch does not move the
    chain."""
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    kb, gamma, n = key_bytes(13), -1.0, 6
    rng = np.random.default_rng(32)
    NS = 3
    host = [{s: rng.integers(0, 256, (F, h, w, 3), dtype=np.uint8) for s, (h, w) in SHAPES.items()}
            for _ in range(NS)]
    order = [(s, t) for t in range(F) for s in (3, 0, 4, 2, 1)]
    streams = [s for s, _ in order]
    seqs = [t for _, t in order]
    frames = [[torch.from_numpy(host[j][s][t]).to(dev) for s, t in order] for j in range(NS)]
    cbuf = [[torch.empty_like(x) for x in frames[j]] for j in range(NS)]
    pbuf = [[torch.empty_like(x) for x in frames[j]] for j in range(NS)]
    H = [torch.zeros((len(order), 32), dtype=torch.uint8, device=dev) for _ in range(NS)]
    enc = V.Cipher.from_bytes(kb, gamma, n, max_streams=len(SHAPES))
    dec = V.Cipher.from_bytes(kb, gamma, n, max_streams=len(SHAPES))
    hb = [V.Batch(enc.ctx, "hash", frames[j], streams, seqs, H[j], None) for j in range(NS)]
    eb = [V.Batch(enc.ctx, "encrypt_hashed", frames[j], streams, seqs, H[j], cbuf[j]) for j in range(NS)]
    db = [V.Batch(dec.ctx, "decrypt", cbuf[j], streams, seqs, H[j], pbuf[j]) for j in range(NS)]

    REPL = 4
    blocks = REPL + 2                       # hashed: 0 .. REPL+1, encrypted: 0 .. REPL, decrypted: 0 .. REPL-1
    ref = {}
    for s in SHAPES:
        Cs, Hs, _ = oracle.encrypt_stream(oracle.key_from_bytes(kb), gamma, n,
                                          [host[b % NS][s][t] for b in range(blocks) for t in range(F)])
        ref[s] = (Cs, Hs)

    def check_hash(b):
        Hn = to_np(H[b % NS])
        for k, (s, t) in enumerate(order):
            assert Hn[k].tobytes() == ref[s][1][b * F + t], ("hash", b, s, t)

    def check_enc(b):
        for k, (s, t) in enumerate(order):
            assert np.array_equal(to_np(cbuf[b % NS][k]), ref[s][0][b * F + t]), ("enc", b, s, t)

    def check_dec(b):
        for k in range(len(order)):
            assert torch.equal(pbuf[b % NS][k], frames[b % NS][k]), ("dec", b, k)

    # prologue, eager: hash blocks 0 and 1, encrypt block 0
    hb[0].launch()
    before = enc.get_state(0)
    eb[0].launch()
    hb[1].launch()
    torch.cuda.synchronize()
    assert enc.get_state(0)[1] == before[1] + F      # only the encrypt launch advanced stream 0
    check_hash(0); check_hash(1); check_enc(0)

    s0, s1, s2 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    graphs = []
    for j in range(NS):                     # graph j: replays r with r % 3 == j
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s0):
            fork = torch.cuda.Event()
            fork.record(s0)
            s1.wait_event(fork)
            s2.wait_event(fork)
            hb[(j + 2) % NS].launch(s0)     # block r + 2
            eb[(j + 1) % NS].launch(s1)     # block r + 1
            db[j].launch(s2)                # block r
            for st in (s1, s2):
                join = torch.cuda.Event()
                join.record(st)
                s0.wait_event(join)
        graphs.append(g)
    other = V.Cipher.from_bytes(kb, gamma, n)
    x = frames[0][0]
    for r in range(REPL):
        for b_ in pbuf[r % NS]:
            b_.zero_()
        graphs[r % NS].replay()
        torch.cuda.synchronize()
        check_hash(r + 2); check_enc(r + 1); check_dec(r)
        Co, _ = other.encrypt(x[None])       # eager work of the program between replays
        torch.cuda.synchronize()
    assert enc.status() == 0 and dec.status() == 0 and other.status() == 0
    del graphs
    for b_ in hb + eb + db:
        b_.close()
    enc.close(); dec.close(); other.close()
