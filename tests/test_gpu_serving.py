"""The library's serving loop (vc_server) on the GPU: each stream's result is
the same alone and in the mix (mixed resolutions, encrypt and decrypt
requests, out-of-order arrivals, batches of several streams in flight at
once), and every served frame equals the oracle's encryption or the
plaintext; the native trace replay gives the same bytes."""
import random

import numpy as np
import pytest
import torch

import oracle
from gpu_util import require_gpu, to_dev, to_np
from workload.synth import SynthVideo, key_bytes

pytestmark = pytest.mark.gpu

ENC_SHAPES = [(48, 64), (64, 96), (96, 128), (48, 64)]   # (h, w) per encrypt stream
DEC_SHAPES = [(64, 96), (32, 40)]                        # per decrypt stream
T = 5


def workload(dev, kb, gamma, n):
    from paper_2505_07158_amd import vcipher as V
    vids = {("enc", s): SynthVideo(w, h, seed=2100 + s).frames(T) for s, (h, w) in enumerate(ENC_SHAPES)}
    vids.update({("dec", s): SynthVideo(w, h, seed=2200 + s).frames(T) for s, (h, w) in enumerate(DEC_SHAPES)})
    # ciphertext for the decrypt streams from a separate sender context
    sender = V.Cipher.from_bytes(kb, gamma, n, max_streams=len(DEC_SHAPES))
    dec_in = {}
    for s in range(len(DEC_SHAPES)):
        C, H = sender.encrypt(to_dev(vids[("dec", s)], dev), streams=[s] * T)
        dec_in[s] = (C, H)
    torch.cuda.synchronize()
    sender.close()
    return vids, dec_in


def requests(dev, vids, dec_in):
    from paper_2505_07158_amd.serving import Server
    reqs, bufs = [], []
    for (kind, s), v in vids.items():
        for t in range(T):
            if kind == "enc":
                frame = to_dev(v[t], dev)
                hashes = torch.zeros(32, dtype=torch.uint8, device=dev)
            else:
                frame, hashes = dec_in[s][0][t], dec_in[s][1][t]
            out = torch.empty_like(frame)
            bufs.append((kind, s, t, frame, out, hashes))
            reqs.append(Server.request(len(reqs), kind, s, t, frame, out, hashes))
    return reqs, bufs


def check(bufs, vids, dec_in, kb, gamma, n, alone):
    base = oracle.key_from_bytes(kb)
    ref = {key: oracle.encrypt_stream(base, gamma, n, list(v))[:2] for key, v in vids.items()}
    for s in range(len(DEC_SHAPES)):          # the sender's ciphertext is the oracle's
        Cs, Hs = ref[("dec", s)]
        for t in range(T):
            assert np.array_equal(to_np(dec_in[s][0][t]), Cs[t]) and to_np(dec_in[s][1][t]).tobytes() == Hs[t]
    for kind, s, t, frame, out, hashes in bufs:
        if kind == "enc":
            Cs, Hs = ref[("enc", s)]
            Ca, Ha = alone[s]
            assert np.array_equal(to_np(out), Ca[t]) and np.array_equal(to_np(out), Cs[t]), (s, t)
            assert to_np(hashes).tobytes() == Ha[t].tobytes() == Hs[t], (s, t)
        else:
            assert np.array_equal(to_np(out), vids[("dec", s)][t]), (s, t)


def streams_alone(dev, vids, kb, gamma, n):
    from paper_2505_07158_amd import vcipher as V
    alone = {}
    for s in range(len(ENC_SHAPES)):
        c = V.Cipher.from_bytes(kb, gamma, n)
        C, H = c.encrypt(to_dev(vids[("enc", s)], dev))
        alone[s] = (to_np(C), to_np(H))
        c.close()
    return alone


@pytest.mark.parametrize("hash_first,max_inflight", [(False, 2), (True, 2), (False, 1)])
def test_results_alone_equal_results_in_the_mix(hash_first, max_inflight):
    dev = require_gpu()
    from paper_2505_07158_amd.serving import Server
    kb, gamma, n = key_bytes(21), -1.0, 8
    vids, dec_in = workload(dev, kb, gamma, n)
    alone = streams_alone(dev, vids, kb, gamma, n)
    classes = sorted({(w, h) for h, w in ENC_SHAPES + DEC_SHAPES})
    srv = Server(kb, gamma, n, classes, max_streams=8, hbm_budget=1 << 30, max_inflight=max_inflight, max_batch=5,
                 hash_first=hash_first, scratch_bytes=64 << 20)
    reqs, bufs = requests(dev, vids, dec_in)
    order = list(reqs)
    random.Random(5).shuffle(order)     # arrivals out of order, also within a stream
    torch.cuda.synchronize()
    done = []
    for r in order:
        srv.submit(r)
        srv.pump()
        done += srv.poll()
    while not srv.idle():
        srv.pump()
        done += srv.poll()
    torch.cuda.synchronize()
    assert sorted(c.tag for c in done) == list(range(len(reqs)))
    st = srv.stats()
    assert st.batches_launched < len(reqs) + (len(ENC_SHAPES) * T if hash_first else 0)   # some batches hold several frames
    assert all(bool(c.hashed) == (hash_first and reqs[c.tag].kind == 0) for c in done)
    assert srv.status() == 0
    check(bufs, vids, dec_in, kb, gamma, n, alone)
    srv.close()


def test_native_trace_replay():
    """vc_server_run_trace: the same requests with staggered arrival times,
    replayed by the library's own loop; completions in request order, every
    frame the oracle's, the same again after a reset."""
    dev = require_gpu()
    from paper_2505_07158_amd.serving import Server
    kb, gamma, n = key_bytes(21), -1.0, 8
    vids, dec_in = workload(dev, kb, gamma, n)
    alone = streams_alone(dev, vids, kb, gamma, n)
    classes = sorted({(w, h) for h, w in ENC_SHAPES + DEC_SHAPES})
    srv = Server(kb, gamma, n, classes, max_streams=8, hbm_budget=1 << 30, max_inflight=1, max_batch=8,
                 scratch_bytes=64 << 20)
    reqs, bufs = requests(dev, vids, dec_in)
    # arrivals: frame t of every stream at 2 ms * t (sorted)
    for r in reqs:
        r.arrival = 0.002 * r.seq
    order = sorted(range(len(reqs)), key=lambda i: (reqs[i].arrival, i))
    trace = [reqs[i] for i in order]
    for k, r in enumerate(trace):
        r.tag = 1000 + k
    # twice: after vc_server_reset every chain and every stream's sequence
    # starts again at frame 0
    for rep in range(2):
        for b in bufs:
            b[4].zero_()
        torch.cuda.synchronize()
        done = srv.run_trace(trace)
        torch.cuda.synchronize()
        for k in range(len(trace)):
            assert done[k].tag == 1000 + k and done[k].done >= done[k].launched >= trace[k].arrival - 1e-9
        assert srv.status() == 0 and srv.idle()
        check([bufs[i] for i in order], vids, dec_in, kb, gamma, n, alone)
        srv.reset()
    srv.close()


def test_server_rejects_bad_requests_before_launching():
    """vc_server's documented errors: a shape that is not one of its classes,
    a stream out of range and a pageable hash buffer are refused at submit
    (VC_EINVAL); a trace whose arrivals are not sorted, or that holds such a
    request anywhere, is refused whole; a reset or a trace replay while
    requests are pending is VC_EBUSY.  None of them launches anything; the
    server then still serves a valid request."""
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    from paper_2505_07158_amd.serving import Server
    kb = key_bytes(22)
    srv = Server(kb, -1.0, 8, [(64, 48)], max_streams=2, hbm_budget=1 << 28, scratch_bytes=64 << 20)
    f = torch.zeros((48, 64, 3), dtype=torch.uint8, device=dev)
    wrong = torch.zeros((40, 64, 3), dtype=torch.uint8, device=dev)
    out = torch.empty_like(f)
    h = torch.zeros(32, dtype=torch.uint8, device=dev)
    pageable = torch.zeros(32, dtype=torch.uint8)
    assert not V.vc_pointer_reachable(pageable)
    for r in (Server.request(0, "enc", 0, 0, wrong, torch.empty_like(wrong), h),   # not a class
              Server.request(1, "enc", 2, 0, f, out, h),                           # stream out of range
              Server.request(2, "enc", 0, 0, f, out, pageable)):                   # hash buffer not reachable
        with pytest.raises(V.VcError) as e:
            srv.submit(r)
        assert e.value.status == V.VC_EINVAL
    a, b = Server.request(3, "enc", 0, 0, f, out, h, arrival=0.5), Server.request(4, "enc", 0, 1, f, out, h)
    with pytest.raises(V.VcError) as e:
        srv.run_trace([a, b])        # arrivals 0.5 then 0.0
    assert e.value.status == V.VC_EINVAL
    # a bad request late in a trace: the whole trace is refused before the
    # valid requests ahead of it are submitted
    good = Server.request(6, "enc", 0, 0, f, out, h)
    bad = Server.request(7, "enc", 0, 1, f, out, pageable, arrival=0.001)
    with pytest.raises(V.VcError) as e:
        srv.run_trace([good, bad])
    assert e.value.status == V.VC_EINVAL
    assert srv.idle() and srv.stats().batches_launched == 0 and srv.stats().pending == 0
    srv.submit(Server.request(5, "enc", 0, 0, f, out, h))
    with pytest.raises(V.VcError) as e:
        srv.reset()                  # one request pending
    assert e.value.status == V.VC_EBUSY
    with pytest.raises(V.VcError) as e:
        srv.run_trace([Server.request(8, "enc", 0, 1, f, out, h)])   # the server is not idle
    assert e.value.status == V.VC_EBUSY
    done = []
    while not srv.idle():
        srv.pump()
        done += srv.poll()
    torch.cuda.synchronize()
    assert [c.tag for c in done] == [5] and done[0].status == 0 and srv.status() == 0
    ref_c, ref_h, _ = oracle.encrypt_stream(oracle.key_from_bytes(kb), -1.0, 8, [to_np(f)])
    assert np.array_equal(to_np(out), ref_c[0]) and to_np(h).tobytes() == ref_h[0]
    srv.close()
