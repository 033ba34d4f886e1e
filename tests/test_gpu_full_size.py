"""Full-size parity: the benchmark's workload (1920x1080x3, 300 frames, one
stream, n = 32) in the benchmark's launch configuration: the frame hashes
by vc_hash_frames on one stream, encrypt_frames_hashed on another (3 parts
on 3 side streams, 4 scratch slots of one batch each, two-pass confusion),
decrypt_frames on a receiver context; then the same batch once more through
encrypt_frames in one call.  Every frame hash and every ciphertext frame
is checked against the oracle (frames in parallel on the host, each from
the chain state the oracle's chain gives it), and decrypt(encrypt(x)) == x
on all 300 frames."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
from gpu_util import require_gpu, to_np
from workload.synth import SynthVideo, config_seed, key_bytes

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_config3_full_size():
    dev = require_gpu()
    from paper_2505_07158_amd import vcipher as V
    w, h, T, n, gamma = 1920, 1080, 300, 32, -1.0
    kb = key_bytes(0)
    host = SynthVideo(w, h, seed=config_seed(3), pan=(3.0, 1.0)).frames(T)
    frames = torch.from_numpy(host).to(dev)
    batch_scratch = V.vc_scratch_per_frame(1920, 1080, n) * T + (64 << 20)
    enc = V.Cipher.from_bytes(kb, gamma, n, scratch_bytes=4 * batch_scratch)
    dec = V.Cipher.from_bytes(kb, gamma, n, scratch_bytes=4 * batch_scratch)
    for c in (enc, dec):
        c.overlap(3, 3, 4)
        c.passes(2)
    s_hash, s_enc, s_dec = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    H = torch.empty((T, 32), dtype=torch.uint8, device=dev)
    C = torch.empty_like(frames)
    P = torch.empty_like(frames)
    hashed, ready = torch.cuda.Event(), torch.cuda.Event()
    torch.cuda.synchronize()
    enc.hash(frames, stream=s_hash, out=H)
    hashed.record(s_hash)
    s_enc.wait_event(hashed)
    enc.encrypt_hashed(frames, H, out=C, stream=s_enc)
    ready.record(s_enc)
    s_dec.wait_event(ready)
    dec.decrypt(C, H, out=P, stream=s_dec)
    torch.cuda.synchronize()
    assert torch.equal(P, frames)
    assert enc.status() == 0 and dec.status() == 0
    # a fresh context's single encrypt_frames call over the batch gives the
    # same bytes
    one = V.Cipher.from_bytes(kb, gamma, n, scratch_bytes=2 * batch_scratch)
    C1, H1 = one.encrypt(frames)
    torch.cuda.synchronize()
    assert torch.equal(C1, C) and torch.equal(H1, H)
    one.close()
    Hn = to_np(H)
    with cf.ThreadPoolExecutor(8) as ex:
        ref_h = list(ex.map(lambda t: oracle.frame_hash(host[t], n), range(T)))
    for t in range(T):
        assert Hn[t].tobytes() == ref_h[t], t
    bases = oracle.chain_states(oracle.key_from_bytes(kb), gamma, n, ref_h)
    Cn = to_np(C)

    def check(t):
        ref_c, ref_hh, nxt = oracle.encrypt_frame(bases[t], gamma, n, host[t])
        return ref_hh == ref_h[t] and np.array_equal(Cn[t], ref_c) and np.array_equal(nxt, bases[t + 1])

    with cf.ThreadPoolExecutor(16) as ex:
        ok = list(ex.map(check, range(T)))
    bad = [t for t in range(T) if not ok[t]]
    assert not bad, bad
    st, nxt = enc.get_state(0)
    assert np.array_equal(np.array(st).view(np.uint64), bases[T].view(np.uint64)) and nxt == T
