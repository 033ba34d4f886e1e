"""Full-size parity: the benchmark's workload (1920x1080x3, 300 frames, one
stream, n = 32) in the benchmark's launch configuration (one encrypt_frames
call for all frames, one decrypt_frames call).  Every frame hash is checked
against the oracle, sampled frames (first, second, middle, last two) are
checked byte for byte through the oracle's chain, and decrypt(encrypt(x))
== x on all 300 frames."""
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
    enc = V.Cipher.from_bytes(kb, gamma, n, scratch_bytes=2 * V.vc_scratch_per_frame(1920, 1080, n) * T)
    dec = V.Cipher.from_bytes(kb, gamma, n, scratch_bytes=2 * V.vc_scratch_per_frame(1920, 1080, n) * T)
    C, H = enc.encrypt(frames)
    P = dec.decrypt(C, H)
    torch.cuda.synchronize()
    assert torch.equal(P, frames)
    assert enc.status() == 0 and dec.status() == 0
    Hn = to_np(H)
    with cf.ThreadPoolExecutor(8) as ex:
        ref_h = list(ex.map(lambda t: oracle.frame_hash(host[t], n), range(T)))
    for t in range(T):
        assert Hn[t].tobytes() == ref_h[t], t
    bases = oracle.chain_states(oracle.key_from_bytes(kb), gamma, n, ref_h)
    for t in (0, 1, T // 2, T - 2, T - 1):
        ref_c, ref_hh, nxt = oracle.encrypt_frame(bases[t], gamma, n, host[t])
        assert ref_hh == ref_h[t]
        assert np.array_equal(to_np(C[t]), ref_c), t
        np.testing.assert_array_equal(nxt, bases[t + 1])
    st, nxt = enc.get_state(0)
    assert np.array_equal(np.array(st).view(np.uint64), bases[T].view(np.uint64)) and nxt == T
