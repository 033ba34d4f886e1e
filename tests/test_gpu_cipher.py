"""End-to-end GPU parity of encrypt_frames / decrypt_frames against the
oracle on the small workloads (one 64x64 frame for several worker counts;
a 24-frame 640x480 video), the differential test of Sec. IV-B on the GPU
path, multi-stream batches (each stream's bytes equal the stream run alone),
chunked scratch, chain-state export/import, the documented errors, and a
seeded sweep of random shapes, keys, worker counts and gamma."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import require_gpu, to_dev, to_np
from metrics import npcr_critical, npcr_mean_sigma, npcr_uaci, uaci_interval, uaci_mean_sigma
from workload.synth import SynthVideo, config1_frame, config2_video, key_bytes, random_frame

pytestmark = pytest.mark.gpu


def V():
    from paper_2505_07158_amd import vcipher
    return vcipher


def oracle_stream(kb, gamma, n, frames):
    return oracle.encrypt_stream(oracle.key_from_bytes(kb), gamma, n, frames)


@pytest.mark.parametrize("n", [1, 6, 32, 64, 256])
def test_config1_parity(n):
    dev = require_gpu()
    kb = key_bytes(0)
    P = config1_frame()
    c = V().Cipher.from_bytes(kb, -1.0, n)
    C, H = c.encrypt(to_dev(P, dev)[None])
    Cs, Hs, _ = oracle_stream(kb, -1.0, n, [P])
    assert to_np(H)[0].tobytes() == Hs[0]
    assert np.array_equal(to_np(C)[0], Cs[0])
    d = V().Cipher.from_bytes(kb, -1.0, n)
    Q = d.decrypt(C, H)
    assert np.array_equal(to_np(Q)[0], P)
    assert c.status() == 0 and d.status() == 0
    c.close(); d.close()


def test_config2_video_parity_and_roundtrip():
    dev = require_gpu()
    kb = key_bytes(0)
    video = config2_video()
    frames = video.frames(24)
    c = V().Cipher.from_bytes(kb, -1.0, 32)
    C, H = c.encrypt(to_dev(frames, dev))
    Cs, Hs, end = oracle_stream(kb, -1.0, 32, list(frames))
    Cn, Hn = to_np(C), to_np(H)
    for t in range(24):
        assert Hn[t].tobytes() == Hs[t], t
        assert np.array_equal(Cn[t], Cs[t]), t
    st, _ = c.get_state(0)
    assert np.array_equal(np.array(st).view(np.uint64), end.view(np.uint64))
    d = V().Cipher.from_bytes(kb, -1.0, 32)
    Q = d.decrypt(C, H)
    assert np.array_equal(to_np(Q), frames)
    c.close(); d.close()


@pytest.mark.parametrize("change", ["increment", "bit_flip"])
def test_config2_differential_npcr_uaci(change):
    """Sec. IV-B on the GPU path: frames 0-7 of the 640x480 video each get
    one random pixel-channel change -- an increment by 1..255 (the paper's
    experiment) or a single flipped bit; per channel the NPCR / UACI against
    the unmodified encryption stay within five standard deviations of the
    ideal-cipher means (99.6094 % and 33.4635 %), and their averages pass
    the alpha = 0.05 tests."""
    dev = require_gpu()
    kb = key_bytes(0)
    frames = config2_video().frames(8)
    rng = np.random.default_rng(2)
    h, w = 480, 640
    M = h * w
    mu_n, s_n = npcr_mean_sigma(M)
    mu_u, s_u = uaci_mean_sigma(M)
    npcrs, uacis = [], []
    for t in range(8):
        g = frames[t].copy()
        i, j, ch = rng.integers(0, h), rng.integers(0, w), rng.integers(0, 3)
        if change == "increment":
            g[i, j, ch] = (int(g[i, j, ch]) + int(rng.integers(1, 256))) % 256
        else:
            g[i, j, ch] ^= np.uint8(1 << int(rng.integers(0, 8)))
        a = V().Cipher.from_bytes(kb, -1.0, 32)
        b = V().Cipher.from_bytes(kb, -1.0, 32)
        Ca, _ = a.encrypt(to_dev(frames[t], dev)[None])
        Cb, _ = b.encrypt(to_dev(g, dev)[None])
        npcr, uaci = npcr_uaci(to_np(Ca)[0], to_np(Cb)[0])
        assert np.all(np.abs(npcr - mu_n) < 5 * s_n), npcr
        assert np.all(np.abs(uaci - mu_u) < 5 * s_u), uaci
        npcrs.append(npcr); uacis.append(uaci)
        a.close(); b.close()
    lo, hi = uaci_interval(M)
    assert np.mean(npcrs) > npcr_critical(M)
    assert lo < np.mean(uacis) < hi


def test_modified_frame_changes_later_frames():
    dev = require_gpu()
    kb = key_bytes(1)
    frames = SynthVideo(160, 120, seed=9).frames(3)
    g = frames.copy()
    g[0, 5, 5, 0] ^= 1
    a = V().Cipher.from_bytes(kb, -1.0, 6)
    b = V().Cipher.from_bytes(kb, -1.0, 6)
    Ca, Ha = a.encrypt(to_dev(frames, dev))
    Cb, Hb = b.encrypt(to_dev(g, dev))
    Ha, Hb = to_np(Ha), to_np(Hb)
    assert Ha[0].tobytes() != Hb[0].tobytes()
    assert Ha[1].tobytes() == Hb[1].tobytes() and Ha[2].tobytes() == Hb[2].tobytes()
    for t in range(3):
        npcr, _ = npcr_uaci(to_np(Ca)[t], to_np(Cb)[t])
        assert np.all(npcr > 99.0), (t, npcr)


def test_multistream_mixed_batch_equals_streams_alone():
    dev = require_gpu()
    kb = key_bytes(3)
    shapes = {0: (48, 64), 1: (30, 42), 2: (48, 64), 3: (17, 23)}
    vids = {s: SynthVideo(w, h, seed=50 + s).frames(4) for s, (h, w) in shapes.items()}
    # interleaved order: frame t of every stream, streams rotating
    order = [(s, t) for t in range(4) for s in (2, 0, 3, 1)]
    mixed = V().Cipher.from_bytes(kb, -1.0, 6, max_streams=4)
    ins = [to_dev(vids[s][t], dev) for s, t in order]
    outs, H = mixed.encrypt(ins, streams=[s for s, _ in order])
    outs = [to_np(o) for o in outs]
    Hn = to_np(H)
    for s in shapes:
        alone = V().Cipher.from_bytes(kb, -1.0, 6)
        Ca, Hal = alone.encrypt(to_dev(vids[s], dev))
        Ca, Hal = to_np(Ca), to_np(Hal)
        Cs, Hs, _ = oracle_stream(kb, -1.0, 6, list(vids[s]))
        for t in range(4):
            k = order.index((s, t))
            assert np.array_equal(outs[k], Ca[t]) and np.array_equal(outs[k], Cs[t]), (s, t)
            assert Hn[k].tobytes() == Hal[t].tobytes() == Hs[t]
        alone.close()
    # and decrypt the mixed batch in the same order
    dec = V().Cipher.from_bytes(kb, -1.0, 6, max_streams=4)
    Cin = [to_dev(o, dev) for o in outs]
    P = dec.decrypt(Cin, H, streams=[s for s, _ in order])
    for (s, t), p in zip(order, P):
        assert np.array_equal(to_np(p), vids[s][t])
    mixed.close(); dec.close()


def test_more_issue_bound_waves_than_simds():
    """3,000 small frames of 12 interleaved streams at n = 32 in one call: the
    SHA-256 launch then holds 3,000 waves and every keygen part about 2,000,
    each wave claiming more than half of a SIMD's registers, against 1,024
    SIMDs, so most workgroups wait for a free SIMD.  Every stream must still
    equal the oracle, and the batch must decrypt back."""
    dev = require_gpu()
    kb = key_bytes(12)
    S, T, n = 12, 250, 32
    vids = {s: [random_frame(16, 24, seed=100000 + 1000 * s + t) for t in range(T)] for s in range(S)}
    order = [(s, t) for t in range(T) for s in range(S)]
    enc = V().Cipher.from_bytes(kb, -1.0, n, max_streams=S)
    outs, H = enc.encrypt([to_dev(vids[s][t], dev) for s, t in order], streams=[s for s, _ in order])
    outs = [to_np(o) for o in outs]
    Hn = to_np(H)
    assert enc.status() == 0
    for s in range(S):
        Cs, Hs, _ = oracle_stream(kb, -1.0, n, vids[s])
        for t in range(T):
            k = t * S + s  # position of (s, t) in order
            assert np.array_equal(outs[k], Cs[t]), (s, t)
            assert Hn[k].tobytes() == Hs[t], (s, t)
    dec = V().Cipher.from_bytes(kb, -1.0, n, max_streams=S)
    P = dec.decrypt([to_dev(o, dev) for o in outs], H, streams=[s for s, _ in order])
    for (s, t), p in zip(order, P):
        assert np.array_equal(to_np(p), vids[s][t]), (s, t)
    assert dec.status() == 0
    enc.close(); dec.close()


def test_small_scratch_processes_in_chunks():
    dev = require_gpu()
    kb = key_bytes(4)
    frames = SynthVideo(128, 96, seed=4).frames(7)
    # two slots of one frame each: every frame is a span of its own
    small = V().Cipher.from_bytes(kb, -1.0, 32, scratch_bytes=2 * (V().vc_scratch_per_frame(128, 96, 32) + 4096))
    big = V().Cipher.from_bytes(kb, -1.0, 32)
    C1, H1 = small.encrypt(to_dev(frames, dev))
    C2, H2 = big.encrypt(to_dev(frames, dev))
    assert torch.equal(C1, C2) and torch.equal(H1, H2)
    small.close(); big.close()


@pytest.mark.parametrize("parts,side,slots", [(1, 0, 1), (4, 2, 2), (3, 1, 3), (7, 4, 2), (64, 3, 4), (2, 0, 2),
                                               (8, 8, 1), (1, 2, 2), (1, 3, 3), (2, 3, 2)])
def test_overlap_settings_match_oracle(parts, side, slots):
    """Parts on side streams, chains on the context's chain stream and
    scratch slots never change bytes: 13 frames of one stream against the
    oracle (default scratch, and a scratch whose slots hold one or two frames,
    so spans reuse slots inside one call), then two streams interleaved in
    one call."""
    dev = require_gpu()
    kb = key_bytes(12)
    n = 6
    video = SynthVideo(96, 64, seed=12).frames(13)
    Cs, Hs, _ = oracle_stream(kb, -1.0, n, list(video))
    per_frame = V().vc_scratch_per_frame(96, 64, n)
    for scratch in (0, slots * (per_frame + per_frame // 2), slots * 2 * per_frame):
        c = V().Cipher.from_bytes(kb, -1.0, n, scratch_bytes=scratch)
        c.overlap(parts, side, slots)
        C, H = c.encrypt(to_dev(video, dev))
        Cn, Hn = to_np(C), to_np(H)
        for t in range(len(video)):
            assert Hn[t].tobytes() == Hs[t], (scratch, t)
            assert np.array_equal(Cn[t], Cs[t]), (scratch, t)
        d = V().Cipher.from_bytes(kb, -1.0, n, scratch_bytes=scratch)
        d.overlap(parts, side, slots)
        assert torch.equal(d.decrypt(C, H), to_dev(video, dev))
        assert c.status() == 0 and d.status() == 0
        c.close(); d.close()
    other = SynthVideo(96, 64, seed=13).frames(5)
    Co, Ho, _ = oracle_stream(kb, -1.0, n, list(other))
    m = V().Cipher.from_bytes(kb, -1.0, n, max_streams=2)
    m.overlap(parts, side, slots)
    frames = [video[0], other[0], video[1], other[1], other[2], video[2]]
    streams = [0, 1, 0, 1, 1, 0]
    seqs = [0, 0, 1, 1, 2, 2]
    C, H = m.encrypt(torch.stack([to_dev(f, dev) for f in frames]), streams=streams)
    Cn = to_np(C)
    for k, (st, sq) in enumerate(zip(streams, seqs)):
        ref = Cs[sq] if st == 0 else Co[sq]
        assert np.array_equal(Cn[k], ref), k
    m.close()
    # one call per frame: consecutive calls start on consecutive side streams
    c = V().Cipher.from_bytes(kb, -1.0, n)
    c.overlap(parts, side, slots)
    outs = [c.encrypt(to_dev(video[t:t + 1], dev)) for t in range(len(video))]
    for t, (C1, H1) in enumerate(outs):
        assert to_np(H1)[0].tobytes() == Hs[t], t
        assert np.array_equal(to_np(C1)[0], Cs[t]), t
    assert c.status() == 0
    c.close()


@pytest.mark.parametrize("slots", [1, 2, 3])
def test_calls_on_alternating_streams_match_oracle(slots):
    """Consecutive calls of one context on different caller streams: the
    library orders the chain and the scratch reuse itself.  Batches of 3
    frames alternate between two streams (with a scratch of one batch per
    slot, so every call reuses a slot another stream's call wrote), then the
    receiver decrypts on two other streams."""
    dev = require_gpu()
    kb = key_bytes(14)
    n = 5
    video = SynthVideo(80, 48, seed=14).frames(15)
    Cs, Hs, _ = oracle_stream(kb, -1.0, n, list(video))
    per = 3 * V().vc_scratch_per_frame(80, 48, n) + 4096  # one batch of 3 frames per slot
    src = to_dev(video, dev)
    enc = V().Cipher.from_bytes(kb, -1.0, n, scratch_bytes=per * slots)
    dec = V().Cipher.from_bytes(kb, -1.0, n, scratch_bytes=per * slots)
    enc.overlap(2, 2, slots)
    dec.overlap(3, 1, slots)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    C = torch.empty_like(src)
    H = torch.empty((len(video), 32), dtype=torch.uint8, device=dev)
    Q = torch.empty_like(src)
    torch.cuda.synchronize()
    done = []
    for k in range(5):
        st = sa if k % 2 == 0 else sb
        enc.encrypt(src[3 * k:3 * k + 3], out=C[3 * k:3 * k + 3], hashes=H[3 * k:3 * k + 3], stream=st)
        ev = torch.cuda.Event()
        ev.record(st)
        done.append(ev)
    da, db = torch.cuda.Stream(), torch.cuda.Stream()
    for k in range(5):
        st = da if k % 2 == 0 else db
        st.wait_event(done[k])
        dec.decrypt(C[3 * k:3 * k + 3], H[3 * k:3 * k + 3], out=Q[3 * k:3 * k + 3], stream=st)
    torch.cuda.synchronize()
    Cn, Hn = to_np(C), to_np(H)
    for t in range(len(video)):
        assert Hn[t].tobytes() == Hs[t], t
        assert np.array_equal(Cn[t], Cs[t]), t
    assert torch.equal(Q, src)
    assert enc.status() == 0 and dec.status() == 0
    enc.close(); dec.close()


def test_overlap_rejects_bad_arguments():
    require_gpu()
    c = V().Cipher.from_bytes(key_bytes(1), -1.0, 4)
    for parts, side, slots in [(0, 2, 2), (65, 2, 2), (4, 9, 2), (4, 2, 0), (4, 2, 5)]:
        with pytest.raises(V().VcError):
            c.overlap(parts, side, slots)
    c.close()


def test_state_export_import_resumes_stream():
    dev = require_gpu()
    kb = key_bytes(5)
    frames = SynthVideo(64, 48, seed=5).frames(4)
    a = V().Cipher.from_bytes(kb, -1.0, 8)
    Ca, Ha = a.encrypt(to_dev(frames, dev))
    b = V().Cipher.from_bytes(kb, -1.0, 8)
    b.encrypt(to_dev(frames[:2], dev))
    st, nxt = b.get_state(0)
    assert nxt == 2
    c = V().Cipher.from_bytes(kb, -1.0, 8)
    c.set_state(0, st, 2)
    Cc, Hc = c.encrypt(to_dev(frames[2:], dev))
    assert torch.equal(Cc, Ca[2:]) and torch.equal(Hc, Ha[2:])
    c.reset(0)
    Cr, _ = c.encrypt(to_dev(frames[:1], dev))
    assert torch.equal(Cr, Ca[:1])
    a.close(); b.close(); c.close()


def test_documented_errors():
    dev = require_gpu()
    Vm = V()
    c = Vm.Cipher.from_bytes(key_bytes(6), -1.0, 8, max_streams=2)
    f = to_dev(random_frame(16, 16, 1), dev)
    out = torch.empty_like(f)
    H = torch.empty((1, 32), dtype=torch.uint8, device=dev)
    # out of sequence
    with pytest.raises(Vm.VcError) as e:
        Vm.encrypt_frames(c.ctx, [f], [0], [1], H, [out])
    assert e.value.status == Vm.VC_EORDER
    # in-place encryption (the gather cannot run in place)
    with pytest.raises(Vm.VcError) as e:
        Vm.encrypt_frames(c.ctx, [f], [0], [0], H, [f])
    assert e.value.status == Vm.VC_EINVAL
    # stream id out of range
    with pytest.raises(Vm.VcError) as e:
        Vm.encrypt_frames(c.ctx, [f], [2], [0], H, [out])
    assert e.value.status == Vm.VC_EINVAL
    # n larger than the frame
    tiny = Vm.Cipher.from_bytes(key_bytes(6), -1.0, 8)
    t = torch.zeros((1, 2, 3), dtype=torch.uint8, device=dev)
    with pytest.raises(Vm.VcError) as e:
        Vm.encrypt_frames(tiny.ctx, [t], [0], [0], H, [torch.empty_like(t)])
    assert e.value.status == Vm.VC_EINVAL
    # a shape whose channel count is not 3 (the binding always sends 3: raw call)
    import ctypes as C
    sh = (Vm.VcShape * 1)(Vm.VcShape(16, 16, 2, 0, 0))
    rc = Vm.lib.encrypt_frames(C.c_void_p(c.ctx), 1, Vm._ptrs([f]), sh, C.c_void_p(H.data_ptr()), Vm._ptrs([out]),
                               None)
    assert rc == Vm.VC_EINVAL
    # empty calls (count 0, NULL arrays) succeed and enqueue nothing
    L, ctx = Vm.lib, C.c_void_p(c.ctx)
    for rc in (L.encrypt_frames(ctx, 0, None, None, None, None, None),
               L.encrypt_frames_noalloc(ctx, 0, None, None, None, None, None),
               L.encrypt_frames_hashed(ctx, 0, None, None, None, None, None),
               L.decrypt_frames(ctx, 0, None, None, None, None, None),
               L.vc_hash_frames(ctx, 0, None, None, None, None)):
        assert rc == Vm.VC_OK
    # neither the failed nor the empty calls moved the chain: the stream
    # still starts at seq 0 with the key, as in the oracle
    Vm.encrypt_frames(c.ctx, [f], [0], [0], H, [out])
    assert c.status() == 0
    Cs, Hs, _ = oracle_stream(key_bytes(6), -1.0, 8, [to_np(f)])
    assert to_np(H)[0].tobytes() == Hs[0] and np.array_equal(to_np(out), Cs[0])
    c.close(); tiny.close()


@pytest.mark.slow
@pytest.mark.parametrize("w,h,n,frames", [(3840, 2160, 32, 2), (1920, 1080, 256, 2), (1280, 720, 6, 3),
                                          (720, 480, 32, 2), (1924, 1084, 32, 2)])
def test_large_shapes_parity(w, h, n, frames):
    """Largest frame of the serving mix (3840x2160), the second worker
    count of the benchmark plan (n = 256), the paper's monitoring setting
    (n = 6), SD, and a frame whose width is not a multiple of the strip."""
    dev = require_gpu()
    kb = key_bytes(7)
    video = SynthVideo(w, h, seed=w + h + n).frames(frames)
    c = V().Cipher.from_bytes(kb, -1.0, n)
    C, H = c.encrypt(to_dev(video, dev))
    Cs, Hs, _ = oracle_stream(kb, -1.0, n, list(video))
    Cn, Hn = to_np(C), to_np(H)
    for t in range(frames):
        assert Hn[t].tobytes() == Hs[t], t
        assert np.array_equal(Cn[t], Cs[t]), t
    d = V().Cipher.from_bytes(kb, -1.0, n)
    assert torch.equal(d.decrypt(C, H), to_dev(video, dev))
    c.close(); d.close()


@pytest.mark.parametrize("passes", [2, 1])
def test_extreme_shapes(passes):
    """The tallest frame the context accepts (a strip of 4 bytes per row,
    two-pass, or of 4 pixels, single pass, fills the LDS) against the oracle,
    one row more rejected, and a single row 65535 pixels wide (the row pass
    then reads global memory)."""
    dev = require_gpu()
    Vm = V()
    kb, n = key_bytes(9), 8
    c = Vm.Cipher.from_bytes(kb, -1.0, n, max_streams=3)
    c.passes(passes)
    hmax = Vm.vc_max_frame_height(c.ctx)
    assert 1000 < hmax < 65535
    for s, (h, w) in enumerate([(hmax, 4), (1, 65535), (hmax, 5)]):
        f = random_frame(h, w, 90 + s)
        C, H = c.encrypt(to_dev(f[None], dev), streams=[s])
        Cs, Hs, _ = oracle_stream(kb, -1.0, n, [f])
        assert to_np(H)[0].tobytes() == Hs[0], (h, w)
        assert np.array_equal(to_np(C)[0], Cs[0]), (h, w)
        d = Vm.Cipher.from_bytes(kb, -1.0, n, max_streams=3)
        d.passes(passes)
        d._next[s] = 0
        assert torch.equal(d.decrypt(C, H, streams=[s]), to_dev(f[None], dev)), (h, w)
        d.close()
    t = torch.zeros((hmax + 1, 4, 3), dtype=torch.uint8, device=dev)
    with pytest.raises(Vm.VcError) as e:
        c.encrypt(t[None], streams=[0])
    assert e.value.status == Vm.VC_EINVAL
    c.close()


def test_batch_shapes_xcd_split_and_ragged():
    """Batches whose frame count is not a multiple of the 8 XCDs, frames of
    two shapes in one call, and a ragged last strip (w = 100), checked
    against the oracle confusion with oracle-generated D and B."""
    dev = require_gpu()
    rng = np.random.default_rng(99)
    c = V().Cipher.from_bytes(key_bytes(8), -1.0, 4)
    for shapes in ([(48, 100)] * 3, [(64, 64)] * 9 + [(33, 100)] * 2, [(120, 160)] * 17):
        Ps = [rng.integers(0, 256, (h, w, 3), dtype=np.uint8) for h, w in shapes]
        Ds = [rng.integers(0, 65536, 3 * h + 3 * w, dtype=np.uint16) for h, w in shapes]
        Bs = [rng.integers(0, 256, (h, w, 3), dtype=np.uint8) for h, w in shapes]
        outs = c.confuse([to_dev(p, dev) for p in Ps], [to_dev(x, dev) for x in Ds], [to_dev(x, dev) for x in Bs])
        for P, D, B, o in zip(Ps, Ds, Bs, outs):
            ref = oracle.confuse_enc(P, D, B)
            assert np.array_equal(to_np(o), ref)
        back = c.confuse(outs, [to_dev(x, dev) for x in Ds], [to_dev(x, dev) for x in Bs], decrypt=True)
        for P, b in zip(Ps, back):
            assert np.array_equal(to_np(b), P)
    c.close()


def test_encrypt_with_precomputed_hashes_matches():
    dev = require_gpu()
    kb = key_bytes(9)
    frames = to_dev(SynthVideo(96, 64, seed=9).frames(5), dev)
    a = V().Cipher.from_bytes(kb, -1.0, 6)
    b = V().Cipher.from_bytes(kb, -1.0, 6)
    Ca, Ha = a.encrypt(frames)
    hs = torch.cuda.Stream()
    H = b.hash(frames, stream=hs)
    ev = torch.cuda.Event()
    ev.record(hs)
    torch.cuda.current_stream().wait_event(ev)
    Cb = b.encrypt_hashed(frames, H)
    assert torch.equal(H, Ha) and torch.equal(Cb, Ca)
    a.close(); b.close()


def test_hash_buffers_in_pinned_host_memory():
    """Hash buffers may be pinned host memory (hipHostMalloc, torch's
    pin_memory): the kernels write H there when encrypting and read it when
    decrypting.  Pageable host memory is refused by the library before
    anything is enqueued (checked only after vc_pointer_reachable has
    classified it, so no kernel ever sees it)."""
    import ctypes as C
    dev = require_gpu()
    Vm = V()
    kb = key_bytes(7)
    video = SynthVideo(64, 48, seed=2300).frames(4)
    frames = to_dev(video, dev)
    pinned = torch.zeros((4, 32), dtype=torch.uint8, pin_memory=True)
    pageable = torch.zeros((4, 32), dtype=torch.uint8)
    on_dev = torch.zeros((4, 32), dtype=torch.uint8, device=dev)
    assert Vm.vc_pointer_reachable(pinned) and Vm.vc_pointer_reachable(on_dev) and Vm.vc_pointer_reachable(frames)
    assert not Vm.vc_pointer_reachable(pageable)
    c = Vm.Cipher.from_bytes(kb, -1.0, 8)
    fr = list(frames)
    out = torch.empty_like(frames)
    rc = Vm.lib.encrypt_frames(C.c_void_p(c.ctx), 4, Vm._ptrs(fr), Vm._shapes(fr, [0] * 4, [0, 1, 2, 3]),
                               C.c_void_p(pageable.data_ptr()), Vm._ptrs(list(out)), None)
    assert rc == Vm.VC_EINVAL
    C1, H1 = c.encrypt(frames, hashes=pinned)
    torch.cuda.synchronize()
    Cs, Hs, _ = oracle_stream(kb, -1.0, 8, list(video))
    for t in range(4):
        assert pinned[t].numpy().tobytes() == Hs[t], t
        assert np.array_equal(to_np(C1[t]), Cs[t]), t
    d = Vm.Cipher.from_bytes(kb, -1.0, 8)
    Q = d.decrypt(C1, pinned)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(Q), video)
    assert c.status() == 0 and d.status() == 0
    c.close(); d.close()


def test_random_shapes_keys_and_worker_counts():
    """A seeded sweep of small frames: random shapes (1..160 x 1..120),
    random keys, gamma across its range, worker counts from 1 to 1024 (up
    to the frame's byte count, n = 3wh included) and both confusion forms.
    Two frames of one stream equal the oracle's (hashes and ciphertext) and
    decrypt back to the plaintext."""
    dev = require_gpu()
    Vm = V()
    rng = np.random.default_rng(77)
    for case in range(24):
        w, h = int(rng.integers(1, 161)), int(rng.integers(1, 121))
        nmax = min(3 * w * h, 1024)
        n = [1, nmax, int(rng.integers(1, nmax + 1)), int(rng.integers(1, min(nmax, 64) + 1))][case % 4]
        gamma = float(rng.uniform(-1.52, -0.06))
        passes = 2 if case % 3 else 1
        kb = bytes(rng.integers(0, 256, 32, dtype=np.uint8).tolist())
        frames = rng.integers(0, 256, (2, h, w, 3), dtype=np.uint8)
        what = (case, w, h, n, round(gamma, 3), passes)
        c = Vm.Cipher.from_bytes(kb, gamma, n, scratch_bytes=64 << 20)
        d = Vm.Cipher.from_bytes(kb, gamma, n, scratch_bytes=64 << 20)
        c.passes(passes)
        d.passes(passes)
        C, H = c.encrypt(to_dev(frames, dev))
        Cs, Hs, _ = oracle_stream(kb, gamma, n, list(frames))
        Cn, Hn = to_np(C), to_np(H)
        for t in range(2):
            assert Hn[t].tobytes() == Hs[t], what + (t,)
            assert np.array_equal(Cn[t], Cs[t]), what + (t,)
        assert torch.equal(d.decrypt(C, H), to_dev(frames, dev)), what
        assert c.status() == 0 and d.status() == 0, what
        c.close(); d.close()
