"""GPU parity of the confusion + XOR kernels and their inverse (Sec. II-C)
against the oracle, byte for byte, with caller-supplied D and B through the
C-ABI testing entry point (the same kernels encrypt_frames uses), for both
the two-pass (row pass + column pass) and the single-pass form."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from gpu_util import require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 4), (2, 3), (3, 1), (5, 7), (4, 4), (8, 12), (17, 5), (64, 64), (33, 100),
          (100, 33), (480, 640), (481, 643), (720, 1280), (1080, 1920), (2, 2000), (2000, 3),
          (3, 56000),  # a row longer than the LDS: the row pass reads global memory
          # rows of a multiple of 16 pixels (the row pass's planar form): one
          # 16-pixel item per row, two, 2 and 1 rows per workgroup, a last
          # workgroup with fewer rows
          (5, 16), (6, 32), (9, 2048), (7, 3840), (6, 20000)]


def case(rng, h, w):
    P = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    D = rng.integers(0, 65536, 3 * h + 3 * w, dtype=np.uint16)
    B = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    return P, D, B


@pytest.fixture(scope="module", params=[2, 1], ids=["two_pass", "single_pass"])
def ctx(request):
    require_gpu()
    from paper_2505_07158_amd import vcipher as V
    c = V.Cipher(V.vc_key_from_bytes(bytes(range(32)), -1.0, 4))
    c.passes(request.param)
    c.form = request.param
    yield c
    c.close()


@pytest.mark.parametrize("h,w", SHAPES)
def test_enc_dec_parity(ctx, h, w):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(h * 10007 + w)
    P, D, B = case(rng, h, w)
    ref = oracle.confuse_enc(P, D, B)
    (C,) = ctx.confuse([to_dev(P, dev)], [to_dev(D, dev)], [to_dev(B, dev)])
    got = to_np(C)
    assert np.array_equal(got, ref), f"{(h, w)}: {(got != ref).sum()} bytes differ"
    (Q,) = ctx.confuse([to_dev(ref, dev)], [to_dev(D, dev)], [to_dev(B, dev)], decrypt=True)
    assert np.array_equal(to_np(Q), P)


# Strip widths: bytes of a row for the two-pass form's column pass (4-128),
# pixels for the single pass (4-64); a strip that the LDS cannot hold at a
# shape falls back to the automatic choice.  Shapes: ragged strips (52, 68, 30 and
# 100 columns), 16-byte rows (640, 1280, 1920 columns: the column pass's
# 16-byte kernels), and the benchmark's 720p and 1080p frames, where 128-byte
# (two-pass) or 32/64-pixel (single-pass) strips fill most of the LDS.
TILING_SHAPES = [(37, 52), (64, 68), (29, 30), (50, 100), (480, 640), (720, 1280), (1080, 1920)]


@pytest.mark.parametrize("strip,threads", list(itertools.product([4, 8, 16, 32, 64, 128], [256, 512, 1024])))
def test_every_tiling_gives_the_same_bytes(ctx, strip, threads):
    if ctx.form == 1 and strip > 64:
        pytest.skip("single-pass strips are at most 64 pixels")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(strip * 7 + threads)
    for k, (h, w) in enumerate(TILING_SHAPES):
        P, D, B = case(rng, h, w)
        # XCD-local mapping on and off, each for every strip and size
        ctx.tune(strip, threads, xcd_map=(k + strip // 4 + threads // 256) % 2 == 0)
        try:
            (C,) = ctx.confuse([to_dev(P, dev)], [to_dev(D, dev)], [to_dev(B, dev)])
            (Q,) = ctx.confuse([C], [to_dev(D, dev)], [to_dev(B, dev)], decrypt=True)
        finally:
            ctx.tune(0, 0, True)
        assert np.array_equal(to_np(C), oracle.confuse_enc(P, D, B)), (h, w)
        assert np.array_equal(to_np(Q), P), (h, w)


def test_mixed_shapes_and_unaligned_pointers(ctx):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(77)
    shapes = [(48, 64), (17, 23), (48, 64), (5, 8), (30, 42), (48, 64)]
    Ps, Ds, Bs, ins, outs = [], [], [], [], []
    for k, (h, w) in enumerate(shapes):
        P, D, B = case(rng, h, w)
        Ps.append(P); Ds.append(to_dev(D, dev)); Bs.append(to_dev(B, dev))
        if k % 2:   # frame at an odd byte offset inside a larger buffer
            buf = torch.zeros(P.size + 1, dtype=torch.uint8, device=dev)
            t = buf[1:].view(h, w, 3)
            t.copy_(to_dev(P, dev))
            ins.append(t)
        else:
            ins.append(to_dev(P, dev))
        outs.append(torch.empty((h, w, 3), dtype=torch.uint8, device=dev))
    from paper_2505_07158_amd import vcipher as V
    V.vc_debug_confuse(ctx.ctx, False, ins, Ds, Bs, outs)
    for P, D, B, C in zip(Ps, Ds, Bs, outs):
        assert np.array_equal(to_np(C), oracle.confuse_enc(P, to_np(D), to_np(B)))


def test_autotuned_tiling_gives_the_same_bytes(ctx):
    """The autotuner picks a tiling for a shape (timed on its own buffers);
    calls on that shape then use it, with unchanged output."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(4242)
    h, w = 90, 124
    for decrypt in (False, True):
        strip, threads = ctx.autotune(w, h, frames=4, decrypt=decrypt)
        assert strip in ((4, 8, 16, 32, 64, 128) if ctx.form == 2 else (4, 8, 16, 32, 64))
        assert threads in (256, 512, 1024)
    P, D, B = case(rng, h, w)
    (C,) = ctx.confuse([to_dev(P, dev)], [to_dev(D, dev)], [to_dev(B, dev)])
    assert np.array_equal(to_np(C), oracle.confuse_enc(P, D, B))
    (Q,) = ctx.confuse([C], [to_dev(D, dev)], [to_dev(B, dev)], decrypt=True)
    assert np.array_equal(to_np(Q), P)
