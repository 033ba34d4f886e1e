"""Pins of the oracle's bit-level confusion + XOR (Sec. II-C: Eq. 2, Eq. 3,
Algs. 3-7) and its inverse.

* The closed per-byte form against the literal bit-matrix form of Algs. 3-7
  on every shape up to 6 x 6 and a few larger ones.
* Both against an independent formulation built from numpy library
  routines: unpackbits/packbits (least significant bit first) and np.roll
  for the circular shifts of Eqs. 2 and 3.
* The permutation is a bijection of bit positions (exhaustive single-bit
  probes), preserves popcount, and reduces to special cases: zero
  distances give C = P xor B; whole-byte row shifts give a pixel roll.
* decrypt(encrypt(x)) == x, and a flipped ciphertext bit damages exactly
  one plaintext bit (no diffusion, Sec. VI)."""
import itertools

import numpy as np
import pytest

import oracle


def numpy_confuse(P, D, B):
    """Eq. 2 then Eq. 3 on unpacked bit planes, then xor (Algs. 3-7)."""
    h, w, _ = P.shape
    out = np.empty_like(P)
    for c in range(3):
        bits = np.unpackbits(P[:, :, c], axis=1, bitorder="little")          # (h, 8w)
        m1 = np.stack([np.roll(bits[r], int(D[c * h + r]) % (8 * w)) for r in range(h)])
        m2 = np.empty_like(m1)
        for x in range(8 * w):
            dv = int(D[3 * h + c * w + x // 8]) % h
            m2[:, x] = np.roll(m1[:, x], dv)
        bb = np.unpackbits(B[:, :, c], axis=1, bitorder="little")
        out[:, :, c] = np.packbits(m2 ^ bb, axis=1, bitorder="little")
    return out


def rand_case(rng, h, w, zero_b=False):
    P = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    D = rng.integers(0, 65536, 3 * h + 3 * w, dtype=np.uint16)
    B = np.zeros_like(P) if zero_b else rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    return P, D, B


@pytest.mark.parametrize("h,w", list(itertools.product(range(1, 7), range(1, 7))))
def test_literal_equals_closed_small(h, w):
    rng = np.random.default_rng(100 * h + w)
    for _ in range(3):
        P, D, B = rand_case(rng, h, w)
        C = oracle.confuse_enc(P, D, B)
        np.testing.assert_array_equal(C, oracle.confuse_enc_literal(P, D, B))
        np.testing.assert_array_equal(oracle.confuse_dec(C, D, B), P)
        np.testing.assert_array_equal(oracle.confuse_dec_literal(C, D, B), P)


@pytest.mark.parametrize("h,w", [(4, 4), (8, 12), (17, 5), (1, 31), (33, 1), (64, 64), (48, 80)])
def test_numpy_formulation(h, w):
    rng = np.random.default_rng(h * 1000 + w)
    P, D, B = rand_case(rng, h, w)
    C = oracle.confuse_enc(P, D, B)
    np.testing.assert_array_equal(C, numpy_confuse(P, D, B))
    np.testing.assert_array_equal(C, oracle.confuse_enc_literal(P, D, B))


@pytest.mark.parametrize("h,w", [(4, 4), (3, 5), (1, 7), (6, 1)])
def test_single_bit_probes_form_a_bijection(h, w):
    rng = np.random.default_rng(h + 10 * w)
    D = rng.integers(0, 65536, 3 * h + 3 * w, dtype=np.uint16)
    B = np.zeros((h, w, 3), np.uint8)
    hit = set()
    for i, j, c, k in itertools.product(range(h), range(w), range(3), range(8)):
        P = np.zeros((h, w, 3), np.uint8)
        P[i, j, c] = 1 << k
        C = oracle.confuse_enc(P, D, B)
        nz = np.argwhere(C)
        assert len(nz) == 1
        ii, jj, cc = nz[0]
        v = int(C[ii, jj, cc])
        assert v & (v - 1) == 0 and cc == c   # one bit, same channel
        hit.add((ii, jj, cc, v.bit_length() - 1))
    assert len(hit) == h * w * 3 * 8


def test_popcount_preserved_per_channel():
    rng = np.random.default_rng(21)
    P, D, B = rand_case(rng, 23, 19, zero_b=True)
    C = oracle.confuse_enc(P, D, B)
    for c in range(3):
        assert np.unpackbits(P[:, :, c]).sum() == np.unpackbits(C[:, :, c]).sum()


def test_zero_distances_give_plain_xor():
    rng = np.random.default_rng(22)
    h, w = 13, 9
    P, _, B = rand_case(rng, h, w)
    np.testing.assert_array_equal(oracle.confuse_enc(P, np.zeros(3 * h + 3 * w, np.uint16), B), P ^ B)
    # distances that are multiples of the rotation periods act as zero
    D = np.concatenate([np.full(3 * h, 8 * w * 3, np.uint16), np.full(3 * w, h * 4, np.uint16)])
    np.testing.assert_array_equal(oracle.confuse_enc(P, D, B), P ^ B)


def test_whole_byte_row_shift_is_pixel_roll():
    rng = np.random.default_rng(23)
    h, w = 7, 10
    P, _, B = rand_case(rng, h, w)
    m = rng.integers(0, w, 3 * h)
    D = np.concatenate([(8 * m).astype(np.uint16), np.zeros(3 * w, np.uint16)])
    C = oracle.confuse_enc(P, D, B)
    for c in range(3):
        for i in range(h):
            np.testing.assert_array_equal(C[i, :, c], np.roll(P[i, :, c], int(m[c * h + i])) ^ B[i, :, c])


@pytest.mark.parametrize("h,w", [(1, 1), (1, 2), (2, 1), (5, 3), (64, 64), (31, 47), (120, 160)])
def test_roundtrip(h, w):
    rng = np.random.default_rng(h * 7 + w)
    P, D, B = rand_case(rng, h, w)
    np.testing.assert_array_equal(oracle.confuse_dec(oracle.confuse_enc(P, D, B), D, B), P)


def test_ciphertext_bit_error_stays_local():
    rng = np.random.default_rng(24)
    h, w = 32, 24
    P, D, B = rand_case(rng, h, w)
    C = oracle.confuse_enc(P, D, B)
    for _ in range(20):
        i, j, c, k = rng.integers(0, h), rng.integers(0, w), rng.integers(0, 3), rng.integers(0, 8)
        C2 = C.copy()
        C2[i, j, c] ^= np.uint8(1 << k)
        diff = np.unpackbits(oracle.confuse_dec(C2, D, B) ^ P)
        assert diff.sum() == 1
