"""Pins of the oracle's SHA-256 and frame hash (Sec. II-A) against
independent implementations: Python's hashlib and the openssl CLI, on the
FIPS 180-4 example messages, every padding boundary, random lengths, and
the sub-frame xor combine."""
import hashlib
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from workload.synth import random_frame

# The example messages of FIPS 180-4 (one-block, two-block, long).  The
# expected digests come from hashlib at run time; nothing is stored.
FIPS_EXAMPLE_MESSAGES = [
    b"abc",
    b"abcdbcdecdefdefgefghfghighijhijkijkljklmklmnlmnomnopnopq",
    b"a" * 1_000_000,
]


@pytest.mark.parametrize("msg", FIPS_EXAMPLE_MESSAGES, ids=["one-block", "two-block", "million-a"])
def test_fips_example_messages(msg):
    assert oracle.sha256(msg) == hashlib.sha256(msg).digest()


def test_every_padding_boundary():
    rng = np.random.default_rng(11)
    for n in range(0, 260):
        m = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        assert oracle.sha256(m) == hashlib.sha256(m).digest(), n


def test_random_lengths():
    rng = np.random.default_rng(12)
    for n in rng.integers(0, 100_000, 40):
        m = rng.integers(0, 256, int(n), dtype=np.uint8).tobytes()
        assert oracle.sha256(m) == hashlib.sha256(m).digest(), n


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI not installed")
def test_against_openssl(tmp_path):
    rng = np.random.default_rng(13)
    for n in (0, 1, 55, 56, 63, 64, 65, 1000, 65537):
        m = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        p = tmp_path / f"m{n}.bin"
        p.write_bytes(m)
        out = subprocess.run(["openssl", "dgst", "-sha256", "-binary", str(p)], capture_output=True, check=True)
        assert oracle.sha256(m) == out.stdout, n


def test_frame_hash_single_subframe_is_sha256():
    f = random_frame(37, 53, seed=3)
    assert oracle.frame_hash(f, 1) == hashlib.sha256(f.tobytes()).digest()


@pytest.mark.parametrize("n", [2, 3, 6, 7, 32, 64, 100, 256])
def test_frame_hash_is_xor_of_subframe_hashes(n):
    f = random_frame(45, 61, seed=n)
    data = f.tobytes()
    L = len(data)
    H = bytearray(32)
    for i in range(n):
        d = hashlib.sha256(data[i * L // n:(i + 1) * L // n]).digest()
        H = bytearray(a ^ b for a, b in zip(H, d))
    assert oracle.frame_hash(f, n) == bytes(H)


def test_frame_hash_one_byte_subframes():
    f = random_frame(2, 3, seed=9)   # L = 18, n = L
    data = f.tobytes()
    H = bytearray(32)
    for b in data:
        H = bytearray(x ^ y for x, y in zip(H, hashlib.sha256(bytes([b])).digest()))
    assert oracle.frame_hash(f, len(data)) == bytes(H)


def test_equal_subframes_cancel():
    # H = h_1 xor h_2 vanishes when the two sub-frames are identical: a
    # property of the combine of Sec. II-A.
    half = random_frame(8, 16, seed=4)
    f = np.concatenate([half, half], axis=0)
    assert oracle.frame_hash(f, 2) == bytes(32)
