"""The oracle's key schedule and whole-frame path against a second,
independent implementation (tests/pyref.py: plain Python floats and
integers, hashlib, numpy bit arrays) of the same protocol-v1 readings.

The paper prints no worked example of the reconstruction (Sec. II-A), the
worker seeding and byte stream (Sec. II-B, Alg. 2) or the D/B partition, so
no value here comes from the paper; what pins the oracle is that two
implementations written separately, in different languages and arithmetic
(C doubles and uint64 vs Python floats and big integers), agree bit for bit
on every double, distance and byte.  The mutation tests show that the check
has teeth: a copy of the oracle with one plausible mistake planted in it (a
transposed seeding component, a reversed byte order, a swapped distance
byte order, a shifted partition, a hash-byte order flip) is built and must
disagree with the Python implementation."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
import pyref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SRC = os.path.join(ROOT, "oracle", "vc_oracle.c")


def u64(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


# ---- reconstruction (R5) ----------------------------------------------------------

def test_reconstruct_bit_for_bit():
    rng = np.random.default_rng(101)
    bases = [rng.uniform(-40, 40, 4), rng.uniform(-1, 1, 4), rng.uniform(-400, 400, 4),
             np.array([0.0, -0.0, 31.999999999, 65536.5]), np.array([1e6 + 0.25, -7.0, 2.0 ** -30, 123456.789])]
    bases += [rng.uniform(-60, 60, 4) for _ in range(300)]
    for b in bases:
        H = rng.bytes(32)
        assert np.array_equal(u64(oracle.reconstruct(b, H)), u64(pyref.reconstruct(b, H))), (b, H.hex())


# ---- worker seeding and byte stream (R6, R7) -----------------------------------------

@pytest.mark.parametrize("n", [1, 2, 6, 32])
def test_worker_streams_bit_for_bit(n):
    rng = np.random.default_rng(200 + n)
    IR = rng.uniform(-20, 20, (2 * n, 4))
    for i in range(n):
        nbytes = 24 * 7 + 5      # a partial last step
        assert oracle.worker_stream(IR, -1.0, i, nbytes).tobytes() == pyref.worker_stream(IR.tolist(), -1.0, i, nbytes), (n, i)


def test_worker_stream_from_a_real_chain():
    # IR from the LHCS_m chain itself (both sides compute it), gamma at both ends
    kb = bytes(range(32))
    for gamma in (-1.52, -0.06):
        base = oracle.key_from_bytes(kb)
        H = bytes(range(100, 132))
        ic = oracle.reconstruct(base, H)
        IR = oracle.chain(ic, gamma, 6)
        IRp = pyref.chain(pyref.reconstruct(base, H), gamma, 6)
        assert np.array_equal(u64(IR), u64(IRp))
        for i in range(6):
            assert oracle.worker_stream(IR, gamma, i, 480).tobytes() == pyref.worker_stream(IRp, gamma, i, 480)


# ---- partition of D and B (R8, R9) ----------------------------------------------------
# shapes where ND = 3(h + w) or L = 3wh is not a multiple of n

@pytest.mark.parametrize("n,h,w", [(1, 5, 7), (2, 5, 7), (2, 6, 7), (6, 5, 7), (6, 7, 10), (32, 9, 13), (32, 3, 4)])
def test_keystream_partition_bit_for_bit(n, h, w):
    rng = np.random.default_rng(n * 100 + h * 10 + w)
    IR = rng.uniform(-20, 20, (2 * n, 4))
    D, B = oracle.keystream(IR, -1.0, n, w, h)
    Dp, Bp = pyref.keystream(IR.tolist(), -1.0, n, w, h)
    assert D.tolist() == Dp
    assert B.reshape(-1).tobytes() == Bp


# ---- whole frames of one stream (Alg. 1) -------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 6, 32])
def test_encrypt_and_decrypt_stream_bit_for_bit(n):
    rng = np.random.default_rng(300 + n)
    key = oracle.key_from_bytes(rng.bytes(32))
    frames = [rng.integers(0, 256, (6, 7, 3), dtype=np.uint8) for _ in range(3)]
    Cs, Hs, st = oracle.encrypt_stream(key, -1.0, n, frames)
    Cp, Hp, stp = pyref.encrypt_stream(key, -1.0, n, frames)
    assert Hs == Hp
    for a, b in zip(Cs, Cp):
        assert np.array_equal(a, b)
    assert np.array_equal(u64(st), u64(stp))
    Ps, _ = oracle.decrypt_stream(key, -1.0, n, Cs, Hs)
    Pp, _ = pyref.decrypt_stream(key, -1.0, n, Cp, Hp)
    for P, a, b in zip(frames, Ps, Pp):
        assert np.array_equal(a, P) and np.array_equal(b, P)


# ---- the check has teeth: mistakes planted in a copy of the oracle ------------------------

MUTATIONS = {
    # R6: one component of the two seeds transposed
    "seed_z_transposed": [("l1[0] = A[0]; l1[1] = Q[1]; l1[2] = A[2]; l1[3] = Q[3];",
                           "l1[0] = A[0]; l1[1] = Q[1]; l1[2] = Q[2]; l1[3] = Q[3];"),
                          ("l2[0] = Q[0]; l2[1] = A[1]; l2[2] = Q[2]; l2[3] = A[3];",
                           "l2[0] = Q[0]; l2[1] = A[1]; l2[2] = A[2]; l2[3] = A[3];")],
    # R6: another interleave, LHCS^1 = (A.x, A.y, Q.z, Q.w).  (Exchanging A
    # and Q as a whole is no mistake: it swaps the two LHCSs, and their xor
    # is symmetric.)
    "seed_halves": [("l1[0] = A[0]; l1[1] = Q[1]; l1[2] = A[2]; l1[3] = Q[3];",
                     "l1[0] = A[0]; l1[1] = A[1]; l1[2] = Q[2]; l1[3] = Q[3];"),
                    ("l2[0] = Q[0]; l2[1] = A[1]; l2[2] = Q[2]; l2[3] = A[3];",
                     "l2[0] = Q[0]; l2[1] = Q[1]; l2[2] = A[2]; l2[3] = A[3];")],
    # R6: iterates of the next worker (worker i from IR_{2i+3}, IR_{2i+4},
    # the last one wrapping to the first pair)
    "seed_next_worker": [("static void worker_init(const double *IR, uint32_t i, double l1[4], double l2[4])\n{",
                          "static void worker_init(const double *IR, uint32_t i, double l1[4], double l2[4])\n{\n"
                          "    i = (i + 1) % g_mutant_n;"),
                         ("int vco_keystream(const double *IR, double gamma, uint32_t n, uint32_t w,\n"
                          "                  uint32_t h, uint16_t *D, uint8_t *B)\n{",
                          "int vco_keystream(const double *IR, double gamma, uint32_t n, uint32_t w,\n"
                          "                  uint32_t h, uint16_t *D, uint8_t *B)\n{\n    g_mutant_n = n;"),
                         ("#define RECON_U 32u", "#define RECON_U 32u\nstatic uint32_t g_mutant_n = 1;")],
    # R7: most significant of the six bytes first
    "stream_byte_order": [("out[pos++] = (uint8_t)(u >> (8 * b));", "out[pos++] = (uint8_t)(u >> (8 * (5 - b)));")],
    # R8: big-endian distances
    "distance_endianness": [("D[d0 + m] = (uint16_t)(s[2 * m] | ((uint16_t)s[2 * m + 1] << 8));",
                             "D[d0 + m] = (uint16_t)(s[2 * m + 1] | ((uint16_t)s[2 * m] << 8));")],
    # R8: keystream bytes taken before the distances
    "bytes_before_distances": [("memcpy(B + b0, s + 2 * nd, (size_t)nb);", "memcpy(B + b0, s, (size_t)nb);")],
    # R5: hash bytes of the fraction little-endian
    "hash_fraction_order": [("for (int b = 2; b < 8; ++b) hb48 = (hb48 << 8) | H[8 * k + b];",
                             "for (int b = 7; b >= 2; --b) hb48 = (hb48 << 8) | H[8 * k + b];")],
}


def _build_mutant(tmp_path, name, edits):
    src = open(ORACLE_SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    cdir = tmp_path / name
    cdir.mkdir()
    (cdir / "vc_oracle.c").write_text(src)
    (cdir / "vc_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "vc_oracle.h")).read())
    so = cdir / "libmutant.so"
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", str(so), str(cdir / "vc_oracle.c"), "-lm"], check=True)
    L = C.CDLL(str(so))
    f64p, u8p, u16p = C.POINTER(C.c_double), C.POINTER(C.c_uint8), C.POINTER(C.c_uint16)
    L.vco_keystream.argtypes = [f64p, C.c_double, C.c_uint32, C.c_uint32, C.c_uint32, u16p, u8p]
    L.vco_reconstruct.argtypes = [f64p, u8p, f64p]
    return L, f64p, u8p, u16p


def _mutant_agrees(L, f64p, u8p, u16p):
    """Whether the mutant agrees with pyref on the partition and
    reconstruction cases above."""
    rng = np.random.default_rng(5)
    for n, h, w in [(2, 5, 7), (6, 7, 10), (32, 9, 13)]:
        IR = rng.uniform(-20, 20, (2 * n, 4))
        D = np.zeros(3 * h + 3 * w, np.uint16)
        B = np.zeros(3 * w * h, np.uint8)
        L.vco_keystream(IR.ctypes.data_as(f64p), -1.0, n, w, h, D.ctypes.data_as(u16p), B.ctypes.data_as(u8p))
        Dp, Bp = pyref.keystream(IR.tolist(), -1.0, n, w, h)
        if D.tolist() != Dp or B.tobytes() != Bp:
            return False
    for _ in range(20):
        base = rng.uniform(-40, 40, 4)
        H = np.frombuffer(rng.bytes(32), np.uint8).copy()
        out = np.zeros(4)
        L.vco_reconstruct(base.ctypes.data_as(f64p), H.ctypes.data_as(u8p), out.ctypes.data_as(f64p))
        if not np.array_equal(u64(out), u64(pyref.reconstruct(base, H.tobytes()))):
            return False
    return True


def test_unmodified_oracle_source_agrees(tmp_path):
    assert _mutant_agrees(*_build_mutant(tmp_path, "unmodified", []))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    assert not _mutant_agrees(*_build_mutant(tmp_path, name, MUTATIONS[name]))
