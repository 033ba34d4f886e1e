"""A second, independent statement of the per-frame cipher in plain Python,
used only to pin the C oracle (test infrastructure; it imports nothing from
the oracle or the GPU library).

It is written from the paper (Sec. II, Eq. 1-3, Algs. 1-7) and from the
protocol-v1 readings of the points the paper leaves open, with Python's own
tools: Python floats (IEEE-754 binary64, every operation rounded once,
nothing fused), Python integers for the bit work, hashlib for SHA-256 and
numpy bit arrays for the confusion.  Where the oracle and this module share
a reading, they share nothing else: a transposed seeding component, a
reversed byte order or a shifted partition in either one makes the two
disagree.

Readings (protocol v1):
  R1  classical RK4, step 0.01, IR starts after the first step
  R2  upper bound u = 32 of the integer part, all four variables
  R4  sub-frame i = bytes [floor(iL/n), floor((i+1)L/n)) of the HWC frame
  R5  reconstruction: integer part's low 16 bits xor H[8k..8k+1] (big
      endian), mod u; 52-bit fraction xor big-endian H[8k+2..8k+7]; sign kept
  R6  worker i from A = IR_{2i+1}, Q = IR_{2i+2} (1-based):
      LHCS^1 = (A.x, Q.y, A.z, Q.w), LHCS^2 = (Q.x, A.y, Q.z, A.w)
  R7  per step both LHCSs advance; for x, y, z, w the two bit patterns are
      xored and the low 48 bits emitted least significant byte first
  R8  worker i owns distances [floor(i ND/n), ...) and bytes
      [floor(i L/n), ...); its stream gives little-endian distance pairs
      first, then its keystream bytes
  R9  d_h(c, r) = D[c h + r], d_v(c, j) = D[3h + c w + j]
  R10 d_v moves a whole pixel column (its 8 bit columns together)
"""
from __future__ import annotations

import hashlib
import math
import struct

import numpy as np

SIGMA, RHO, BETA = 10.0, 28.0, 8.0 / 3.0
STEP = 0.01
U_BOUND = 32


# ---- Eq. 1 and its integrator (R1) --------------------------------------------

def rk4_step(s, gamma):
    """Classical RK4 (step 0.01) of Eq. 1 in plain Python floats, in the
    evaluation order protocol v1 fixes (right-hand sides as printed, the
    weights summed as ((k1 + 2 k2) + 2 k3) + k4 and scaled by h/6)."""
    def f(x, y, z, w):
        return (SIGMA * (y - x) + w, (RHO * x - y) - x * z, x * y - BETA * z, gamma * w - y * z)
    hh, h6 = STEP * 0.5, STEP / 6.0
    k1 = f(*s)
    k2 = f(*[a + hh * b for a, b in zip(s, k1)])
    k3 = f(*[a + hh * b for a, b in zip(s, k2)])
    k4 = f(*[a + STEP * b for a, b in zip(s, k3)])
    return [a + h6 * (((b1 + 2.0 * b2) + 2.0 * b3) + b4) for a, b1, b2, b3, b4 in zip(s, k1, k2, k3, k4)]


def chain(ic, gamma, n):
    """IR: the 2n states after ic (ic itself excluded), as a list of 4-lists."""
    s = [float(v) for v in ic]
    out = []
    for _ in range(2 * n):
        s = rk4_step(s, gamma)
        if not all(math.isfinite(v) for v in s):
            raise ValueError("non-finite LHCS_m state")
        out.append(list(s))
    return out


# ---- hash and reconstruction (Sec. II-A; R4, R5) -------------------------------

def frame_hash(frame_bytes: bytes, n: int) -> bytes:
    L = len(frame_bytes)
    acc = 0
    for i in range(n):
        part = frame_bytes[i * L // n:(i + 1) * L // n]
        acc ^= int.from_bytes(hashlib.sha256(part).digest(), "big")
    return acc.to_bytes(32, "big")


def reconstruct(base, H: bytes):
    out = []
    for k in range(4):
        v = float(base[k])
        a = abs(v)
        whole = math.floor(a)
        integer16 = int(whole) & 0xFFFF
        frac52 = int(math.floor((a - whole) * 2.0 ** 52))   # a - whole and the scaling are exact
        h16 = int.from_bytes(H[8 * k:8 * k + 2], "big")
        h48 = int.from_bytes(H[8 * k + 2:8 * k + 8], "big")
        mag = float((integer16 ^ h16) % U_BOUND) + float(frac52 ^ h48) * 2.0 ** -52
        out.append(-mag if math.copysign(1.0, v) < 0 else mag)
    return out


# ---- workers (Sec. II-B; R6-R8) ------------------------------------------------

def _pattern(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def worker_seeds(IR, i):
    """The two LHCS states of worker i (0-based) from the iterates."""
    A, Q = IR[2 * i], IR[2 * i + 1]
    first = [A[0], Q[1], A[2], Q[3]]
    second = [Q[0], A[1], Q[2], A[3]]
    return [float(v) for v in first], [float(v) for v in second]


def worker_stream(IR, gamma, i, nbytes):
    one, two = worker_seeds(IR, i)
    out = bytearray()
    while len(out) < nbytes:
        one, two = rk4_step(one, gamma), rk4_step(two, gamma)
        if not all(math.isfinite(v) for v in one + two):
            raise ValueError("non-finite worker state")
        for a, b in zip(one, two):
            low48 = (_pattern(a) ^ _pattern(b)) & ((1 << 48) - 1)
            out += low48.to_bytes(6, "little")
    return bytes(out[:nbytes])


def keystream(IR, gamma, n, w, h):
    """(D, B): D a list of 3h + 3w ints, B bytes of length 3wh."""
    ND, L = 3 * h + 3 * w, 3 * w * h
    D = [0] * ND
    B = bytearray(L)
    for i in range(n):
        d0, d1 = i * ND // n, (i + 1) * ND // n
        b0, b1 = i * L // n, (i + 1) * L // n
        s = worker_stream(IR, gamma, i, 2 * (d1 - d0) + (b1 - b0))
        for m in range(d1 - d0):
            D[d0 + m] = s[2 * m] + 256 * s[2 * m + 1]
        B[b0:b1] = s[2 * (d1 - d0):]
    return D, bytes(B)


# ---- confusion + XOR (Sec. II-C; R9, R10) on numpy bit arrays ---------------------

def _bit_rows(frame):
    """(3, h, 8w) bits: channel c, row r, bit 8j + k = bit k of pixel (r, j, c)."""
    return np.unpackbits(np.transpose(frame, (2, 0, 1))[..., None], axis=-1, bitorder="little").reshape(
        3, frame.shape[0], -1)


def _bytes_of(bits, h, w):
    return np.transpose(np.packbits(bits.reshape(3, h, w, 8), axis=-1, bitorder="little")[..., 0], (1, 2, 0))


def _as_frame(B, h, w):
    if isinstance(B, (bytes, bytearray)):
        B = np.frombuffer(bytes(B), dtype=np.uint8)
    return np.asarray(B, dtype=np.uint8).reshape(h, w, 3)


def confuse_enc(P, D, B):
    h, w, _ = P.shape
    M = _bit_rows(P)
    for c in range(3):
        for r in range(h):
            M[c, r] = np.roll(M[c, r], D[c * h + r] % (8 * w))            # Eq. 2
    for c in range(3):
        for j in range(w):
            M[c, :, 8 * j:8 * j + 8] = np.roll(M[c, :, 8 * j:8 * j + 8], D[3 * h + c * w + j] % h, axis=0)  # Eq. 3
    M ^= _bit_rows(_as_frame(B, h, w))                                     # one XOR round
    return _bytes_of(M, h, w)


def confuse_dec(C, D, B):
    h, w, _ = C.shape
    M = _bit_rows(C) ^ _bit_rows(_as_frame(B, h, w))
    for c in range(3):
        for j in range(w):
            M[c, :, 8 * j:8 * j + 8] = np.roll(M[c, :, 8 * j:8 * j + 8], -(D[3 * h + c * w + j] % h), axis=0)
    for c in range(3):
        for r in range(h):
            M[c, r] = np.roll(M[c, r], -(D[c * h + r] % (8 * w)))
    return _bytes_of(M, h, w)


# ---- Alg. 1: frames of one stream ------------------------------------------------

def encrypt_stream(key_ic, gamma, n, frames):
    """Returns (ciphertexts, hashes, final chain state)."""
    base = [float(v) for v in key_ic]
    Cs, Hs = [], []
    for P in frames:
        h, w, _ = P.shape
        H = frame_hash(P.tobytes(), n)
        IR = chain(reconstruct(base, H), gamma, n)
        D, B = keystream(IR, gamma, n, w, h)
        Cs.append(confuse_enc(P, D, B))
        Hs.append(H)
        base = IR[-1]
    return Cs, Hs, base


def decrypt_stream(key_ic, gamma, n, ciphertexts, hashes):
    base = [float(v) for v in key_ic]
    Ps = []
    for Cf, H in zip(ciphertexts, hashes):
        h, w, _ = Cf.shape
        IR = chain(reconstruct(base, H), gamma, n)
        D, B = keystream(IR, gamma, n, w, h)
        Ps.append(confuse_dec(Cf, D, B))
        base = IR[-1]
    return Ps, base
