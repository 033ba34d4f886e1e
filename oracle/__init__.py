"""CPU oracle of the diffusion-free video cipher (arXiv 2505.07158).

TEST INFRASTRUCTURE ONLY.  A thin ctypes wrapper over ``vc_oracle.c``, a
plain scalar C statement of the cipher written from the paper.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import this
package; the GPU library never does, and the two share no code.

Frames are numpy ``uint8`` arrays of shape ``(h, w, 3)`` (row-major, channels
interleaved).  ``n`` is the paper's worker count (sub-frames and worker LHCS
pairs).  Keys are four doubles ``(x0, y0, z0, w0)`` plus ``gamma``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libvc_oracle.so")

# gcc flags: scalar SSE2 doubles, IEEE rounding, no contraction into FMA.
CFLAGS = ["-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra", "-pthread"]


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/libvc_oracle.so`` and return its path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None

_u8p = C.POINTER(C.c_uint8)
_u16p = C.POINTER(C.c_uint16)
_f64p = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        L.vco_sha256.argtypes = [_u8p, C.c_uint64, _u8p]
        L.vco_frame_hash.argtypes = [_u8p, C.c_uint64, C.c_uint32, _u8p]
        L.vco_key_from_bytes.argtypes = [_u8p, _f64p]
        L.vco_reconstruct.argtypes = [_f64p, _u8p, _f64p]
        L.vco_rk4_step.argtypes = [_f64p, C.c_double]
        L.vco_rk4_step.restype = C.c_int
        L.vco_lhcs_rhs.argtypes = [_f64p, C.c_double, _f64p]
        L.vco_chain.argtypes = [_f64p, C.c_double, C.c_uint32, _f64p]
        L.vco_chain.restype = C.c_int
        L.vco_keystream.argtypes = [_f64p, C.c_double, C.c_uint32, C.c_uint32,
                                    C.c_uint32, _u16p, _u8p]
        L.vco_keystream.restype = C.c_int
        L.vco_worker_stream.argtypes = [_f64p, C.c_double, C.c_uint32, C.c_uint64, _u8p]
        L.vco_worker_stream.restype = C.c_int
        for name in ("vco_confuse_enc", "vco_confuse_dec"):
            getattr(L, name).argtypes = [_u8p, C.c_uint32, C.c_uint32, _u16p, _u8p, _u8p]
            getattr(L, name).restype = None
        for name in ("vco_confuse_enc_literal", "vco_confuse_dec_literal"):
            getattr(L, name).argtypes = [_u8p, C.c_uint32, C.c_uint32, _u16p, _u8p, _u8p]
            getattr(L, name).restype = C.c_int
        L.vco_encrypt_frame.argtypes = [_f64p, C.c_double, C.c_uint32, _u8p,
                                        C.c_uint32, C.c_uint32, _u8p, _u8p]
        L.vco_encrypt_frame.restype = C.c_int
        L.vco_decrypt_frame.argtypes = [_f64p, C.c_double, C.c_uint32, _u8p,
                                        C.c_uint32, C.c_uint32, _u8p, _u8p]
        L.vco_decrypt_frame.restype = C.c_int
        L.vco_encrypt_frame_mt.argtypes = [_f64p, C.c_double, C.c_uint32, _u8p,
                                           C.c_uint32, C.c_uint32, _u8p, _u8p, C.c_uint32]
        L.vco_encrypt_frame_mt.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _frame(P) -> np.ndarray:
    P = _u8(P)
    if P.ndim != 3 or P.shape[2] != 3:
        raise ValueError("frame must have shape (h, w, 3)")
    return P


class OracleError(RuntimeError):
    pass


# --- SHA-256 and the frame hash (Sec. II-A) -------------------------------

def sha256(msg: bytes) -> bytes:
    m = np.frombuffer(bytes(msg), dtype=np.uint8).copy() if len(msg) else np.zeros(1, np.uint8)
    out = np.zeros(32, np.uint8)
    lib().vco_sha256(_p(m, _u8p), len(msg), _p(out, _u8p))
    return out.tobytes()


def frame_hash(frame, n: int) -> bytes:
    f = _u8(frame).reshape(-1)
    out = np.zeros(32, np.uint8)
    lib().vco_frame_hash(_p(f, _u8p), f.size, n, _p(out, _u8p))
    return out.tobytes()


# --- key schedule (Sec. II-A, II-B) ---------------------------------------

def key_from_bytes(key32: bytes) -> np.ndarray:
    k = np.frombuffer(bytes(key32), dtype=np.uint8).copy()
    if k.size != 32:
        raise ValueError("key must be 32 bytes")
    ic = np.zeros(4, np.float64)
    lib().vco_key_from_bytes(_p(k, _u8p), _p(ic, _f64p))
    return ic


def reconstruct(base, H: bytes) -> np.ndarray:
    b = _f64(base)
    h = np.frombuffer(bytes(H), dtype=np.uint8).copy()
    ic = np.zeros(4, np.float64)
    lib().vco_reconstruct(_p(b, _f64p), _p(h, _u8p), _p(ic, _f64p))
    return ic


def lhcs_rhs(s, gamma: float) -> np.ndarray:
    s = _f64(s)
    d = np.zeros(4, np.float64)
    lib().vco_lhcs_rhs(_p(s, _f64p), gamma, _p(d, _f64p))
    return d


def rk4_step(s, gamma: float) -> np.ndarray:
    s = _f64(s).copy()
    if lib().vco_rk4_step(_p(s, _f64p), gamma) != 0:
        raise OracleError("non-finite LHCS state")
    return s


def chain(ic, gamma: float, n: int) -> np.ndarray:
    ic = _f64(ic)
    IR = np.zeros((2 * n, 4), np.float64)
    if lib().vco_chain(_p(ic, _f64p), gamma, n, _p(IR, _f64p)) != 0:
        raise OracleError("non-finite LHCS_m trajectory")
    return IR


def worker_stream(IR, gamma: float, i: int, nbytes: int) -> np.ndarray:
    IR = _f64(IR)
    out = np.zeros(max(nbytes, 1), np.uint8)
    if lib().vco_worker_stream(_p(IR, _f64p), gamma, i, nbytes, _p(out, _u8p)) != 0:
        raise OracleError("non-finite worker trajectory")
    return out[:nbytes]


def keystream(IR, gamma: float, n: int, w: int, h: int):
    """Return (D, B): D uint16 of length 3h + 3w, B uint8 of shape (h, w, 3)."""
    IR = _f64(IR)
    if IR.shape != (2 * n, 4):
        raise ValueError("IR must have shape (2n, 4)")
    D = np.zeros(3 * h + 3 * w, np.uint16)
    B = np.zeros((h, w, 3), np.uint8)
    if lib().vco_keystream(_p(IR, _f64p), gamma, n, w, h, _p(D, _u16p), _p(B, _u8p)) != 0:
        raise OracleError("non-finite worker trajectory")
    return D, B


# --- confusion + XOR (Sec. II-C) ------------------------------------------

def _confuse(name, X, D, B):
    X = _frame(X)
    h, w, _ = X.shape
    D = np.ascontiguousarray(D, dtype=np.uint16)
    B = _u8(B)
    if D.size != 3 * h + 3 * w or B.size != X.size:
        raise ValueError("D or B has the wrong size")
    out = np.zeros_like(X)
    rc = getattr(lib(), name)(_p(X, _u8p), w, h, _p(D, _u16p), _p(B, _u8p), _p(out, _u8p))
    if rc not in (None, 0):
        raise OracleError(name + " failed")
    return out


def confuse_enc(P, D, B):
    return _confuse("vco_confuse_enc", P, D, B)


def confuse_dec(Cf, D, B):
    return _confuse("vco_confuse_dec", Cf, D, B)


def confuse_enc_literal(P, D, B):
    return _confuse("vco_confuse_enc_literal", P, D, B)


def confuse_dec_literal(Cf, D, B):
    return _confuse("vco_confuse_dec_literal", Cf, D, B)


# --- whole frames and streams (Alg. 1) ------------------------------------

def encrypt_frame(base, gamma: float, n: int, P, threads: int = 1):
    """Encrypt one frame.  Returns (C, H, next_base)."""
    P = _frame(P)
    h, w, _ = P.shape
    b = _f64(base).copy()
    Cf = np.zeros_like(P)
    H = np.zeros(32, np.uint8)
    if threads > 1:
        rc = lib().vco_encrypt_frame_mt(_p(b, _f64p), gamma, n, _p(P, _u8p), w, h,
                                        _p(Cf, _u8p), _p(H, _u8p), threads)
    else:
        rc = lib().vco_encrypt_frame(_p(b, _f64p), gamma, n, _p(P, _u8p), w, h,
                                     _p(Cf, _u8p), _p(H, _u8p))
    if rc != 0:
        raise OracleError("encryption failed (non-finite trajectory)")
    return Cf, H.tobytes(), b


def decrypt_frame(base, gamma: float, n: int, Cf, H: bytes):
    """Decrypt one frame with the sender's hash H.  Returns (P, next_base)."""
    Cf = _frame(Cf)
    h, w, _ = Cf.shape
    b = _f64(base).copy()
    Hb = np.frombuffer(bytes(H), dtype=np.uint8).copy()
    P = np.zeros_like(Cf)
    if lib().vco_decrypt_frame(_p(b, _f64p), gamma, n, _p(Cf, _u8p), w, h,
                               _p(Hb, _u8p), _p(P, _u8p)) != 0:
        raise OracleError("decryption failed (non-finite trajectory)")
    return P, b


def encrypt_stream(key_ic, gamma: float, n: int, frames):
    """Encrypt a sequence of frames of one stream from the user key.
    Returns (C list, H list, final chain state)."""
    base = _f64(key_ic).copy()
    Cs, Hs = [], []
    for P in frames:
        Cf, H, base = encrypt_frame(base, gamma, n, P)
        Cs.append(Cf)
        Hs.append(H)
    return Cs, Hs, base


def decrypt_stream(key_ic, gamma: float, n: int, cipher_frames, hashes):
    base = _f64(key_ic).copy()
    Ps = []
    for Cf, H in zip(cipher_frames, hashes):
        P, base = decrypt_frame(base, gamma, n, Cf, H)
        Ps.append(P)
    return Ps, base


def stream_hashes(frames, n: int):
    """Frame hashes of a sequence (the only part of the chain that does not
    depend on earlier frames)."""
    return [frame_hash(P, n) for P in frames]


def chain_states(key_ic, gamma: float, n: int, hashes):
    """Chain bases of a stream: element t is the state used for frame t."""
    base = _f64(key_ic).copy()
    out = []
    for H in hashes:
        out.append(base.copy())
        IR = chain(reconstruct(base, H), gamma, n)
        base = IR[-1].copy()
    out.append(base.copy())
    return out
