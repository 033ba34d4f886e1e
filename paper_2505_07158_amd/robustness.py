"""Security experiments of Sec. IV on the GPU path.

* Differences between frames (``frame_diff``): NPCR and UACI (Sec. IV-B,
  Eqs. 14-16), MSE and PSNR, and the number of differing bits, from the
  integer counts of ``vc_frame_diff``.
* Key sensitivity (Sec. IV-A): ciphertext decrypted with the correct key and
  with one initial condition moved by delta (1e-14 in the paper).
* Cropping and channel noise (Sec. IV-C): damaged ciphertext decrypted with
  the sender's hashes (which travel beside the frames), compared with the
  plaintext.  Since decryption is a bit permutation plus a XOR with a
  keystream that depends on the key and the hash only, every damaged
  ciphertext bit damages exactly one plaintext bit: the differing-bit counts
  of ciphertext and decryption are equal, whatever the damage.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import torch

from . import vcipher as V

PEAK = 255.0
VARIABLES = ("x0", "y0", "z0", "w0")


def frame_diff(a: Sequence[torch.Tensor], b: Sequence[torch.Tensor], stream=None) -> List[Dict[str, object]]:
    """Per frame pair: per-channel ``npcr`` and ``uaci`` (percent), ``mse`` and
    ``psnr`` (dB; inf for identical channels), ``psnr_all`` over the three
    channels together, and ``bits`` (differing bits, all channels)."""
    cnt = V.vc_frame_diff(list(a), list(b), stream=stream).cpu().tolist()
    out = []
    for t, x in zip(cnt, a):
        m = int(x.shape[0]) * int(x.shape[1])
        mse = [c[2] / m for c in t]
        mse_all = sum(c[2] for c in t) / (3 * m)
        out.append({
            "npcr": [100.0 * c[0] / m for c in t],
            "uaci": [100.0 * c[1] / (PEAK * m) for c in t],
            "mse": mse,
            "psnr": [psnr_from_mse(v) for v in mse],
            "psnr_all": psnr_from_mse(mse_all),
            "bits": sum(c[3] for c in t),
        })
    return out


def psnr_from_mse(mse: float) -> float:
    return math.inf if mse == 0 else 10.0 * math.log10(PEAK * PEAK / mse)


def perturbed_key(key: "V.VcKey", var: str, delta: float) -> "V.VcKey":
    k = V.VcKey(key.x0, key.y0, key.z0, key.w0, key.gamma, key.n)
    setattr(k, var, getattr(k, var) + delta)
    return k


def key_sensitivity(key: "V.VcKey", frames: torch.Tensor, delta: float = 1e-14) -> Dict[str, List[Dict[str, object]]]:
    """Encrypts a sequence of frames (T, h, w, 3) as one stream with ``key``,
    then decrypts it with ``key`` and with each initial condition moved by
    ``delta``; returns, per key, the differences of each decrypted frame from
    the plaintext (the correct key must give none)."""
    enc = V.Cipher(key)
    try:
        C, H = enc.encrypt(frames)
    finally:
        enc.close()
    res = {}
    for name in ("correct",) + VARIABLES:
        k = key if name == "correct" else perturbed_key(key, name, delta)
        dec = V.Cipher(k)
        try:
            P = dec.decrypt(C, H)
        finally:
            dec.close()
        res[name] = frame_diff(list(P), list(frames))
    return res
