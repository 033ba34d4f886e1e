"""Whole-cipher pins of the oracle (Alg. 1): round trips for every worker
count, the frame-to-frame chain, plaintext sensitivity against the
ideal-cipher NPCR/UACI closed forms (whose 512x512 critical values must
reproduce the numbers printed in Sec. IV-B), and the threaded form."""
import json
import os

import numpy as np
import pytest

import oracle
from metrics import npcr_critical, npcr_mean_sigma, npcr_uaci, uaci_interval, uaci_mean_sigma
from workload.synth import SynthVideo, config1_frame, key_bytes, random_frame

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_closed_forms_reproduce_paper_critical_values():
    g = json.load(open(os.path.join(GOLDEN, "npcr_uaci_512.json")))
    M = g["width"] * g["height"]
    tol = 0.5 * 10 ** -g["decimals"]
    assert abs(npcr_critical(M, g["alpha"]) - g["npcr_critical_percent"]) <= tol
    lo, hi = uaci_interval(M, g["alpha"])
    assert abs(lo - g["uaci_lower_percent"]) <= tol
    assert abs(hi - g["uaci_upper_percent"]) <= tol


@pytest.mark.parametrize("n", [1, 6, 32, 64, 256])
def test_roundtrip_config1(n):
    key = oracle.key_from_bytes(key_bytes(0))
    frames = [config1_frame(), random_frame(64, 64, 2), random_frame(64, 64, 3)]
    Cs, Hs, end_enc = oracle.encrypt_stream(key, -1.0, n, frames)
    Ps, end_dec = oracle.decrypt_stream(key, -1.0, n, Cs, Hs)
    for P, Q in zip(frames, Ps):
        np.testing.assert_array_equal(P, Q)
    np.testing.assert_array_equal(end_enc, end_dec)
    for P, C in zip(frames, Cs):
        assert (P != C).mean() > 0.98


@pytest.mark.parametrize("gamma", [-1.52, -0.06])
def test_roundtrip_gamma_range(gamma):
    key = oracle.key_from_bytes(key_bytes(5))
    frames = [random_frame(30, 41, s) for s in range(3)]
    Cs, Hs, _ = oracle.encrypt_stream(key, gamma, 7, frames)
    Ps, _ = oracle.decrypt_stream(key, gamma, 7, Cs, Hs)
    for P, Q in zip(frames, Ps):
        np.testing.assert_array_equal(P, Q)


def test_deterministic_and_hash_bound():
    key = oracle.key_from_bytes(key_bytes(1))
    P = random_frame(40, 40, 8)
    C1, H1, b1 = oracle.encrypt_frame(key, -1.0, 6, P)
    C2, H2, b2 = oracle.encrypt_frame(key, -1.0, 6, P)
    np.testing.assert_array_equal(C1, C2)
    assert H1 == H2 == oracle.frame_hash(P, 6)
    # a wrong hash at decryption gives garbage, not the plaintext (a flipped
    # bit of the integer-part byte of x moves LHCS_m by 1 in x)
    bad = H1[:1] + bytes([H1[1] ^ 1]) + H1[2:]
    Q, _ = oracle.decrypt_frame(key, -1.0, 6, C1, bad)
    assert (Q != P).mean() > 0.9


def _within(values, mu, sigma, k=5.0):
    return all(abs(v - mu) < k * sigma for v in values)


def test_plaintext_sensitivity_and_chain():
    """One pixel-channel increment in frame 0 (the experiment of Sec. IV-B)
    changes frame 0's ciphertext and, through the chain, frame 1's
    (Sec. VI-A), both as an ideal cipher would: NPCR and UACI within five
    standard deviations of the closed-form means."""
    h = w = 256
    M = h * w
    mu_n, s_n = npcr_mean_sigma(M)
    mu_u, s_u = uaci_mean_sigma(M)
    key = oracle.key_from_bytes(key_bytes(0))
    rng = np.random.default_rng(31)
    video = SynthVideo(w, h, seed=31)
    for trial in range(3):
        f0, f1 = video.frame(2 * trial), video.frame(2 * trial + 1)
        g0 = f0.copy()
        i, j, c = rng.integers(0, h), rng.integers(0, w), rng.integers(0, 3)
        g0[i, j, c] = (int(g0[i, j, c]) + int(rng.integers(1, 256))) % 256
        Ca, _, _ = oracle.encrypt_stream(key, -1.0, 32, [f0, f1])
        Cb, _, _ = oracle.encrypt_stream(key, -1.0, 32, [g0, f1])
        for t in range(2):
            npcr, uaci = npcr_uaci(Ca[t], Cb[t])
            assert _within(npcr, mu_n, s_n), (trial, t, npcr)
            assert _within(uaci, mu_u, s_u), (trial, t, uaci)


def test_threaded_equals_serial():
    key = oracle.key_from_bytes(key_bytes(2))
    P = random_frame(90, 120, 4)
    C1, H1, b1 = oracle.encrypt_frame(key, -1.0, 32, P)
    C2, H2, b2 = oracle.encrypt_frame(key, -1.0, 32, P, threads=5)
    np.testing.assert_array_equal(C1, C2)
    assert H1 == H2
    np.testing.assert_array_equal(b1, b2)
