"""Pins of the oracle's key schedule: Eq. 1 at points where it reduces to
closed forms, the RK4 integrator against an independent high-order solver
and an exact linear sub-case, boundedness of the trajectories, the
reconstruction of Sec. II-A through closed-form invariants, and the worker
byte stream through invariants (equal LHCS pairs give a zero stream; bytes
sit at the stated mantissa positions).

The IR -> worker mapping, byte order and D/B partition are protocol-v1
readings of text the paper leaves open; beyond these invariants their
parity with the authors' program is unpinned."""
import math
import struct

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle

SIGMA, RHO, BETA = 10.0, 28.0, 8.0 / 3.0
H_STEP = 0.01


def bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


# ---- Eq. 1 -----------------------------------------------------------------

def test_origin_is_fixed_point():
    assert np.all(oracle.lhcs_rhs([0.0, 0.0, 0.0, 0.0], -1.0) == 0.0)


@pytest.mark.parametrize("gamma", [-1.52, -1.0, -0.06])
def test_linear_part_at_origin(gamma):
    # With one non-zero variable every product term vanishes, leaving the
    # Jacobian column of Eq. 1 at the origin.
    e = 0.375
    np.testing.assert_array_equal(oracle.lhcs_rhs([e, 0, 0, 0], gamma), [-SIGMA * e, RHO * e, 0, 0])
    np.testing.assert_array_equal(oracle.lhcs_rhs([0, e, 0, 0], gamma), [SIGMA * e, -e, 0, 0])
    np.testing.assert_array_equal(oracle.lhcs_rhs([0, 0, e, 0], gamma), [0, 0, -BETA * e, 0])
    np.testing.assert_array_equal(oracle.lhcs_rhs([0, 0, 0, e], gamma), [e, 0, 0, gamma * e])


def test_product_terms():
    a, b = 1.5, -2.25
    # x, z: dy gets -xz
    np.testing.assert_array_equal(oracle.lhcs_rhs([a, 0, b, 0], -1.0), [-SIGMA * a, RHO * a - a * b, -BETA * b, 0])
    # x, y: dz gets +xy
    np.testing.assert_array_equal(oracle.lhcs_rhs([a, b, 0, 0], -1.0),
                                  [SIGMA * (b - a), RHO * a - b, a * b, 0])
    # y, z: dw gets -yz
    np.testing.assert_array_equal(oracle.lhcs_rhs([0, a, b, 0], -1.0), [SIGMA * a, -a, -BETA * b, -a * b])


# ---- RK4 -------------------------------------------------------------------

def _eq1(gamma):
    def f(t, s):
        x, y, z, w = s
        return [SIGMA * (y - x) + w, RHO * x - y - x * z, x * y - BETA * z, -y * z + gamma * w]
    return f


@pytest.mark.parametrize("gamma", [-1.52, -1.0, -0.06])
def test_rk4_step_matches_high_order_solver(gamma):
    # One step of classical RK4 has local error O(h^5): ~1e-8 relative here,
    # while a second-order scheme is off by ~3e-5 at the same points.
    s = np.array([1.0, 2.0, 3.0, 4.0])
    for _ in range(1500):
        s = oracle.rk4_step(s, gamma)
    f = _eq1(gamma)
    for _ in range(5):
        nxt = oracle.rk4_step(s, gamma)
        ref = solve_ivp(f, (0, H_STEP), s, method="DOP853", rtol=3e-14, atol=1e-14).y[:, -1]
        k1 = np.array(f(0, s))
        mid = s + H_STEP * np.array(f(0, s + 0.5 * H_STEP * k1))   # explicit midpoint, order 2
        err4 = np.abs(nxt - ref).max() / np.abs(ref).max()
        err2 = np.abs(mid - ref).max() / np.abs(ref).max()
        assert err4 < 1e-6 and err4 < err2 / 50, (err4, err2)
        s = nxt


def test_rk4_exact_on_linear_subspace():
    # x = y = w = 0 is invariant and z' = -beta z there; RK4 multiplies z by
    # the stability polynomial R(q) = 1 + q + q^2/2 + q^3/6 + q^4/24, q = -beta h.
    q = -BETA * H_STEP
    R = 1 + q + q * q / 2 + q ** 3 / 6 + q ** 4 / 24
    z = 7.0
    s = np.array([0.0, 0.0, z, 0.0])
    for m in range(1, 50):
        s = oracle.rk4_step(s, -1.0)
        assert s[0] == 0.0 and s[1] == 0.0 and s[3] == 0.0
        assert abs(s[2] - z * R ** m) <= 1e-13 * abs(z)


def _rk4_python(s, gamma):
    """Classical RK4 (step 0.01) of Eq. 1 in plain Python floats: IEEE-754
    binary64, every operation rounded once, nothing fused.  Written
    independently of the oracle, in the evaluation order protocol v1 fixes
    (right-hand sides as printed, the weights summed as ((k1 + 2 k2) + 2 k3) + k4
    and scaled by h/6)."""
    def f(x, y, z, w):
        return (SIGMA * (y - x) + w, (RHO * x - y) - x * z, x * y - BETA * z, gamma * w - y * z)
    hh, h6 = H_STEP * 0.5, H_STEP / 6.0
    k1 = f(*s)
    k2 = f(*[a + hh * b for a, b in zip(s, k1)])
    k3 = f(*[a + hh * b for a, b in zip(s, k2)])
    k4 = f(*[a + H_STEP * b for a, b in zip(s, k3)])
    return [a + h6 * (((b1 + 2.0 * b2) + 2.0 * b3) + b4) for a, b1, b2, b3, b4 in zip(s, k1, k2, k3, k4)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_chain_equals_python_floats_bit_for_bit(seed):
    # Cross-implementation check of the C oracle: Python floats round every
    # operation exactly like an IEEE-754 FP64 unit with no contraction, so a
    # 600-step trajectory must agree in every bit.  A fused multiply-add, a
    # reordered sum or an extended-precision temporary in the C build would
    # show up here within a few steps (the system is chaotic).
    rng = np.random.default_rng(seed)
    for _ in range(4):
        s = [float(v) for v in rng.uniform(-20.0, 20.0, 4)]
        gamma = float(rng.uniform(-1.52, -0.06))
        IR = oracle.chain(np.array(s), gamma, 300)
        assert IR.shape == (600, 4)
        for m in range(600):
            s = _rk4_python(s, gamma)
            assert [bits(v) for v in s] == [bits(float(v)) for v in IR[m]], (seed, m)


@pytest.mark.parametrize("gamma", [-1.52, -0.8, -0.06])
def test_trajectories_stay_bounded(gamma):
    rng = np.random.default_rng(int(-gamma * 100))
    for _ in range(6):
        s = rng.uniform(-32, 32, 4)
        for _ in range(4000):
            s = oracle.rk4_step(s, gamma)
            assert np.all(np.isfinite(s))
        assert np.abs(s).max() < 1000


def test_chain_excludes_initial_condition():
    ic = np.array([0.0, 0.0, 5.0, 0.0])
    IR = oracle.chain(ic, -1.0, 3)
    q = -BETA * H_STEP
    R = 1 + q + q * q / 2 + q ** 3 / 6 + q ** 4 / 24
    assert IR.shape == (6, 4)
    for m in range(6):
        assert abs(IR[m, 2] - 5.0 * R ** (m + 1)) < 1e-12
        assert IR[m, 0] == IR[m, 1] == IR[m, 3] == 0.0


# ---- key bytes and reconstruction -------------------------------------------

def test_key_from_bytes_closed_form():
    K = bytes(32)
    assert np.all(oracle.key_from_bytes(K) == 0.0)
    K = bytes([0x00, 0x25, 0x80, 0, 0, 0, 0, 0]) + bytes([0xFF] * 8) + bytes([0x01, 0x00, 0, 0, 0, 0, 0, 1]) + bytes(8)
    v = oracle.key_from_bytes(K)
    assert v[0] == 5.5                                  # 0x0025 mod 32 = 5; 0x80 << 40 / 2^48 = 0.5
    assert v[1] == 31 + (2 ** 48 - 1) / 2 ** 48         # 0xFFFF mod 32 = 31
    assert v[2] == 0 + 2.0 ** -48                       # 0x0100 mod 32 = 0
    assert v[3] == 0.0


def _fraction52(x):
    return np.array([math.ldexp(float(v), -52) for v in x])


def test_reconstruct_zero_hash_is_identity():
    rng = np.random.default_rng(5)
    for _ in range(200):
        # values in [1, 32) with at most 52 fractional bits
        base = np.floor(rng.uniform(1, 32, 4) * 2 ** 48) / 2 ** 48 * rng.choice([-1, 1], 4)
        np.testing.assert_array_equal(oracle.reconstruct(base, bytes(32)), base)


def test_reconstruct_range_and_sign():
    rng = np.random.default_rng(6)
    for _ in range(300):
        base = rng.uniform(-60, 60, 4)
        H = rng.bytes(32)
        once = oracle.reconstruct(base, H)
        assert np.all(np.abs(once) < 32)
        assert np.all(np.signbit(once) == np.signbit(base))
        np.testing.assert_array_equal(oracle.reconstruct(-base, H), -once)


def test_reconstruct_involution_exact_when_integer_part_cancels():
    # If the two hash bytes cancel the integer part (I xor h16 = 0 mod 32),
    # the intermediate value is the bare fraction, exactly representable,
    # and applying the same hash again restores reconstruct(base, 0) exactly.
    rng = np.random.default_rng(16)
    for _ in range(200):
        base = rng.uniform(1, 60, 4) * rng.choice([-1, 1], 4)
        H = bytearray(rng.bytes(32))
        for k in range(4):
            I = int(math.floor(abs(base[k]))) & 0xFFFF
            H[8 * k + 1] = (H[8 * k + 1] & 0xE0) | (I & 0x1F)
        H = bytes(H)
        once = oracle.reconstruct(base, H)
        assert np.all(np.abs(once) < 1)
        np.testing.assert_array_equal(oracle.reconstruct(once, H), oracle.reconstruct(base, bytes(32)))


def test_reconstruct_bit_positions():
    # integer part 0 keeps every result below 2, where doubles resolve 2^-52
    base = np.array([0.75, 0.5625, 0.6875, 0.9375])
    ref = oracle.reconstruct(base, bytes(32))
    for k in range(4):
        def flip(byte, bit):
            H = bytearray(32)
            H[8 * k + byte] ^= 1 << bit
            return oracle.reconstruct(base, bytes(H))
        # least significant hash byte -> least significant fraction bit 2^-52
        assert abs(flip(7, 0)[k] - ref[k]) == 2.0 ** -52
        # most significant of the six fraction bytes -> 2^-5
        assert abs(flip(2, 7)[k] - ref[k]) == 2.0 ** -5
        # low byte of the integer part -> +-1 (mod 32)
        assert abs(flip(1, 0)[k] - ref[k]) == 1.0
        # bits above the bound u = 32 are removed by the modulo
        assert flip(0, 3)[k] == ref[k] and flip(1, 5)[k] == ref[k]
        # other variables are untouched
        others = [m for m in range(4) if m != k]
        np.testing.assert_array_equal(flip(7, 0)[others], ref[others])


# ---- worker streams -----------------------------------------------------------

def test_equal_pair_gives_zero_stream():
    rng = np.random.default_rng(7)
    IR = rng.uniform(-20, 20, (8, 4))
    IR[3] = IR[2]      # worker 1: A = IR_3, Q = IR_4 (1-based) identical
    assert not oracle.worker_stream(IR, -1.0, 1, 2400).any()
    assert oracle.worker_stream(IR, -1.0, 0, 2400).any()


def test_stream_byte_positions():
    # A = origin, Q = (0, 0, q, 0): LHCS^1 = origin (a fixed point), LHCS^2
    # runs on the invariant z-axis.  Per step the x, y, w bytes are zero and
    # the z bytes are the low 48 mantissa bits of z_s, least significant first.
    q = 11.0
    IR = np.zeros((2, 4))
    IR[1, 2] = q
    steps = 40
    s = oracle.worker_stream(IR, -1.0, 0, 24 * steps).reshape(steps, 24)
    assert not s[:, 0:12].any() and not s[:, 18:24].any()
    qq = -BETA * H_STEP
    R = 1 + qq + qq * qq / 2 + qq ** 3 / 6 + qq ** 4 / 24
    for m in range(steps):
        approx = q * R ** (m + 1)
        low48 = int.from_bytes(s[m, 12:18].tobytes(), "little")
        rebuilt = struct.unpack("<d", struct.pack("<Q", (bits(approx) & ~((1 << 48) - 1)) | low48))[0]
        assert abs(rebuilt - approx) <= 1e-12 * abs(approx)


def test_keystream_partition_single_worker():
    rng = np.random.default_rng(8)
    IR = rng.uniform(-20, 20, (2, 4))
    h, w = 5, 7
    ND, L = 3 * h + 3 * w, 3 * w * h
    D, B = oracle.keystream(IR, -1.0, 1, w, h)
    s = oracle.worker_stream(IR, -1.0, 0, 2 * ND + L)
    np.testing.assert_array_equal(D, s[:2 * ND].view("<u2"))
    np.testing.assert_array_equal(B.reshape(-1), s[2 * ND:])


def test_keystream_partition_many_workers():
    rng = np.random.default_rng(9)
    n, h, w = 6, 9, 11
    IR = rng.uniform(-20, 20, (2 * n, 4))
    ND, L = 3 * h + 3 * w, 3 * w * h
    D, B = oracle.keystream(IR, -1.0, n, w, h)
    Bf = B.reshape(-1)
    for i in range(n):
        d0, d1 = i * ND // n, (i + 1) * ND // n
        b0, b1 = i * L // n, (i + 1) * L // n
        s = oracle.worker_stream(IR, -1.0, i, 2 * (d1 - d0) + (b1 - b0))
        np.testing.assert_array_equal(D[d0:d1], s[:2 * (d1 - d0)].view("<u2"))
        np.testing.assert_array_equal(Bf[b0:b1], s[2 * (d1 - d0):])


def test_keystream_bytes_look_uniform():
    from scipy.stats import chisquare
    ic = oracle.reconstruct(oracle.key_from_bytes(bytes(range(32))), bytes(32))
    IR = oracle.chain(ic, -1.0, 6)
    D, B = oracle.keystream(IR, -1.0, 6, 640, 480)
    counts = np.bincount(B.reshape(-1), minlength=256)
    assert chisquare(counts).pvalue > 1e-4
    lo = np.bincount((D & 0xFF).astype(np.int64), minlength=256)
    assert chisquare(lo).pvalue > 1e-4
