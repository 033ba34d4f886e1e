/*
 * vc_oracle.c -- CPU oracle of the diffusion-free video cipher of
 * arXiv 2505.07158 ("Real-Time Bit-Level Encryption of Full High-Definition
 * Video Without Diffusion").
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, scalar statement of the cipher,
 * written from the paper, used to check the GPU library byte for byte.  It
 * shares no code with the GPU library.  Only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * Where the paper leaves a detail open, the reading used here is marked
 * [Rk] where it is applied (protocol version 1), with the passage it
 * interprets and the choice made.
 *
 * Parity status of each part:
 *   SHA-256 and the frame hash ....... pinned (hashlib, openssl, FIPS 180-4
 *                                      example messages)
 *   Eq. 1 right-hand side, RK4 ....... pinned (solve_ivp, exact linear
 *                                      sub-case, convergence order)
 *   reconstruction ................... pinned by closed-form invariants
 *                                      (involution, bit positions, H = 0)
 *   worker init / byte stream / D,B .. readings R6-R9; pinned by
 *                                      invariants (zero stream for equal
 *                                      LHCS pairs, byte accounting) and bit
 *                                      for bit by a separate pure-Python
 *                                      statement of the same readings,
 *                                      which catches planted mistakes.
 *                                      Against the authors' program the
 *                                      readings stay unpinned: their code
 *                                      is not available.
 *   confusion + XOR and inverse ...... pinned (bit-matrix form of Eqs. 2-3
 *                                      and Algs. 3-7, numpy roll/packbits,
 *                                      bijection probes)
 */
#include "vc_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* SHA-256, FIPS 180-4                                                 */
/* ------------------------------------------------------------------ */

static uint32_t sha_K[64];
static uint32_t sha_H0[8];
static pthread_once_t sha_once = PTHREAD_ONCE_INIT;

/* First 64 primes, by trial division. */
static void first_primes(uint32_t *p, int count)
{
    int found = 0;
    for (uint32_t c = 2; found < count; ++c) {
        int prime = 1;
        for (uint32_t d = 2; d * d <= c; ++d)
            if (c % d == 0) { prime = 0; break; }
        if (prime) p[found++] = c;
    }
}

/* floor(cbrt(p) * 2^32) by bisection on exact integers: the largest r with
 * r^3 <= p * 2^96.  The low 32 bits are the first 32 bits of the fraction. */
static uint64_t icbrt_scaled(uint32_t p)
{
    unsigned __int128 target = (unsigned __int128)p << 96;
    uint64_t lo = 0, hi = (uint64_t)1 << 40;
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        unsigned __int128 m = mid;
        if (m * m * m <= target) lo = mid; else hi = mid;
    }
    return lo;
}

/* floor(sqrt(p) * 2^32): the largest r with r^2 <= p * 2^64. */
static uint64_t isqrt_scaled(uint32_t p)
{
    unsigned __int128 target = (unsigned __int128)p << 64;
    uint64_t lo = 0, hi = (uint64_t)1 << 40;
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        unsigned __int128 m = mid;
        if (m * m <= target) lo = mid; else hi = mid;
    }
    return lo;
}

/* FIPS 180-4 sec. 4.2.2 (K: cube roots of the first 64 primes) and
 * sec. 5.3.3 (H(0): square roots of the first 8 primes). */
static void sha_init_constants(void)
{
    uint32_t p[64];
    first_primes(p, 64);
    for (int t = 0; t < 64; ++t) sha_K[t] = (uint32_t)icbrt_scaled(p[t]);
    for (int t = 0; t < 8; ++t) sha_H0[t] = (uint32_t)isqrt_scaled(p[t]);
}

static uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }
static uint32_t Ch(uint32_t x, uint32_t y, uint32_t z) { return (x & y) ^ (~x & z); }
static uint32_t Maj(uint32_t x, uint32_t y, uint32_t z) { return (x & y) ^ (x & z) ^ (y & z); }
static uint32_t Sig0(uint32_t x) { return rotr(x, 2) ^ rotr(x, 13) ^ rotr(x, 22); }
static uint32_t Sig1(uint32_t x) { return rotr(x, 6) ^ rotr(x, 11) ^ rotr(x, 25); }
static uint32_t sig0(uint32_t x) { return rotr(x, 7) ^ rotr(x, 18) ^ (x >> 3); }
static uint32_t sig1(uint32_t x) { return rotr(x, 17) ^ rotr(x, 19) ^ (x >> 10); }

/* FIPS 180-4 sec. 6.2.2: process one 512-bit block. */
static void sha_compress(uint32_t Hs[8], const uint8_t block[64])
{
    uint32_t W[64];
    for (int t = 0; t < 16; ++t)
        W[t] = ((uint32_t)block[4 * t] << 24) | ((uint32_t)block[4 * t + 1] << 16) |
               ((uint32_t)block[4 * t + 2] << 8) | (uint32_t)block[4 * t + 3];
    for (int t = 16; t < 64; ++t)
        W[t] = sig1(W[t - 2]) + W[t - 7] + sig0(W[t - 15]) + W[t - 16];
    uint32_t a = Hs[0], b = Hs[1], c = Hs[2], d = Hs[3];
    uint32_t e = Hs[4], f = Hs[5], g = Hs[6], h = Hs[7];
    for (int t = 0; t < 64; ++t) {
        uint32_t T1 = h + Sig1(e) + Ch(e, f, g) + sha_K[t] + W[t];
        uint32_t T2 = Sig0(a) + Maj(a, b, c);
        h = g; g = f; f = e; e = d + T1;
        d = c; c = b; b = a; a = T1 + T2;
    }
    Hs[0] += a; Hs[1] += b; Hs[2] += c; Hs[3] += d;
    Hs[4] += e; Hs[5] += f; Hs[6] += g; Hs[7] += h;
}

/* FIPS 180-4 sec. 5.1.1 (padding) and 6.2 (hash computation). */
void vco_sha256(const uint8_t *msg, uint64_t len, uint8_t out[32])
{
    pthread_once(&sha_once, sha_init_constants);
    uint32_t Hs[8];
    memcpy(Hs, sha_H0, sizeof Hs);
    uint64_t full = len / 64;
    for (uint64_t blk = 0; blk < full; ++blk) sha_compress(Hs, msg + 64 * blk);
    /* Tail: the remaining bytes, a single 1 bit, zeros, 64-bit length. */
    uint8_t tail[128];
    memset(tail, 0, sizeof tail);
    uint64_t rem = len - 64 * full;
    memcpy(tail, msg + 64 * full, (size_t)rem);
    tail[rem] = 0x80;
    uint64_t tail_len = (rem + 1 + 8 <= 64) ? 64 : 128;
    uint64_t bits = len * 8;
    for (int k = 0; k < 8; ++k) tail[tail_len - 1 - k] = (uint8_t)(bits >> (8 * k));
    for (uint64_t off = 0; off < tail_len; off += 64) sha_compress(Hs, tail + off);
    for (int t = 0; t < 8; ++t) {
        out[4 * t] = (uint8_t)(Hs[t] >> 24);
        out[4 * t + 1] = (uint8_t)(Hs[t] >> 16);
        out[4 * t + 2] = (uint8_t)(Hs[t] >> 8);
        out[4 * t + 3] = (uint8_t)Hs[t];
    }
}

/* Sub-frame i covers bytes [floor(i*L/n), floor((i+1)*L/n)) [R4]. */
static uint64_t split_at(uint64_t L, uint32_t n, uint32_t i)
{
    return (uint64_t)(((unsigned __int128)L * i) / n);
}

/* Sec. II-A: h_i = SHA-256(f_i); H = h_1 xor ... xor h_n. */
void vco_frame_hash(const uint8_t *frame, uint64_t L, uint32_t n, uint8_t H[32])
{
    memset(H, 0, 32);
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t a = split_at(L, n, i), b = split_at(L, n, i + 1);
        uint8_t hi[32];
        vco_sha256(frame + a, b - a, hi);
        for (int k = 0; k < 32; ++k) H[k] ^= hi[k];
    }
}

/* ------------------------------------------------------------------ */
/* Key, reconstruction, LHCS                                           */
/* ------------------------------------------------------------------ */

/* [R2] predefined upper bound u of the integer part, same for x, y, z, w. */
#define RECON_U 32u
static const double TWO52 = 4503599627370496.0;          /* 2^52 */
static const double TWO_M52 = 1.0 / 4503599627370496.0;  /* 2^-52, exact */
static const double TWO_M48 = 1.0 / 281474976710656.0;   /* 2^-48, exact */

/* [R3] key bytes 8k..8k+7 give IC k: integer part (big-endian u16 of the
 * first two bytes) mod u, fraction = big-endian u48 of the next six bytes
 * times 2^-48.  Exact in double. */
void vco_key_from_bytes(const uint8_t K[32], double ic[4])
{
    for (int k = 0; k < 4; ++k) {
        const uint8_t *q = K + 8 * k;
        uint32_t ip = (((uint32_t)q[0] << 8) | q[1]) % RECON_U;
        uint64_t fr = 0;
        for (int b = 2; b < 8; ++b) fr = (fr << 8) | q[b];
        ic[k] = (double)ip + (double)fr * TWO_M48;
    }
}

/* Sec. II-A reconstruction [R5], per variable v of base:
 *  1. integer part: the two least significant bytes of floor(|v|) xor two
 *     hash bytes (big-endian H[8k], H[8k+1]), reduced mod u;
 *  2. fraction: the 52-bit binary fraction of |v|, whose six least
 *     significant bytes are xored with H[8k+2..8k+7] (big-endian);
 *  3. combine integer + fraction * 2^-52 (one rounding), sign of v kept. */
void vco_reconstruct(const double base[4], const uint8_t H[32], double ic[4])
{
    for (int k = 0; k < 4; ++k) {
        double a = fabs(base[k]);
        double ip = floor(a);
        /* ip mod 65536, exact for every finite ip */
        double low16 = ip - 65536.0 * floor(ip / 65536.0);
        uint64_t I = (uint64_t)low16;
        uint64_t G = (uint64_t)floor((a - ip) * TWO52);
        uint64_t hb16 = ((uint64_t)H[8 * k] << 8) | H[8 * k + 1];
        uint64_t hb48 = 0;
        for (int b = 2; b < 8; ++b) hb48 = (hb48 << 8) | H[8 * k + b];
        uint64_t I2 = (I ^ hb16) % RECON_U;
        uint64_t G2 = G ^ hb48;
        double r = (double)I2 + (double)G2 * TWO_M52;
        ic[k] = signbit(base[k]) ? -r : r;
    }
}

/* Eq. 1 constants. */
static const double SIGMA = 10.0;
static const double RHO = 28.0;
#define BETA (8.0 / 3.0)
/* [R1] classical RK4 with step 0.01 */
static const double STEP = 0.01;

void vco_lhcs_rhs(const double s[4], double gamma, double ds[4])
{
    const double x = s[0], y = s[1], z = s[2], w = s[3];
    ds[0] = SIGMA * (y - x) + w;          /* dx/dt = sigma(y - x) + w   */
    ds[1] = (RHO * x - y) - x * z;        /* dy/dt = rho x - y - x z    */
    ds[2] = x * y - BETA * z;             /* dz/dt = x y - beta z       */
    ds[3] = gamma * w - y * z;            /* dw/dt = -y z + gamma w     */
}

int vco_rk4_step(double s[4], double gamma)
{
    const double hh = STEP * 0.5, h6 = STEP / 6.0;
    double k1[4], k2[4], k3[4], k4[4], t[4];
    vco_lhcs_rhs(s, gamma, k1);
    for (int i = 0; i < 4; ++i) t[i] = s[i] + hh * k1[i];
    vco_lhcs_rhs(t, gamma, k2);
    for (int i = 0; i < 4; ++i) t[i] = s[i] + hh * k2[i];
    vco_lhcs_rhs(t, gamma, k3);
    for (int i = 0; i < 4; ++i) t[i] = s[i] + STEP * k3[i];
    vco_lhcs_rhs(t, gamma, k4);
    int ok = 0;
    for (int i = 0; i < 4; ++i) {
        s[i] = s[i] + h6 * (((k1[i] + 2.0 * k2[i]) + 2.0 * k3[i]) + k4[i]);
        if (!isfinite(s[i])) ok = -1;
    }
    return ok;
}

/* Alg. 1: IR = {x_1..w_1, ..., x_2n..w_2n}, the 2n states after the
 * reconstructed initial condition (which itself is not part of IR). */
int vco_chain(const double ic[4], double gamma, uint32_t n, double *IR)
{
    double s[4] = {ic[0], ic[1], ic[2], ic[3]};
    for (uint32_t m = 0; m < 2 * n; ++m) {
        if (vco_rk4_step(s, gamma) != 0) return -1;
        memcpy(IR + 4 * (uint64_t)m, s, sizeof s);
    }
    return 0;
}

static uint64_t dbits(double v)
{
    uint64_t u;
    memcpy(&u, &v, sizeof u);
    return u;
}

/* [R6] worker i (0-based) is seeded from A = IR_{2i+1}, Q = IR_{2i+2}:
 * LHCS^{i,1} = (A.x, Q.y, A.z, Q.w), LHCS^{i,2} = (Q.x, A.y, Q.z, A.w). */
static void worker_init(const double *IR, uint32_t i, double l1[4], double l2[4])
{
    const double *A = IR + 4 * (uint64_t)(2 * i);
    const double *Q = IR + 4 * (uint64_t)(2 * i + 1);
    l1[0] = A[0]; l1[1] = Q[1]; l1[2] = A[2]; l1[3] = Q[3];
    l2[0] = Q[0]; l2[1] = A[1]; l2[2] = Q[2]; l2[3] = A[3];
}

/* Sec. II-B [R7]: each step advances both LHCSs one RK4 step, then for
 * x, y, z, w in turn the two iterates' FP64 bit patterns are xored and the
 * six least significant mantissa bytes are emitted, least significant
 * first: 24 bytes per step. */
int vco_worker_stream(const double *IR, double gamma, uint32_t i,
                      uint64_t nbytes, uint8_t *out)
{
    double l1[4], l2[4];
    worker_init(IR, i, l1, l2);
    uint64_t pos = 0;
    while (pos < nbytes) {
        if (vco_rk4_step(l1, gamma) != 0) return -1;
        if (vco_rk4_step(l2, gamma) != 0) return -1;
        for (int c = 0; c < 4; ++c) {
            uint64_t u = dbits(l1[c]) ^ dbits(l2[c]);
            for (int b = 0; b < 6 && pos < nbytes; ++b)
                out[pos++] = (uint8_t)(u >> (8 * b));
        }
    }
    return 0;
}

/* [R8] worker i owns distances [floor(i*ND/n), floor((i+1)*ND/n)) and
 * bytes [floor(i*L/n), floor((i+1)*L/n)); its stream gives its distances
 * first (two bytes each, little-endian) and then its bytes. */
static int keystream_worker(const double *IR, double gamma, uint32_t n,
                            uint32_t w, uint32_t h, uint32_t i,
                            uint16_t *D, uint8_t *B)
{
    uint64_t ND = 3ull * h + 3ull * w, L = 3ull * w * h;
    uint64_t d0 = split_at(ND, n, i), d1 = split_at(ND, n, i + 1);
    uint64_t b0 = split_at(L, n, i), b1 = split_at(L, n, i + 1);
    uint64_t nd = d1 - d0, nb = b1 - b0;
    uint64_t total = 2 * nd + nb;
    uint8_t *s = (uint8_t *)malloc(total ? total : 1);
    if (!s) return -1;
    int rc = vco_worker_stream(IR, gamma, i, total, s);
    if (rc == 0) {
        for (uint64_t m = 0; m < nd; ++m)
            D[d0 + m] = (uint16_t)(s[2 * m] | ((uint16_t)s[2 * m + 1] << 8));
        memcpy(B + b0, s + 2 * nd, (size_t)nb);
    }
    free(s);
    return rc;
}

int vco_keystream(const double *IR, double gamma, uint32_t n, uint32_t w,
                  uint32_t h, uint16_t *D, uint8_t *B)
{
    for (uint32_t i = 0; i < n; ++i)
        if (keystream_worker(IR, gamma, n, w, h, i, D, B) != 0) return -1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Confusion + XOR (Sec. II-C)                                         */
/* ------------------------------------------------------------------ */
/* [R9] d_h(c, r) = D[c*h + r] (one per row and channel), d_v(c, j) =
 * D[3h + c*w + j] (one per pixel column and channel) [R10]; B and frames
 * are indexed (i*w + j)*3 + c. */

#define PIX(buf, w, i, j, c) ((buf)[((uint64_t)(i) * (w) + (j)) * 3 + (c)])

/* Closed form.  Eq. 2 moves bit x of bit-row r to (x + d_h) mod 8w; Eq. 3
 * moves bit-row r of bit-column x to (r + d_v) mod h.  Output byte (i,j,c)
 * therefore takes the eight bits that start at bit s = (8j - d_h(c,r))
 * mod 8w of source row r = (i - d_v(c,j)) mod h, least significant bit
 * first (Algs. 3 and 7), and is xored with B (Alg. 6). */
void vco_confuse_enc(const uint8_t *P, uint32_t w, uint32_t h,
                     const uint16_t *D, const uint8_t *B, uint8_t *C)
{
    const uint64_t W8 = 8ull * w;
    for (uint32_t i = 0; i < h; ++i)
        for (uint32_t j = 0; j < w; ++j)
            for (uint32_t c = 0; c < 3; ++c) {
                uint64_t dv = D[3ull * h + (uint64_t)c * w + j] % h;
                uint64_t r = (i + h - dv) % h;
                uint64_t dh = D[(uint64_t)c * h + r] % W8;
                uint64_t s = (8ull * j + W8 - dh) % W8;
                uint64_t q = s >> 3, t = s & 7, q2 = (q + 1) % w;
                uint32_t pair = PIX(P, w, r, q, c) | ((uint32_t)PIX(P, w, r, q2, c) << 8);
                PIX(C, w, i, j, c) = (uint8_t)((pair >> t) & 0xFF) ^ PIX(B, w, i, j, c);
            }
}

/* Inverse: Y = C xor B; undo Eq. 3 (bit-row r of column j comes from row
 * (r + d_v(c,j)) mod h); undo Eq. 2 (bit x of row r comes from bit
 * (x + d_h(c,r)) mod 8w). */
void vco_confuse_dec(const uint8_t *C, uint32_t w, uint32_t h,
                     const uint16_t *D, const uint8_t *B, uint8_t *P)
{
    const uint64_t W8 = 8ull * w;
    for (uint32_t r = 0; r < h; ++r)
        for (uint32_t q = 0; q < w; ++q)
            for (uint32_t c = 0; c < 3; ++c) {
                uint64_t dh = D[(uint64_t)c * h + r] % W8;
                uint64_t a = dh >> 3, t = dh & 7;
                uint64_t j1 = (q + a) % w, j2 = (j1 + 1) % w;
                uint64_t i1 = (r + D[3ull * h + (uint64_t)c * w + j1] % h) % h;
                uint64_t i2 = (r + D[3ull * h + (uint64_t)c * w + j2] % h) % h;
                uint32_t y1 = PIX(C, w, i1, j1, c) ^ PIX(B, w, i1, j1, c);
                uint32_t y2 = PIX(C, w, i2, j2, c) ^ PIX(B, w, i2, j2, c);
                PIX(P, w, r, q, c) = (uint8_t)(((y1 | (y2 << 8)) >> t) & 0xFF);
            }
}

/* Bit-matrix form.  Each channel c of a frame is the h x 8w bit matrix of
 * Alg. 3: entry (i, 8j + k) is bit k (least significant first) of byte
 * (i, j, c); Alg. 7 reads a byte back as the sum of its eight entries times
 * 2^k.  Eq. 2 and Eq. 3 are then permutations of whole matrices, written
 * here in gather form (each destination entry fetched through the inverse
 * index), one full matrix per stage, independent of the per-byte closed
 * form above.  One byte per bit: M[(c*h + i)*8w + x]. */
#define BIT(M, w, h, c, i, x) ((M)[((uint64_t)(c) * (h) + (i)) * (8ull * (w)) + (x)])

/* Alg. 3: the bit matrices of a frame. */
static void to_bits(const uint8_t *F, uint32_t w, uint32_t h, uint8_t *M)
{
    for (uint32_t c = 0; c < 3; ++c)
        for (uint32_t i = 0; i < h; ++i)
            for (uint64_t x = 0; x < 8ull * w; ++x)
                BIT(M, w, h, c, i, x) = (uint8_t)((PIX(F, w, i, x / 8, c) >> (x % 8)) & 1u);
}

/* Alg. 7: bytes from bit matrices. */
static void from_bits(const uint8_t *M, uint32_t w, uint32_t h, uint8_t *F)
{
    for (uint32_t c = 0; c < 3; ++c)
        for (uint32_t i = 0; i < h; ++i)
            for (uint32_t j = 0; j < w; ++j) {
                uint32_t sum = 0;
                for (uint32_t k = 0; k < 8; ++k) sum += (uint32_t)BIT(M, w, h, c, i, 8ull * j + k) << k;
                PIX(F, w, i, j, c) = (uint8_t)sum;
            }
}

/* Eq. 2 on every bit row r of channel c, by d_h(c, r): the entry at column
 * x moves to column (x + d_h) mod 8w, so destination column x holds source
 * column (x - d_h) mod 8w.  inverse != 0 applies the inverse permutation. */
static void rotate_rows(const uint8_t *src, uint8_t *dst, uint32_t w, uint32_t h, const uint16_t *D, int inverse)
{
    const uint64_t W8 = 8ull * w;
    for (uint32_t c = 0; c < 3; ++c)
        for (uint32_t r = 0; r < h; ++r) {
            const uint64_t d = D[(uint64_t)c * h + r] % W8;
            const uint64_t back = inverse ? d : W8 - d;   /* destination x reads source x + back */
            for (uint64_t x = 0; x < W8; ++x) BIT(dst, w, h, c, r, x) = BIT(src, w, h, c, r, (x + back) % W8);
        }
}

/* Eq. 3 on every bit column x of channel c, by d_v(c, x / 8) (one distance
 * per pixel column [R10]): the entry at row i moves to row (i + d_v) mod h. */
static void rotate_columns(const uint8_t *src, uint8_t *dst, uint32_t w, uint32_t h, const uint16_t *D, int inverse)
{
    const uint64_t W8 = 8ull * w;
    for (uint32_t c = 0; c < 3; ++c)
        for (uint64_t x = 0; x < W8; ++x) {
            const uint64_t d = D[3ull * h + (uint64_t)c * w + x / 8] % h;
            const uint64_t back = inverse ? d : h - d;
            for (uint32_t i = 0; i < h; ++i) BIT(dst, w, h, c, i, x) = BIT(src, w, h, c, (i + back) % h, x);
        }
}

/* Alg. 6: xor with the bit matrices of B, in place. */
static void xor_bits(uint8_t *M, uint32_t w, uint32_t h, const uint8_t *B, uint8_t *scratch)
{
    to_bits(B, w, h, scratch);
    for (uint64_t q = 0; q < 3ull * h * 8ull * w; ++q) M[q] ^= scratch[q];
}

/* Encryption on the bit matrices: Alg. 3, Eq. 2 (Alg. 4), Eq. 3 (Alg. 5),
 * Alg. 6, Alg. 7, read as a dataflow chain [R11]. */
int vco_confuse_enc_literal(const uint8_t *P, uint32_t w, uint32_t h,
                            const uint16_t *D, const uint8_t *B, uint8_t *C)
{
    const uint64_t cells = 3ull * h * 8ull * w;
    uint8_t *M0 = (uint8_t *)malloc(cells), *M1 = (uint8_t *)malloc(cells), *M2 = (uint8_t *)malloc(cells);
    if (!M0 || !M1 || !M2) { free(M0); free(M1); free(M2); return -1; }
    to_bits(P, w, h, M0);
    rotate_rows(M0, M1, w, h, D, 0);
    rotate_columns(M1, M2, w, h, D, 0);
    xor_bits(M2, w, h, B, M0);
    from_bits(M2, w, h, C);
    free(M0); free(M1); free(M2);
    return 0;
}

/* Decryption on the bit matrices: the same stages undone in reverse order. */
int vco_confuse_dec_literal(const uint8_t *C, uint32_t w, uint32_t h,
                            const uint16_t *D, const uint8_t *B, uint8_t *P)
{
    const uint64_t cells = 3ull * h * 8ull * w;
    uint8_t *M0 = (uint8_t *)malloc(cells), *M1 = (uint8_t *)malloc(cells), *M2 = (uint8_t *)malloc(cells);
    if (!M0 || !M1 || !M2) { free(M0); free(M1); free(M2); return -1; }
    to_bits(C, w, h, M2);
    xor_bits(M2, w, h, B, M0);
    rotate_columns(M2, M1, w, h, D, 1);
    rotate_rows(M1, M0, w, h, D, 1);
    from_bits(M0, w, h, P);
    free(M0); free(M1); free(M2);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Whole frames (Alg. 1)                                               */
/* ------------------------------------------------------------------ */

static int key_material(double base[4], double gamma, uint32_t n, uint32_t w,
                        uint32_t h, const uint8_t H[32], uint16_t **D, uint8_t **B)
{
    double ic[4];
    vco_reconstruct(base, H, ic);
    double *IR = (double *)malloc(sizeof(double) * 8 * (uint64_t)n);
    *D = (uint16_t *)malloc(sizeof(uint16_t) * (3ull * h + 3ull * w));
    *B = (uint8_t *)malloc(3ull * w * h);
    if (!IR || !*D || !*B) goto fail;
    if (vco_chain(ic, gamma, n, IR) != 0) goto fail;
    if (vco_keystream(IR, gamma, n, w, h, *D, *B) != 0) goto fail;
    memcpy(base, IR + 4 * (uint64_t)(2 * n - 1), 4 * sizeof(double));
    free(IR);
    return 0;
fail:
    free(IR); free(*D); free(*B);
    *D = NULL; *B = NULL;
    return -1;
}

int vco_encrypt_frame(double base[4], double gamma, uint32_t n,
                      const uint8_t *P, uint32_t w, uint32_t h,
                      uint8_t *C, uint8_t H[32])
{
    uint16_t *D; uint8_t *B;
    vco_frame_hash(P, 3ull * w * h, n, H);
    if (key_material(base, gamma, n, w, h, H, &D, &B) != 0) return -1;
    vco_confuse_enc(P, w, h, D, B, C);
    free(D); free(B);
    return 0;
}

int vco_decrypt_frame(double base[4], double gamma, uint32_t n,
                      const uint8_t *C, uint32_t w, uint32_t h,
                      const uint8_t H[32], uint8_t *P)
{
    uint16_t *D; uint8_t *B;
    if (key_material(base, gamma, n, w, h, H, &D, &B) != 0) return -1;
    vco_confuse_dec(C, w, h, D, B, P);
    free(D); free(B);
    return 0;
}

/* Threaded form: threads take sub-frames, then workers, then output rows,
 * round robin, as the paper's worker threads do (Algs. 1, 2). */
typedef struct {
    int phase; uint32_t tid, threads, n, w, h;
    const uint8_t *P; uint8_t (*hs)[32];
    const double *IR; double gamma; uint16_t *D; uint8_t *B; uint8_t *C;
    int rc;
} mt_job;

static void enc_rows(const uint8_t *P, uint32_t w, uint32_t h, const uint16_t *D,
                     const uint8_t *B, uint8_t *C, uint32_t i0, uint32_t step)
{
    const uint64_t W8 = 8ull * w;
    for (uint32_t i = i0; i < h; i += step)
        for (uint32_t j = 0; j < w; ++j)
            for (uint32_t c = 0; c < 3; ++c) {
                uint64_t dv = D[3ull * h + (uint64_t)c * w + j] % h;
                uint64_t r = (i + h - dv) % h;
                uint64_t dh = D[(uint64_t)c * h + r] % W8;
                uint64_t s = (8ull * j + W8 - dh) % W8;
                uint64_t q = s >> 3, t = s & 7, q2 = (q + 1) % w;
                uint32_t pair = PIX(P, w, r, q, c) | ((uint32_t)PIX(P, w, r, q2, c) << 8);
                PIX(C, w, i, j, c) = (uint8_t)((pair >> t) & 0xFF) ^ PIX(B, w, i, j, c);
            }
}

static void *mt_run(void *arg)
{
    mt_job *j = (mt_job *)arg;
    uint64_t L = 3ull * j->w * j->h;
    if (j->phase == 0) {
        for (uint32_t i = j->tid; i < j->n; i += j->threads) {
            uint64_t a = split_at(L, j->n, i), b = split_at(L, j->n, i + 1);
            vco_sha256(j->P + a, b - a, j->hs[i]);
        }
    } else if (j->phase == 1) {
        for (uint32_t i = j->tid; i < j->n; i += j->threads)
            if (keystream_worker(j->IR, j->gamma, j->n, j->w, j->h, i, j->D, j->B) != 0) j->rc = -1;
    } else {
        enc_rows(j->P, j->w, j->h, j->D, j->B, j->C, j->tid, j->threads);
    }
    return NULL;
}

static int mt_phase(mt_job *jobs, uint32_t threads, int phase)
{
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    if (!th) return -1;
    int rc = 0;
    for (uint32_t t = 0; t < threads; ++t) {
        jobs[t].phase = phase;
        if (pthread_create(&th[t], NULL, mt_run, &jobs[t]) != 0) { mt_run(&jobs[t]); th[t] = 0; }
    }
    for (uint32_t t = 0; t < threads; ++t) {
        if (th[t]) pthread_join(th[t], NULL);
        if (jobs[t].rc != 0) rc = -1;
    }
    free(th);
    return rc;
}

int vco_encrypt_frame_mt(double base[4], double gamma, uint32_t n,
                         const uint8_t *P, uint32_t w, uint32_t h,
                         uint8_t *C, uint8_t H[32], uint32_t threads)
{
    if (threads < 1) threads = 1;
    uint8_t (*hs)[32] = (uint8_t (*)[32])malloc(32ull * n);
    mt_job *jobs = (mt_job *)calloc(threads, sizeof(mt_job));
    double *IR = (double *)malloc(sizeof(double) * 8 * (uint64_t)n);
    uint16_t *D = (uint16_t *)malloc(sizeof(uint16_t) * (3ull * h + 3ull * w));
    uint8_t *B = (uint8_t *)malloc(3ull * w * h);
    int rc = -1;
    if (!hs || !jobs || !IR || !D || !B) goto done;
    for (uint32_t t = 0; t < threads; ++t) {
        mt_job *j = &jobs[t];
        j->tid = t; j->threads = threads; j->n = n; j->w = w; j->h = h;
        j->P = P; j->hs = hs; j->IR = IR; j->gamma = gamma; j->D = D; j->B = B; j->C = C;
    }
    if (mt_phase(jobs, threads, 0) != 0) goto done;
    memset(H, 0, 32);
    for (uint32_t i = 0; i < n; ++i)
        for (int k = 0; k < 32; ++k) H[k] ^= hs[i][k];
    double ic[4];
    vco_reconstruct(base, H, ic);
    if (vco_chain(ic, gamma, n, IR) != 0) goto done;
    if (mt_phase(jobs, threads, 1) != 0) goto done;
    if (mt_phase(jobs, threads, 2) != 0) goto done;
    memcpy(base, IR + 4 * (uint64_t)(2 * n - 1), 4 * sizeof(double));
    rc = 0;
done:
    free(hs); free(jobs); free(IR); free(D); free(B);
    return rc;
}
