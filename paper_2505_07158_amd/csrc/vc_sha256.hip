// vc_sha256.hip -- frame hash H = SHA-256(f_1) xor ... xor SHA-256(f_n)
// (Sec. II-A of arXiv 2505.07158; Alg. 1 partition + combine, Alg. 2 hash).
//
// One lane per sub-frame: SHA-256 is a serial chain of 64-byte compressions,
// so n (part of the key) fixes the parallelism of one frame; frames of a
// batch run side by side.  Sub-frame i of a frame of L bytes is the byte
// range [floor(i*L/n), floor((i+1)*L/n)).  A workgroup holds whole frames
// (several when n is small), xor-reduces their digests in LDS and writes H in
// FIPS 180-4 digest byte order.
//
// SHA-256 follows FIPS 180-4 (sec. 4.1.2 functions, 4.2.2 constants, 5.1.1
// padding, 6.2.2 compression).  The round constants are generated at compile
// time from their definition (fractional parts of cube / square roots of the
// first primes) by exact integer root extraction.
#include <utility>

#include "vc_internal.hpp"

namespace vc {
namespace {

constexpr bool is_prime(uint32_t c) {
    if (c < 2) return false;
    for (uint32_t d = 2; d * d <= c; ++d)
        if (c % d == 0) return false;
    return true;
}

// floor(p^(1/k) * 2^32) for k = 2 or 3, by bisection on exact integers.
constexpr uint64_t root_scaled(uint32_t p, int k) {
    const unsigned __int128 target = static_cast<unsigned __int128>(p) << (32 * k);
    uint64_t lo = 0, hi = uint64_t(1) << 40;
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        unsigned __int128 m = mid, pw = m * m;
        if (k == 3) pw *= m;
        if (pw <= target) lo = mid; else hi = mid;
    }
    return lo;
}

struct ShaConstants {
    uint32_t K[64];
    uint32_t H0[8];
};

constexpr ShaConstants make_sha_constants() {
    ShaConstants s{};
    int found = 0;
    for (uint32_t c = 2; found < 64; ++c) {
        if (!is_prime(c)) continue;
        s.K[found] = static_cast<uint32_t>(root_scaled(c, 3));
        if (found < 8) s.H0[found] = static_cast<uint32_t>(root_scaled(c, 2));
        ++found;
    }
    return s;
}

constexpr ShaConstants kSha = make_sha_constants();

// gfx950 v_bitop3_b32 evaluates any 3-input bitwise function given by its
// truth table: bit (4a + 2b + c) of the immediate is f(a, b, c).
constexpr uint32_t kXor3 = 0x96;  // a ^ b ^ c
constexpr uint32_t kCh = 0xCA;    // (a & b) ^ (~a & c)
constexpr uint32_t kMaj = 0xE8;   // (a & b) ^ (a & c) ^ (b & c)

__device__ __forceinline__ uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, kXor3);
}
// FIPS 180-4 sec. 4.1.2, functions (4.2)-(4.7).
__device__ __forceinline__ uint32_t bsig0(uint32_t x) { return xor3(rotr(x, 2), rotr(x, 13), rotr(x, 22)); }
__device__ __forceinline__ uint32_t bsig1(uint32_t x) { return xor3(rotr(x, 6), rotr(x, 11), rotr(x, 25)); }
__device__ __forceinline__ uint32_t ssig0(uint32_t x) { return xor3(rotr(x, 7), rotr(x, 18), x >> 3); }
__device__ __forceinline__ uint32_t ssig1(uint32_t x) { return xor3(rotr(x, 17), rotr(x, 19), x >> 10); }
__device__ __forceinline__ uint32_t ch(uint32_t x, uint32_t y, uint32_t z) {
    return __builtin_amdgcn_bitop3_b32(x, y, z, kCh);
}
__device__ __forceinline__ uint32_t maj(uint32_t x, uint32_t y, uint32_t z) {
    return __builtin_amdgcn_bitop3_b32(x, y, z, kMaj);
}

// Round t with the working variables kept in place: at round t, variable
// a lives in v[(0 - t) & 7], b in v[(1 - t) & 7], ..., h in v[(7 - t) & 7],
// so the a..h renaming of FIPS 180-4 sec. 6.2.2 costs no register moves.
// The 16-word ring W[t & 15] holds the message schedule.
template <int t>
__device__ __forceinline__ void sha_round(uint32_t (&v)[8], uint32_t (&W)[16]) {
    constexpr uint32_t K = kSha.K[t];
    if constexpr (t >= 16) {
        W[t & 15] = ssig1(W[(t - 2) & 15]) + W[(t - 7) & 15] + ssig0(W[(t - 15) & 15]) + W[t & 15];
    }
    const uint32_t a = v[(0 - t) & 7], b = v[(1 - t) & 7], c = v[(2 - t) & 7];
    const uint32_t d = v[(3 - t) & 7], e = v[(4 - t) & 7], f = v[(5 - t) & 7];
    const uint32_t g = v[(6 - t) & 7], h = v[(7 - t) & 7];
    const uint32_t T1 = h + bsig1(e) + ch(e, f, g) + K + W[t & 15];
    const uint32_t T2 = bsig0(a) + maj(a, b, c);
    v[(3 - t) & 7] = d + T1;   // becomes e
    v[(7 - t) & 7] = T1 + T2;  // becomes a
}

template <int... t>
__device__ __forceinline__ void sha_rounds(uint32_t (&v)[8], uint32_t (&W)[16],
                                           std::integer_sequence<int, t...>) {
    (sha_round<t>(v, W), ...);
}

__device__ __forceinline__ void sha_compress(uint32_t (&H)[8], uint32_t (&W)[16]) {
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = H[k];
    sha_rounds(v, W, std::make_integer_sequence<int, 64>{});
    // after 64 rounds (a multiple of 8) the variables are back in place
#pragma unroll
    for (int k = 0; k < 8; ++k) H[k] += v[k];
}

__device__ __forceinline__ uint32_t bswap32(uint32_t x) { return __builtin_bswap32(x); }

// Big-endian word m of a 64-byte block read byte by byte (bounded paths).
__device__ __forceinline__ uint32_t load_be_bytes(const VC_GLOBAL uint8_t *p) {
    return (uint32_t(p[0]) << 24) | (uint32_t(p[1]) << 16) | (uint32_t(p[2]) << 8) | uint32_t(p[3]);
}

// Four-byte-aligned 16-byte vector (global_load_dwordx4 needs only dword
// alignment).
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

// 17 consecutive dwords from a dword-aligned address.
__device__ __forceinline__ void load_window(const VC_GLOBAL uint32_t *p, uint32_t (&w)[17]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const u32x4_a4 v = *reinterpret_cast<const VC_GLOBAL u32x4_a4 *>(p + 4 * q);
        w[4 * q] = v.x; w[4 * q + 1] = v.y; w[4 * q + 2] = v.z; w[4 * q + 3] = v.w;
    }
    w[16] = p[16];
}

// SHA-256 of bytes [a, b) of a frame of L bytes at `frame`.
__device__ void sha256_range(const VC_GLOBAL uint8_t *frame, uint64_t a, uint64_t b, uint64_t L,
                             uint32_t (&H)[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) H[k] = kSha.H0[k];
    const uint64_t len = b - a;
    const uint64_t nfull = len / 64;

    // Fast blocks: 17 dwords from the dword-aligned address at or below the
    // block start, shifted into place with alignbyte.  Block k reads bytes
    // [base + 64k, base + 64k + 68), which must end inside the frame.
    const uintptr_t start = reinterpret_cast<uintptr_t>(frame + a);
    const uint32_t sh = static_cast<uint32_t>(start & 3);
    const uintptr_t base = start - sh;
    const uintptr_t end = reinterpret_cast<uintptr_t>(frame + L);
    uint64_t nfast = 0;
    if (end >= base + 68) {
        nfast = (end - base - 68) / 64 + 1;
        if (nfast > nfull) nfast = nfull;
    }
    const VC_GLOBAL uint32_t *wp = reinterpret_cast<const VC_GLOBAL uint32_t *>(base);
    uint32_t W[16];
    if (nfast > 0) {
        uint32_t cur[17];
        load_window(wp, cur);
        for (uint64_t k = 0; k < nfast; ++k) {
            // prefetch the next block (clamped so the address stays valid)
            const uint64_t kn = (k + 1 < nfast) ? k + 1 : k;
            uint32_t nxt[17];
            load_window(wp + 16 * kn, nxt);
#pragma unroll
            for (int m = 0; m < 16; ++m) W[m] = bswap32(__builtin_amdgcn_alignbyte(cur[m + 1], cur[m], sh));
            sha_compress(H, W);
#pragma unroll
            for (int m = 0; m < 17; ++m) cur[m] = nxt[m];
        }
    }
    // Remaining full blocks, byte by byte.
    for (uint64_t k = nfast; k < nfull; ++k) {
        const VC_GLOBAL uint8_t *p = frame + a + 64 * k;
#pragma unroll
        for (int m = 0; m < 16; ++m) W[m] = load_be_bytes(p + 4 * m);
        sha_compress(H, W);
    }
    // Padding (FIPS 180-4 sec. 5.1.1): tail bytes, 0x80, zeros, 64-bit
    // big-endian bit length; one or two blocks.
    const uint32_t rem = static_cast<uint32_t>(len - 64 * nfull);
    const VC_GLOBAL uint8_t *p = frame + a + 64 * nfull;
    const uint64_t bits = len * 8;
    const int blocks = (rem + 9 <= 64) ? 1 : 2;
    for (int blk = 0; blk < blocks; ++blk) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            uint32_t word = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t j = 64 * blk + 4 * m + q;
                uint32_t byte = 0;
                if (j < rem) byte = p[j];
                else if (j == rem) byte = 0x80;
                word = (word << 8) | byte;
            }
            W[m] = word;
        }
        if (blk == blocks - 1) {
            W[14] = static_cast<uint32_t>(bits >> 32);
            W[15] = static_cast<uint32_t>(bits);
        }
        sha_compress(H, W);
    }
}

// ----------------------------------------------------------------------
// Two-wave form (n <= 64): the message schedule does not depend on the
// compression state, so one wave (the schedule wave) loads each block,
// expands W and writes K[t] + W[t] to LDS while the other wave (the
// compression wave) runs the 64 rounds of the previous block.  Lane l of
// both waves serves the same sub-frame.  Double-buffered, one barrier per
// block.
// ----------------------------------------------------------------------
constexpr int kKwStride = 68;  // words per lane and buffer (64 + 4: 16-byte rows, no bank aliasing)

// Message words of block k of the padded sub-frame [a, b) of a frame of L
// bytes (FIPS 180-4 sec. 5.1.1), for any k < blocks.
struct SubFrame {
    const VC_GLOBAL uint8_t *frame;
    uint64_t a, len, L;
    uint64_t nfull, nfast;
    uint32_t sh;
    const VC_GLOBAL uint32_t *wp;
    uint32_t blocks;
};

__device__ __forceinline__ SubFrame make_subframe(const VC_GLOBAL uint8_t *frame, uint64_t a, uint64_t b,
                                                  uint64_t L) {
    SubFrame f;
    f.frame = frame;
    f.a = a;
    f.len = b - a;
    f.L = L;
    f.nfull = f.len / 64;
    const uintptr_t start = reinterpret_cast<uintptr_t>(frame + a);
    f.sh = static_cast<uint32_t>(start & 3);
    const uintptr_t base = start - f.sh;
    const uintptr_t end = reinterpret_cast<uintptr_t>(frame + L);
    f.nfast = 0;
    if (end >= base + 68) {
        f.nfast = (end - base - 68) / 64 + 1;
        if (f.nfast > f.nfull) f.nfast = f.nfull;
    }
    f.wp = reinterpret_cast<const VC_GLOBAL uint32_t *>(base);
    const uint32_t rem = static_cast<uint32_t>(f.len - 64 * f.nfull);
    f.blocks = static_cast<uint32_t>(f.nfull) + ((rem + 9 <= 64) ? 1 : 2);
    return f;
}

__device__ __forceinline__ void block_words(const SubFrame &f, uint64_t k, uint32_t (&W)[16]) {
    if (k < f.nfast) {
        uint32_t cur[17];
        load_window(f.wp + 16 * k, cur);
#pragma unroll
        for (int m = 0; m < 16; ++m) W[m] = bswap32(__builtin_amdgcn_alignbyte(cur[m + 1], cur[m], f.sh));
    } else if (k < f.nfull) {
        const VC_GLOBAL uint8_t *p = f.frame + f.a + 64 * k;
#pragma unroll
        for (int m = 0; m < 16; ++m) W[m] = load_be_bytes(p + 4 * m);
    } else {
        const uint32_t rem = static_cast<uint32_t>(f.len - 64 * f.nfull);
        const VC_GLOBAL uint8_t *p = f.frame + f.a + 64 * f.nfull;
        const uint32_t blk = static_cast<uint32_t>(k - f.nfull);
        const int last = (rem + 9 <= 64) ? 0 : 1;
        for (int m = 0; m < 16; ++m) {
            uint32_t word = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t j = 64 * blk + 4 * m + q;
                uint32_t byte = 0;
                if (j < rem) byte = p[j];
                else if (j == rem) byte = 0x80;
                word = (word << 8) | byte;
            }
            W[m] = word;
        }
        if (static_cast<int>(blk) == last) {
            const uint64_t bits = f.len * 8;
            W[14] = static_cast<uint32_t>(bits >> 32);
            W[15] = static_cast<uint32_t>(bits);
        }
    }
}

// Schedule wave: W[0..63] of one block, plus K, into the lane's LDS row.
template <int t>
__device__ __forceinline__ void sched_step(uint32_t (&W)[16], uint32_t (&kw)[64]) {
    if constexpr (t >= 16)
        W[t & 15] = ssig1(W[(t - 2) & 15]) + W[(t - 7) & 15] + ssig0(W[(t - 15) & 15]) + W[t & 15];
    kw[t] = W[t & 15] + kSha.K[t];
}
template <int... t>
__device__ __forceinline__ void sched_all(uint32_t (&W)[16], uint32_t (&kw)[64], std::integer_sequence<int, t...>) {
    (sched_step<t>(W, kw), ...);
}

// Compression wave: round t with K[t] + W[t] precomputed.
template <int t>
__device__ __forceinline__ void round_kw(uint32_t (&v)[8], const uint32_t (&kw)[64]) {
    const uint32_t a = v[(0 - t) & 7], b = v[(1 - t) & 7], c = v[(2 - t) & 7];
    const uint32_t d = v[(3 - t) & 7], e = v[(4 - t) & 7], f = v[(5 - t) & 7];
    const uint32_t g = v[(6 - t) & 7], h = v[(7 - t) & 7];
    const uint32_t T1 = h + bsig1(e) + ch(e, f, g) + kw[t];
    const uint32_t T2 = bsig0(a) + maj(a, b, c);
    v[(3 - t) & 7] = d + T1;
    v[(7 - t) & 7] = T1 + T2;
}
template <int... t>
__device__ __forceinline__ void rounds_kw(uint32_t (&v)[8], const uint32_t (&kw)[64], std::integer_sequence<int, t...>) {
    (round_kw<t>(v, kw), ...);
}

typedef uint32_t u32x4_lds __attribute__((ext_vector_type(4)));

// 128 threads: wave 0 schedules, wave 1 compresses; 64/n frames per group.
__global__ __launch_bounds__(128) void sha256_subframes_2w(const FrameDesc *__restrict__ desc, uint32_t count,
                                                           uint32_t n, uint32_t frames_per_group) {
    __shared__ __align__(16) uint32_t kwbuf[2][64][kKwStride];
    __shared__ uint32_t dig[64][9];
    __builtin_amdgcn_s_setprio(2);  // latency-bound: ahead of the bandwidth-bound confusion waves
    claim_half_simd();
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t lf = lane / n, sub = lane % n;
    const uint32_t f = blockIdx.x * frames_per_group + lf;
    const bool active = lf < frames_per_group && f < count;
    SubFrame sf{};
    uint32_t blocks = 0;
    if (active) {
        const FrameDesc d = desc[f];
        const uint64_t a = (d.L * sub) / n, b = (d.L * (sub + 1)) / n;
        sf = make_subframe(gmem(d.in), a, b, d.L);
        blocks = sf.blocks;
    }
    // every wave of the group runs the same number of iterations
    uint32_t nb = blocks;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nb = max(nb, static_cast<uint32_t>(__shfl_xor(static_cast<int>(nb), o)));

    if (wave == 0) {
        uint32_t W[16], kw[64];
        auto produce = [&](uint32_t k, int buf) {
            if (k < blocks) {
                block_words(sf, k, W);
                sched_all(W, kw, std::make_integer_sequence<int, 64>{});
                u32x4_lds *row = reinterpret_cast<u32x4_lds *>(&kwbuf[buf][lane][0]);
#pragma unroll
                for (int q = 0; q < 16; ++q) row[q] = u32x4_lds{kw[4 * q], kw[4 * q + 1], kw[4 * q + 2], kw[4 * q + 3]};
            }
        };
        produce(0, 0);
        __syncthreads();
        for (uint32_t k = 0; k < nb; ++k) {
            if (k + 1 < nb) produce(k + 1, (k + 1) & 1);
            __syncthreads();
        }
        __syncthreads();  // matches the digest barrier of the compression wave
    } else {
        uint32_t H[8], kw[64];
#pragma unroll
        for (int m = 0; m < 8; ++m) H[m] = kSha.H0[m];
        __syncthreads();
        for (uint32_t k = 0; k < nb; ++k) {
            if (k < blocks) {
                const u32x4_lds *row = reinterpret_cast<const u32x4_lds *>(&kwbuf[k & 1][lane][0]);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const u32x4_lds x = row[q];
                    kw[4 * q] = x.x; kw[4 * q + 1] = x.y; kw[4 * q + 2] = x.z; kw[4 * q + 3] = x.w;
                }
                uint32_t v[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) v[m] = H[m];
                rounds_kw(v, kw, std::make_integer_sequence<int, 64>{});
#pragma unroll
                for (int m = 0; m < 8; ++m) H[m] += v[m];
            }
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) dig[lane][m] = active ? H[m] : 0u;
        __syncthreads();
        // lane t < frames_per_group*8: word t%8 of local frame t/8
        for (uint32_t t = lane; t < frames_per_group * 8; t += 64) {
            const uint32_t lf2 = t / 8, word = t % 8;
            const uint32_t f2 = blockIdx.x * frames_per_group + lf2;
            if (f2 >= count) break;
            uint32_t x = 0;
            for (uint32_t i = 0; i < n; ++i) x ^= dig[lf2 * n + i][word];
            VC_GLOBAL uint8_t *out = gmem(desc[f2].hash) + 4 * word;
            out[0] = uint8_t(x >> 24);
            out[1] = uint8_t(x >> 16);
            out[2] = uint8_t(x >> 8);
            out[3] = uint8_t(x);
        }
    }
}

constexpr int kShaMaxThreads = 1024;

// Threads: blockDim.x lanes; frames_per_group frames of n lanes each.
__global__ __launch_bounds__(kShaMaxThreads) void sha256_subframes(const FrameDesc *__restrict__ desc,
                                                                   uint32_t count, uint32_t n,
                                                                   uint32_t frames_per_group) {
    extern __shared__ uint32_t dig_raw[];  // blockDim.x x 9 words (9: no bank conflicts)
    uint32_t (*dig)[9] = reinterpret_cast<uint32_t (*)[9]>(dig_raw);
    __builtin_amdgcn_s_setprio(2);
    const uint32_t tid = threadIdx.x;
    const uint32_t lf = tid / n, sub = tid % n;
    const uint32_t f = blockIdx.x * frames_per_group + lf;
    uint32_t H[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) H[k] = 0;
    if (lf < frames_per_group && f < count) {
        const FrameDesc d = desc[f];
        const uint64_t a = (d.L * sub) / n, b = (d.L * (sub + 1)) / n;
        sha256_range(gmem(d.in), a, b, d.L, H);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) dig[tid][k] = H[k];
    __syncthreads();
    // item t: word t%8 of local frame t/8
    for (uint32_t t = tid; t < frames_per_group * 8; t += blockDim.x) {
        const uint32_t lf2 = t / 8, word = t % 8;
        const uint32_t f2 = blockIdx.x * frames_per_group + lf2;
        if (f2 >= count) break;
        uint32_t x = 0;
        for (uint32_t i = 0; i < n; ++i) x ^= dig[lf2 * n + i][word];
        VC_GLOBAL uint8_t *out = gmem(desc[f2].hash) + 4 * word;
        out[0] = uint8_t(x >> 24);
        out[1] = uint8_t(x >> 16);
        out[2] = uint8_t(x >> 8);
        out[3] = uint8_t(x);
    }
}

}  // namespace

hipError_t launch_sha256_subframes(const FrameDesc *d_desc, uint32_t count, uint32_t n,
                                   hipStream_t s) {
    if (count == 0) return hipSuccess;
    // n <= 64: a pair of waves (schedule + compression) holds 64/n frames.
    // Otherwise one frame per workgroup, one wave per 64 sub-frames.
    uint32_t threads, fpg;
    if (n <= 64) {
        fpg = 64 / n;
        const uint32_t groups = (count + fpg - 1) / fpg;
        hipLaunchKernelGGL(sha256_subframes_2w, dim3(groups), dim3(128), 0, s, d_desc, count, n, fpg);
        return hipGetLastError();
    } else {
        fpg = 1;
        threads = ((n + 63) / 64) * 64;
    }
    const uint32_t groups = (count + fpg - 1) / fpg;
    hipLaunchKernelGGL(sha256_subframes, dim3(groups), dim3(threads), threads * 9 * sizeof(uint32_t), s,
                       d_desc, count, n, fpg);
    return hipGetLastError();
}

}  // namespace vc
