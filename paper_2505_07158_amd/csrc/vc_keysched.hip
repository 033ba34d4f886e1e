// vc_keysched.hip -- the chaotic key schedule of arXiv 2505.07158 on gfx950:
//   lhcs_chain : IC reconstruction from the chain state and H, then 2n RK4
//                iterations of LHCS_m (Sec. II-A, Alg. 1).  Serial per stream
//                (frame t+1 starts from x_2n..w_2n of frame t), so one wave
//                walks one stream's frames; its other lanes only fetch the
//                hashes and record pointers of the next 64 frames, so the
//                walk itself never waits on memory.
//   lhcs_keygen: the n workers of Alg. 2: two LHCS_w seeded from IR,
//                iterated in lock step; the xor of their FP64 bit patterns
//                gives six mantissa bytes per variable per step (Sec. II-B),
//                cut into shift distances D and bytes B.
//
// Bit-exact agreement with any IEEE-754 FP64 implementation of the same
// steps: only +, -, *, / (correctly rounded, round-to-nearest-even), floor
// and exact bit manipulation are used, in a fixed order, and the library is
// built with -ffp-contract=off (plus the pragma below) so that no product is
// fused into an FMA.
#include "vc_internal.hpp"

#pragma clang fp contract(off)

namespace vc {
namespace {

// Eq. 1 constants and the integrator step (protocol v1: classical RK4, 0.01).
constexpr double kSigma = 10.0;
constexpr double kRho = 28.0;
constexpr double kBeta = 8.0 / 3.0;
constexpr double kStep = 0.01;
constexpr double kHalfStep = kStep * 0.5;
constexpr double kSixthStep = kStep / 6.0;
constexpr double kTwo52 = 4503599627370496.0;        // 2^52
constexpr double kTwoM52 = 1.0 / 4503599627370496.0;  // 2^-52
constexpr uint32_t kReconU = 32;                      // upper bound u of the integer part

struct V4 {
    double x, y, z, w;
};

__device__ __forceinline__ V4 lhcs_rhs(const V4 &s, double gamma) {
    V4 d;
    d.x = kSigma * (s.y - s.x) + s.w;
    d.y = (kRho * s.x - s.y) - s.x * s.z;
    d.z = s.x * s.y - kBeta * s.z;
    d.w = gamma * s.w - s.y * s.z;
    return d;
}

__device__ __forceinline__ V4 axpy(const V4 &s, double a, const V4 &k) {
    return V4{s.x + a * k.x, s.y + a * k.y, s.z + a * k.z, s.w + a * k.w};
}

// s + h/6 * (((k1 + 2 k2) + 2 k3) + k4).  Doubling is exact, so
// fma(2, k, a) rounds the same exact sum 2k + a once, exactly as a + 2k
// does after the exact product: bit-identical to the unfused expression as
// long as 2k does not overflow (|k| < 2^1023, far outside the attractor).
__device__ __forceinline__ double rk4_comb(double s, double k1, double k2, double k3, double k4) {
    return s + kSixthStep * (__builtin_fma(2.0, k3, __builtin_fma(2.0, k2, k1)) + k4);
}

// One classical RK4 step.  (A non-finite state stays non-finite under
// these operations, so callers check finiteness once, at the end.)
__device__ __forceinline__ void rk4_step(V4 &s, double gamma) {
    const V4 k1 = lhcs_rhs(s, gamma);
    const V4 k2 = lhcs_rhs(axpy(s, kHalfStep, k1), gamma);
    const V4 k3 = lhcs_rhs(axpy(s, kHalfStep, k2), gamma);
    const V4 k4 = lhcs_rhs(axpy(s, kStep, k3), gamma);
    s.x = rk4_comb(s.x, k1.x, k2.x, k3.x, k4.x);
    s.y = rk4_comb(s.y, k1.y, k2.y, k3.y, k4.y);
    s.z = rk4_comb(s.z, k1.z, k2.z, k3.z, k4.z);
    s.w = rk4_comb(s.w, k1.w, k2.w, k3.w, k4.w);
}

// Integer-valued x in [0, 2^52) -> uint64, exactly (x + 2^52 has x as its
// mantissa).
__device__ __forceinline__ uint64_t exact_u52(double x) {
    return static_cast<uint64_t>(__double_as_longlong(x + kTwo52)) & ((uint64_t(1) << 52) - 1);
}
// uint64 below 2^52 -> double, exactly.
__device__ __forceinline__ double exact_f52(uint64_t v) {
    return __longlong_as_double(static_cast<long long>(0x4330000000000000ull | v)) - kTwo52;
}

// Reconstruction of one variable (Sec. II-A, Fig. 1a as described in the
// text): the two low bytes of the integer part of |v| xor two hash bytes,
// reduced mod u; the six low bytes of the 52-bit fraction of |v| xor six
// hash bytes; recombined with the sign of v.  hw0, hw1 are H[8k..8k+3] and
// H[8k+4..8k+7] as little-endian words.
__device__ __forceinline__ double reconstruct1(double v, uint32_t hw0, uint32_t hw1) {
    const double a = __builtin_fabs(v);
    const double ip = __builtin_floor(a);
    const double low16 = ip - 65536.0 * __builtin_floor(ip / 65536.0);
    const uint64_t I = exact_u52(low16);
    const uint64_t G = exact_u52(__builtin_floor((a - ip) * kTwo52));
    // H[8k..8k+7] as one big-endian number: its top 16 bits, then 48 bits
    const uint64_t be = (static_cast<uint64_t>(__builtin_bswap32(hw0)) << 32) | __builtin_bswap32(hw1);
    const uint64_t h16 = be >> 48;
    const uint64_t h48 = be & ((uint64_t(1) << 48) - 1);
    const uint64_t I2 = (I ^ h16) % kReconU;
    const uint64_t G2 = G ^ h48;
    const double r = static_cast<double>(static_cast<uint32_t>(I2)) + exact_f52(G2) * kTwoM52;
    return (__double_as_longlong(v) < 0) ? -r : r;
}

typedef uint32_t u32x4_a16 __attribute__((ext_vector_type(4), aligned(16)));

// The 32 bytes at p as eight little-endian words.
__device__ __forceinline__ void load_hash_words(const uint8_t *p, uint32_t (&w)[8]) {
    const VC_GLOBAL uint8_t *g = gmem(p);
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
        const u32x4_a16 a = reinterpret_cast<const VC_GLOBAL u32x4_a16 *>(g)[0];
        const u32x4_a16 b = reinterpret_cast<const VC_GLOBAL u32x4_a16 *>(g)[1];
        w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
        w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            w[k] = uint32_t(g[4 * k]) | (uint32_t(g[4 * k + 1]) << 8) | (uint32_t(g[4 * k + 2]) << 16) |
                   (uint32_t(g[4 * k + 3]) << 24);
    }
}

__device__ __forceinline__ uint32_t lane_u32(uint32_t v, uint32_t lane) {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), static_cast<int>(lane)));
}

// One wave per stream run.  Frames are taken in blocks of 64: lane j loads
// the record and hash of frame (block + j); lane 0 then walks the block,
// reading each frame's words from the loading lane with v_readlane, so the
// serial FP64 walk (raised to the top issue priority of its SIMD, since the
// rest of the path waits on it) has no memory wait inside a block.
__global__ __launch_bounds__(64) void lhcs_chain(const StreamRun *__restrict__ runs,
                                                 const ChainRec *__restrict__ recs, double *__restrict__ state,
                                                 uint32_t n, double gamma, int *__restrict__ flags) {
    __builtin_amdgcn_s_setprio(3);
    const StreamRun run = runs[blockIdx.x];
    const uint32_t lane = threadIdx.x;
    double *st = state + 4 * static_cast<uint64_t>(run.slot);
    V4 base{st[0], st[1], st[2], st[3]};
    bool ok = true;
    for (uint32_t blk = 0; blk < run.count; blk += 64) {
        const uint32_t nb = (run.count - blk < 64) ? run.count - blk : 64;
        uint32_t H[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        uint64_t irp = 0;
        if (lane < nb) {
            const ChainRec rec = recs[run.first + blk + lane];
            load_hash_words(rec.hash, H);
            irp = reinterpret_cast<uintptr_t>(rec.IR);
        }
        if (lane == 0) {
            for (uint32_t u = 0; u < nb; ++u) {
                uint32_t hw[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) hw[k] = lane_u32(H[k], u);
                const uint64_t ira = (static_cast<uint64_t>(lane_u32(static_cast<uint32_t>(irp >> 32), u)) << 32) |
                                     lane_u32(static_cast<uint32_t>(irp), u);
                V4 s{reconstruct1(base.x, hw[0], hw[1]), reconstruct1(base.y, hw[2], hw[3]),
                     reconstruct1(base.z, hw[4], hw[5]), reconstruct1(base.w, hw[6], hw[7])};
                VC_GLOBAL double *ir = gmem(reinterpret_cast<double *>(ira));
                for (uint32_t m = 0; m < 2 * n; ++m) {
                    rk4_step(s, gamma);
                    ir[4 * m + 0] = s.x;
                    ir[4 * m + 1] = s.y;
                    ir[4 * m + 2] = s.z;
                    ir[4 * m + 3] = s.w;
                }
                ok &= __builtin_isfinite(s.x) && __builtin_isfinite(s.y) && __builtin_isfinite(s.z) &&
                      __builtin_isfinite(s.w);
                base = s;
            }
        }
    }
    if (lane == 0) {
        st[0] = base.x;
        st[1] = base.y;
        st[2] = base.z;
        st[3] = base.w;
        if (!ok) flags[0] = FLAG_NONFINITE;
    }
}

__device__ __forceinline__ uint64_t bits(double v) { return static_cast<uint64_t>(__double_as_longlong(v)); }

__device__ __forceinline__ bool finite4(const V4 &s) {
    return __builtin_isfinite(s.x) && __builtin_isfinite(s.y) && __builtin_isfinite(s.z) &&
           __builtin_isfinite(s.w);
}

typedef uint32_t u32x3_a4 __attribute__((ext_vector_type(3), aligned(4)));

// Worker i of frame f owns distances [floor(i*ND/n), floor((i+1)*ND/n)) and
// bytes [floor(i*L/n), floor((i+1)*L/n)); its byte stream gives its
// distances first (little-endian pairs) and then its bytes.  Seeds:
// A = IR_{2i+1}, Q = IR_{2i+2}; LHCS^1 = (A.x, Q.y, A.z, Q.w), LHCS^2 =
// (Q.x, A.y, Q.z, A.w).  Each step emits, for x, y, z, w in turn, the six
// low mantissa bytes of the xor of the two bit patterns, least significant
// first.
//
// A workgroup is two waves serving the same 32 workers.  Wave 0 integrates:
// lane 2p iterates LHCS^1 and lane 2p+1 LHCS^2 of worker p, writing each
// step's state to an LDS ring.  Wave 1 turns the ring into bytes: lane 2p
// stores the first twelve bytes of each step (x, y), lane 2p+1 the last
// twelve (z, w).  The ring holds kKgRing steps and is handed over in halves
// with one barrier per half, so the integrating wave -- the serial part --
// issues almost nothing but its FP64 arithmetic while the byte work runs on
// another SIMD.
//
// Stores: steps whose 24 bytes lie inside the keystream region are written
// as six dwords at dword-aligned addresses; the dword straddling the
// previous step takes that step's last bytes from a carry register.  The
// distance bytes, and the few steps at either end of the region, are
// stored byte by byte.
constexpr uint32_t kKgRing = 8;
constexpr uint32_t kKgHalf = kKgRing / 2;

__global__ __launch_bounds__(128) void lhcs_keygen(const FrameDesc *__restrict__ desc, uint32_t count,
                                                   uint32_t n, double gamma, int *__restrict__ flags) {
    __shared__ __align__(16) V4 ring[kKgRing][64];
    __builtin_amdgcn_s_setprio(2);  // latency-bound: ahead of the bandwidth-bound confusion waves
    claim_half_simd();
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t g = static_cast<uint64_t>(blockIdx.x) * 64 + lane;  // same worker lanes in both waves
    const uint64_t worker = g >> 1;
    const uint32_t odd = lane & 1;
    const uint64_t f = worker / n;
    const uint32_t i = static_cast<uint32_t>(worker % n);
    const bool live = f < count;
    FrameDesc d{};
    uint64_t d0 = 0, d1 = 0, b0 = 0, b1 = 0;
    if (live) {
        d = desc[f];
        const uint64_t ND = 3ull * d.h + 3ull * d.w;
        d0 = ND * i / n;
        d1 = ND * (i + 1) / n;
        b0 = d.L * i / n;
        b1 = d.L * (i + 1) / n;
    }
    const uint64_t two_nd = 2 * (d1 - d0);
    const uint64_t total = two_nd + (b1 - b0);
    const uint64_t steps = (total + 23) / 24;
    // Both waves run the same number of ring halves: enough for the
    // longest worker of the wave.
    uint32_t smax = static_cast<uint32_t>(steps);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t other = static_cast<uint32_t>(__shfl_xor(static_cast<int>(smax), o));
        smax = other > smax ? other : smax;
    }
    const uint32_t nblk = (smax + kKgHalf - 1) / kKgHalf;

    if (wave == 0) {
        V4 l{0.0, 0.0, 0.0, 0.0};
        if (live) {
            const VC_GLOBAL double *A = gmem(d.IR) + 8 * static_cast<uint64_t>(i);
            const VC_GLOBAL double *Q = A + 4;
            l = odd ? V4{Q[0], A[1], Q[2], A[3]} : V4{A[0], Q[1], A[2], Q[3]};
        }
        for (uint32_t blk = 0; blk < nblk; ++blk) {
            V4 *slot = &ring[(blk & 1) * kKgHalf][lane];
#pragma unroll
            for (uint32_t j = 0; j < kKgHalf; ++j) {
                rk4_step(l, gamma);
                slot[64 * j] = l;
            }
            __syncthreads();
        }
        return;
    }

    VC_GLOBAL uint8_t *Dbytes = live ? reinterpret_cast<VC_GLOBAL uint8_t *>(gmem(d.D) + d0) : nullptr;
    VC_GLOBAL uint8_t *Bw = live ? gmem(d.B) + b0 : nullptr;
    // Fast steps s in [s_a, s_b): dwords cover stream bytes
    // [24s - phi, 24s + 24 - phi), all inside [two_nd, total).
    const uint32_t phi = static_cast<uint32_t>((reinterpret_cast<uintptr_t>(d.B + b0) - two_nd) & 3);
    const uint64_t s_a = (two_nd + phi + 23) / 24;
    const uint64_t s_b = (total + phi >= 24) ? (total + phi - 24) / 24 + 1 : 0;
    const uint64_t fast_lo = (s_a < s_b) ? s_a : steps;  // no fast steps: fast_lo = fast_hi = steps
    const uint64_t fast_hi = (s_a < s_b) ? s_b : steps;
    const uint32_t shr = 8 * (4 - phi);  // 32 when phi == 0
    const uint32_t jlo = odd ? 12 : 0;
    // Finiteness of the worker's two LHCSs after its last step, read from the
    // ring by this wave on either store path (a non-finite value never
    // becomes finite again under +, -, x, so the last state decides).
    bool ok = true;
    uint32_t carry = 0;  // word 5 of the previous step

    // Steps [fast_lo, fast_core) need no bytewise work at all; the last fast
    // step also stores its final phi bytes bytewise.
    const uint64_t fast_core = (phi && fast_hi > fast_lo) ? fast_hi - 1 : fast_hi;

    for (uint32_t blk = 0; blk < nblk; ++blk) {
        __syncthreads();
        if (!live) continue;
        const uint64_t s0 = static_cast<uint64_t>(blk) * kKgHalf;
        const V4 *half = &ring[(blk & 1) * kKgHalf][0];
        if (s0 >= fast_lo && s0 + kKgHalf <= fast_core) {
            // a whole half of the ring in the keystream region: dword stores only
            VC_GLOBAL uint8_t *dst = Bw + (24 * s0 - two_nd - phi) + (odd ? 12 : 0);
#pragma unroll
            for (uint32_t j = 0; j < kKgHalf; ++j) {
                const V4 a = half[64 * j + (lane & ~1u)];
                const V4 b = half[64 * j + (lane | 1u)];
                if (s0 + j + 1 == steps) ok = finite4(a) && finite4(b);
                const uint64_t u0 = bits(a.x) ^ bits(b.x), u1 = bits(a.y) ^ bits(b.y);
                const uint64_t u2 = bits(a.z) ^ bits(b.z), u3 = bits(a.w) ^ bits(b.w);
                const uint32_t w0 = static_cast<uint32_t>(u0);
                const uint32_t w1 = static_cast<uint32_t>((u0 >> 32) & 0xFFFF) | (static_cast<uint32_t>(u1) << 16);
                const uint32_t w2 = static_cast<uint32_t>(u1 >> 16);
                const uint32_t w3 = static_cast<uint32_t>(u2);
                const uint32_t w4 = static_cast<uint32_t>((u2 >> 32) & 0xFFFF) | (static_cast<uint32_t>(u3) << 16);
                const uint32_t w5 = static_cast<uint32_t>(u3 >> 16);
                const uint32_t p0 = odd ? w2 : carry;
                const uint32_t p1 = odd ? w3 : w0;
                const uint32_t p2 = odd ? w4 : w1;
                const uint32_t p3 = odd ? w5 : w2;
                u32x3_a4 v;
                v.x = static_cast<uint32_t>(((static_cast<uint64_t>(p1) << 32) | p0) >> shr);
                v.y = static_cast<uint32_t>(((static_cast<uint64_t>(p2) << 32) | p1) >> shr);
                v.z = static_cast<uint32_t>(((static_cast<uint64_t>(p3) << 32) | p2) >> shr);
                *reinterpret_cast<VC_GLOBAL u32x3_a4 *>(dst) = v;
                dst += 24;
                carry = w5;
            }
            continue;
        }
#pragma unroll 1
        for (uint32_t j = 0; j < kKgHalf; ++j) {
            const uint64_t s = s0 + j;
            if (s >= steps) break;
            const V4 a = half[64 * j + (lane & ~1u)];
            const V4 b = half[64 * j + (lane | 1u)];
            const uint64_t u0 = bits(a.x) ^ bits(b.x), u1 = bits(a.y) ^ bits(b.y);
            const uint64_t u2 = bits(a.z) ^ bits(b.z), u3 = bits(a.w) ^ bits(b.w);
            uint32_t w[6];
            w[0] = static_cast<uint32_t>(u0);
            w[1] = static_cast<uint32_t>((u0 >> 32) & 0xFFFF) | (static_cast<uint32_t>(u1) << 16);
            w[2] = static_cast<uint32_t>(u1 >> 16);
            w[3] = static_cast<uint32_t>(u2);
            w[4] = static_cast<uint32_t>((u2 >> 32) & 0xFFFF) | (static_cast<uint32_t>(u3) << 16);
            w[5] = static_cast<uint32_t>(u3 >> 16);
            if (s >= fast_lo && s < fast_hi) {
                // dword k of the window = stream bytes [24s - phi + 4k, +4)
                VC_GLOBAL uint8_t *dst = Bw + (24 * s - two_nd - phi);
                const uint32_t p0 = odd ? w[2] : carry;
                const uint32_t p1 = odd ? w[3] : w[0];
                const uint32_t p2 = odd ? w[4] : w[1];
                const uint32_t p3 = odd ? w[5] : w[2];
                u32x3_a4 v;
                v.x = static_cast<uint32_t>(((static_cast<uint64_t>(p1) << 32) | p0) >> shr);
                v.y = static_cast<uint32_t>(((static_cast<uint64_t>(p2) << 32) | p1) >> shr);
                v.z = static_cast<uint32_t>(((static_cast<uint64_t>(p3) << 32) | p2) >> shr);
                *reinterpret_cast<VC_GLOBAL u32x3_a4 *>(dst + (odd ? 12 : 0)) = v;
                // the last fast step leaves its final phi bytes to bytewise stores
                const uint32_t tail_from = (odd && phi && s + 1 == fast_hi) ? 24 - phi : 24;
                for (uint32_t jb = tail_from; jb < 24; ++jb)
                    if (24 * s + jb < total) Bw[24 * s + jb - two_nd] = static_cast<uint8_t>(w[jb >> 2] >> (8 * (jb & 3)));
            } else {
                for (uint32_t jb = jlo; jb < jlo + 12; ++jb) {
                    const uint64_t q = 24 * s + jb;
                    const uint8_t byte = static_cast<uint8_t>(w[jb >> 2] >> (8 * (jb & 3)));
                    if (q < two_nd) Dbytes[q] = byte;
                    else if (q < total) Bw[q - two_nd] = byte;
                }
            }
            carry = w[5];
            if (s + 1 == steps) ok = finite4(a) && finite4(b);
        }
    }
    if (live && !ok) flags[0] = FLAG_NONFINITE;
}

}  // namespace

hipError_t launch_lhcs_chain(const StreamRun *d_runs, const ChainRec *d_rec, uint32_t nruns, double *d_state,
                             uint32_t n, double gamma, int *d_flags, hipStream_t s) {
    if (nruns == 0) return hipSuccess;
    hipLaunchKernelGGL(lhcs_chain, dim3(nruns), dim3(64), 0, s, d_runs, d_rec, d_state, n, gamma, d_flags);
    return hipGetLastError();
}

hipError_t launch_lhcs_keygen(const FrameDesc *d_desc, uint32_t count, uint32_t n, double gamma,
                              int *d_flags, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint64_t lanes = 2ull * count * n;  // one worker per lane pair, 64 lanes per workgroup
    hipLaunchKernelGGL(lhcs_keygen, dim3(static_cast<uint32_t>((lanes + 63) / 64)), dim3(128), 0, s,
                       d_desc, count, n, gamma, d_flags);
    return hipGetLastError();
}

}  // namespace vc
