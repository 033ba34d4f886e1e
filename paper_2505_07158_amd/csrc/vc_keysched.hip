// vc_keysched.hip -- the chaotic key schedule of arXiv 2505.07158 on gfx950:
//   lhcs_chain : IC reconstruction from the chain state and H, then 2n RK4
//                iterations of LHCS_m (Sec. II-A, Alg. 1).  Serial per stream
//                (frame t+1 starts from x_2n..w_2n of frame t), so one lane
//                walks one stream's frames.
//   lhcs_keygen: the n workers of Alg. 2, one lane each: two LHCS_w seeded
//                from IR, iterated in lock step; the xor of their FP64 bit
//                patterns gives six mantissa bytes per variable per step
//                (Sec. II-B), cut into shift distances D and bytes B.
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

__device__ __forceinline__ double rk4_comb(double s, double k1, double k2, double k3, double k4) {
    return s + kSixthStep * (((k1 + 2.0 * k2) + 2.0 * k3) + k4);
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
// hash bytes; recombined with the sign of v.  hb points at H[8k].
__device__ __forceinline__ double reconstruct1(double v, const uint8_t *hb) {
    const double a = __builtin_fabs(v);
    const double ip = __builtin_floor(a);
    const double low16 = ip - 65536.0 * __builtin_floor(ip / 65536.0);
    const uint64_t I = exact_u52(low16);
    const uint64_t G = exact_u52(__builtin_floor((a - ip) * kTwo52));
    const uint64_t h16 = (uint64_t(hb[0]) << 8) | hb[1];
    uint64_t h48 = 0;
#pragma unroll
    for (int b = 2; b < 8; ++b) h48 = (h48 << 8) | hb[b];
    const uint64_t I2 = (I ^ h16) % kReconU;
    const uint64_t G2 = G ^ h48;
    const double r = static_cast<double>(static_cast<uint32_t>(I2)) + exact_f52(G2) * kTwoM52;
    return (__double_as_longlong(v) < 0) ? -r : r;
}

__global__ __launch_bounds__(64) void lhcs_chain(const FrameDesc *__restrict__ desc,
                                                 const StreamRun *__restrict__ runs,
                                                 const uint32_t *__restrict__ order, uint32_t nruns,
                                                 double *__restrict__ state, uint32_t n, double gamma,
                                                 int *__restrict__ flags) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nruns) return;
    const StreamRun run = runs[r];
    double *st = state + 4 * static_cast<uint64_t>(run.slot);
    V4 base{st[0], st[1], st[2], st[3]};
    bool ok = true;
    for (uint32_t u = 0; u < run.count; ++u) {
        const FrameDesc d = desc[order[run.first + u]];
        uint8_t H[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) H[k] = gmem(d.hash)[k];
        V4 s{reconstruct1(base.x, H), reconstruct1(base.y, H + 8), reconstruct1(base.z, H + 16),
             reconstruct1(base.w, H + 24)};
        VC_GLOBAL double *ir = gmem(d.IR);
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
    st[0] = base.x;
    st[1] = base.y;
    st[2] = base.z;
    st[3] = base.w;
    if (!ok) flags[0] = FLAG_NONFINITE;
}

__device__ __forceinline__ uint64_t bits(double v) { return static_cast<uint64_t>(__double_as_longlong(v)); }

__device__ __forceinline__ bool finite4(const V4 &s) {
    return __builtin_isfinite(s.x) && __builtin_isfinite(s.y) && __builtin_isfinite(s.z) &&
           __builtin_isfinite(s.w);
}

// Exchange a double with the other lane of the pair (lanes 2k, 2k+1) by a
// DPP quad permutation [1, 0, 3, 2].
__device__ __forceinline__ double pair_swap(double v) {
    const uint64_t b = bits(v);
    const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(static_cast<uint32_t>(b)), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(static_cast<uint32_t>(b >> 32)), 0xB1, 0xF, 0xF,
                                            false);
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                                       static_cast<uint32_t>(lo)));
}

typedef uint32_t u32x3_a4 __attribute__((ext_vector_type(3), aligned(4)));

// Worker i of frame f runs on a lane pair: the even lane iterates LHCS^1,
// the odd lane LHCS^2, and after every step the pair swaps its four
// iterates so both hold the 24 stream bytes of the step.
//
// Worker i owns distances [floor(i*ND/n), floor((i+1)*ND/n)) and bytes
// [floor(i*L/n), floor((i+1)*L/n)); its byte stream gives its distances
// first (little-endian pairs) and then its bytes.  Seeds: A = IR_{2i+1},
// Q = IR_{2i+2}; LHCS^1 = (A.x, Q.y, A.z, Q.w), LHCS^2 = (Q.x, A.y, Q.z,
// A.w).  Each step emits, for x, y, z, w in turn, the six low mantissa
// bytes of the xor of the two bit patterns, least significant first.
//
// Stores: steps whose 24 bytes lie inside the keystream region are written
// as six dwords at dword-aligned addresses (the even lane three, the odd
// lane three); the dword straddling the previous step takes that step's
// last bytes from a carry register.  The distance bytes, and the few steps
// at either end of the region, are stored byte by byte.
__global__ __launch_bounds__(64) void lhcs_keygen(const FrameDesc *__restrict__ desc, uint32_t count,
                                                  uint32_t n, double gamma, int *__restrict__ flags) {
    const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t worker = g >> 1;
    const uint32_t odd = static_cast<uint32_t>(g & 1);
    const uint64_t f = worker / n;
    const uint32_t i = static_cast<uint32_t>(worker % n);
    if (f >= count) return;
    const FrameDesc d = desc[f];
    const uint64_t ND = 3ull * d.h + 3ull * d.w;
    const uint64_t d0 = ND * i / n, d1 = ND * (i + 1) / n;
    const uint64_t b0 = d.L * i / n, b1 = d.L * (i + 1) / n;
    const uint64_t two_nd = 2 * (d1 - d0);
    const uint64_t total = two_nd + (b1 - b0);
    const uint64_t steps = (total + 23) / 24;
    const VC_GLOBAL double *A = gmem(d.IR) + 8 * static_cast<uint64_t>(i);
    const VC_GLOBAL double *Q = A + 4;
    V4 l = odd ? V4{Q[0], A[1], Q[2], A[3]} : V4{A[0], Q[1], A[2], Q[3]};
    VC_GLOBAL uint8_t *Dbytes = reinterpret_cast<VC_GLOBAL uint8_t *>(gmem(d.D) + d0);
    VC_GLOBAL uint8_t *Bw = gmem(d.B) + b0;

    // Fast steps s in [s_a, s_b): dwords cover stream bytes
    // [24s - phi, 24s + 24 - phi), all inside [two_nd, total).
    const uint32_t phi = static_cast<uint32_t>((reinterpret_cast<uintptr_t>(d.B + b0) - two_nd) & 3);
    const uint64_t s_a = (two_nd + phi + 23) / 24;
    const uint64_t s_b = (total + phi >= 24) ? (total + phi - 24) / 24 + 1 : 0;
    const uint32_t shr = 8 * (4 - phi);  // 32 when phi == 0

    uint32_t w[6];
    uint32_t carry = 0;  // word 5 of the previous step
    auto step = [&]() {
        rk4_step(l, gamma);
        const double ox = pair_swap(l.x), oy = pair_swap(l.y), oz = pair_swap(l.z), ow = pair_swap(l.w);
        const uint64_t u0 = bits(l.x) ^ bits(ox), u1 = bits(l.y) ^ bits(oy);
        const uint64_t u2 = bits(l.z) ^ bits(oz), u3 = bits(l.w) ^ bits(ow);
        w[0] = static_cast<uint32_t>(u0);
        w[1] = static_cast<uint32_t>((u0 >> 32) & 0xFFFF) | (static_cast<uint32_t>(u1) << 16);
        w[2] = static_cast<uint32_t>(u1 >> 16);
        w[3] = static_cast<uint32_t>(u2);
        w[4] = static_cast<uint32_t>((u2 >> 32) & 0xFFFF) | (static_cast<uint32_t>(u3) << 16);
        w[5] = static_cast<uint32_t>(u3 >> 16);
    };
    auto emit_bytes = [&](uint64_t s, uint32_t jlo, uint32_t jhi) {
        for (uint32_t j = jlo; j < jhi; ++j) {
            const uint64_t q = 24 * s + j;
            const uint8_t byte = static_cast<uint8_t>(w[j >> 2] >> (8 * (j & 3)));
            if (q < two_nd) Dbytes[q] = byte;
            else if (q < total) Bw[q - two_nd] = byte;
        }
    };

    uint64_t s = 0;
    const uint64_t head_end = (s_a < s_b) ? s_a : steps;
    for (; s < head_end && s < steps; ++s) {
        step();
        emit_bytes(s, odd ? 12 : 0, odd ? 24 : 12);
        carry = w[5];
    }
    if (s_a < s_b) {
        for (; s < s_b; ++s) {
            step();
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
            carry = w[5];
        }
        // the last fast step leaves its final phi bytes to the carry
        if (odd && phi) emit_bytes(s - 1, 24 - phi, 24);
        for (; s < steps; ++s) {
            step();
            emit_bytes(s, odd ? 12 : 0, odd ? 24 : 12);
        }
    }
    if (!finite4(l)) flags[0] = FLAG_NONFINITE;
}

}  // namespace

hipError_t launch_lhcs_chain(const FrameDesc *d_desc, const StreamRun *d_runs, const uint32_t *d_order,
                             uint32_t nruns, double *d_state, uint32_t n, double gamma, int *d_flags,
                             hipStream_t s) {
    if (nruns == 0) return hipSuccess;
    hipLaunchKernelGGL(lhcs_chain, dim3((nruns + 63) / 64), dim3(64), 0, s, d_desc, d_runs, d_order,
                       nruns, d_state, n, gamma, d_flags);
    return hipGetLastError();
}

hipError_t launch_lhcs_keygen(const FrameDesc *d_desc, uint32_t count, uint32_t n, double gamma,
                              int *d_flags, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint64_t lanes = 2ull * count * n;
    hipLaunchKernelGGL(lhcs_keygen, dim3(static_cast<uint32_t>((lanes + 63) / 64)), dim3(64), 0, s,
                       d_desc, count, n, gamma, d_flags);
    return hipGetLastError();
}

}  // namespace vc
