// vc_stats.hip -- the integer reductions behind the statistical tests of
// Sec. III of arXiv 2505.07158, on gfx950:
//   * 256-level intensity histograms per channel of whole frames (Eqs. 4-5:
//     histogram variance and chi-square; Eq. 10: information entropy),
//   * the same over k sub-blocks of T_B pixels per frame (Eq. 11: local
//     Shannon entropy),
//   * exact integer moments (sums of x, y, x^2, y^2, xy) of adjacent pixel
//     pairs in the horizontal, vertical and diagonal directions (Eqs. 6-9:
//     correlation coefficients), over given pixel positions or over every
//     pixel that has all three neighbours,
//   * difference counts of two frames (Sec. IV: NPCR and UACI of Eqs. 14-16,
//     and the PSNR of frames decrypted after cropping or channel noise).
// Positions and block origins are validated on the host before upload.
// Everything here is integer arithmetic, so results are exact; the
// floating-point formulas of the tests run on the host from these counts.
#include "vc_internal.hpp"

namespace vc {
namespace {

constexpr uint32_t kHistThreads = 256;
constexpr uint32_t kHistChunk = 1u << 16;  // bytes of one frame per workgroup

// Workgroup (frame f, chunk k): bytes [k*kHistChunk, ...) of frame f into an
// LDS histogram (3 x 256 counters, channel = byte index mod 3), then added
// to the frame's global histogram.
__global__ __launch_bounds__(kHistThreads) void frame_histograms(const StatFrame *__restrict__ frames,
                                                                uint32_t chunks_per_frame,
                                                                uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[3 * 256];
    const uint32_t f = blockIdx.x / chunks_per_frame, k = blockIdx.x - f * chunks_per_frame;
    for (uint32_t i = threadIdx.x; i < 3 * 256; i += kHistThreads) h[i] = 0;
    __syncthreads();
    const StatFrame fr = frames[f];
    const uint64_t L = 3ull * fr.w * fr.h;
    const uint64_t b0 = static_cast<uint64_t>(k) * kHistChunk;
    const uint64_t b1 = (b0 + kHistChunk < L) ? b0 + kHistChunk : L;
    const VC_GLOBAL uint8_t *p = gmem(fr.data);
    // the channel of byte b is b mod 3; the stride is 1 mod 3
    static_assert(kHistThreads % 3 == 1, "the channel update assumes a stride of 1 mod 3");
    uint32_t c = static_cast<uint32_t>((b0 + threadIdx.x) % 3);
    for (uint64_t b = b0 + threadIdx.x; b < b1; b += kHistThreads) {
        atomicAdd(&h[c * 256 + p[b]], 1u);
        c = (c == 2) ? 0 : c + 1;
    }
    __syncthreads();
    uint32_t *out = hist + 3ull * 256 * f;
    for (uint32_t i = threadIdx.x; i < 3 * 256; i += kHistThreads)
        if (h[i]) atomicAdd(&out[i], h[i]);
}

// Workgroup (frame f, block m): the bh x bw pixels at origin (r, c) of
// frame f, channel by channel, into hist[f][m][c][256].
__global__ __launch_bounds__(kHistThreads) void block_histograms(const StatFrame *__restrict__ frames,
                                                                uint32_t blocks, uint32_t bw, uint32_t bh,
                                                                const uint32_t *__restrict__ origins,
                                                                uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[3 * 256];
    const uint32_t f = blockIdx.x / blocks, m = blockIdx.x - f * blocks;
    for (uint32_t i = threadIdx.x; i < 3 * 256; i += kHistThreads) h[i] = 0;
    __syncthreads();
    const StatFrame fr = frames[f];
    const VC_GLOBAL uint32_t *o = gmem(origins) + 2ull * (static_cast<uint64_t>(f) * blocks + m);
    const uint32_t r0 = o[0], c0 = o[1];
    const VC_GLOBAL uint8_t *p = gmem(fr.data);
    const uint32_t n = bw * bh * 3;
    for (uint32_t t = threadIdx.x; t < n; t += kHistThreads) {
        const uint32_t row = t / (3 * bw), rem = t - row * 3 * bw;
        const uint64_t off = (static_cast<uint64_t>(r0 + row) * fr.w + c0) * 3 + rem;
        atomicAdd(&h[(rem % 3) * 256 + p[off]], 1u);
    }
    __syncthreads();
    VC_GLOBAL uint32_t *out = gmem(hist) + 3ull * 256 * (static_cast<uint64_t>(f) * blocks + m);
    for (uint32_t i = threadIdx.x; i < 3 * 256; i += kHistThreads) out[i] = h[i];
}

// Moments of adjacent pairs: for direction d (0 horizontal: (r, c+1),
// 1 vertical: (r+1, c), 2 diagonal: (r+1, c+1)) and channel ch, the sums
// of x, y, x^2, y^2, xy over the pixel positions of frame f.  Each lane
// accumulates in 64-bit registers; lanes of a workgroup meet in LDS; one
// atomic add per sum per workgroup.
constexpr uint32_t kMomThreads = 256;
constexpr uint32_t kMomPerGroup = 4096;  // positions per workgroup

__global__ __launch_bounds__(kMomThreads) void pair_moments(const StatFrame *__restrict__ frames,
                                                            uint32_t groups_per_frame, uint32_t npos,
                                                            const uint32_t *__restrict__ positions,
                                                            unsigned long long *__restrict__ moments) {
    __shared__ unsigned long long acc[45];
    const uint32_t f = blockIdx.x / groups_per_frame, g = blockIdx.x - f * groups_per_frame;
    for (uint32_t i = threadIdx.x; i < 45; i += kMomThreads) acc[i] = 0;
    __syncthreads();
    const StatFrame fr = frames[f];
    const VC_GLOBAL uint8_t *p = gmem(fr.data);
    const uint32_t w = fr.w, h = fr.h;
    // without positions: every pixel (r, c) with r < h-1 and c < w-1 takes
    // part in all three directions
    const uint64_t total = positions ? npos : static_cast<uint64_t>(h - 1) * (w - 1);
    unsigned long long s[45];
#pragma unroll
    for (int i = 0; i < 45; ++i) s[i] = 0;
    const uint64_t i0 = static_cast<uint64_t>(g) * kMomPerGroup;
    const uint64_t i1 = (i0 + kMomPerGroup < total) ? i0 + kMomPerGroup : total;
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += kMomThreads) {
        uint32_t r, c;
        if (positions) {
            const VC_GLOBAL uint32_t *q = gmem(positions) + 2ull * (static_cast<uint64_t>(f) * npos + i);
            r = q[0];
            c = q[1];
        } else {
            const uint32_t i32 = static_cast<uint32_t>(i);  // (h-1)(w-1) < 2^32
            r = i32 / (w - 1);
            c = i32 - r * (w - 1);
        }
        const uint64_t base = (static_cast<uint64_t>(r) * w + c) * 3;
        const uint64_t nb[3] = {base + 3, base + 3ull * w, base + 3ull * w + 3};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const unsigned long long x = p[base + ch];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const unsigned long long y = p[nb[d] + ch];
                unsigned long long *t = s + 15 * d + 5 * ch;
                t[0] += x;
                t[1] += y;
                t[2] += x * x;
                t[3] += y * y;
                t[4] += x * y;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 45; ++i) {
        unsigned long long v = s[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & 63) == 0) atomicAdd(&acc[i], v);
    }
    __syncthreads();
    unsigned long long *out = moments + 45ull * f;
    for (uint32_t i = threadIdx.x; i < 45; i += kMomThreads) atomicAdd(&out[i], acc[i]);
}

// Workgroup (frame f, chunk k): per channel, over bytes [k*kHistChunk, ...)
// of the frames a[f] and b[f] (same shape): the number of differing bytes,
// the sum of |a - b|, the sum of (a - b)^2 and the number of differing bits
// -- the counts behind NPCR and UACI (Sec. IV-B, Eqs. 14-16) and the PSNR of
// a decryption after cropping or noise (Sec. IV-C).  A lane sees at most
// kHistChunk / kHistThreads bytes, so its 32-bit sums cannot overflow
// (256 * 255^2 < 2^24), nor can a wave's (64 times that).
__global__ __launch_bounds__(kHistThreads) void frame_diff(const StatFrame *__restrict__ fa,
                                                          const StatFrame *__restrict__ fb,
                                                          uint32_t chunks_per_frame,
                                                          unsigned long long *__restrict__ out) {
    __shared__ unsigned long long acc[12];
    const uint32_t f = blockIdx.x / chunks_per_frame, k = blockIdx.x - f * chunks_per_frame;
    if (threadIdx.x < 12) acc[threadIdx.x] = 0;
    __syncthreads();
    const StatFrame A = fa[f];
    const uint64_t L = 3ull * A.w * A.h;
    const uint64_t b0 = static_cast<uint64_t>(k) * kHistChunk;
    const uint64_t b1 = (b0 + kHistChunk < L) ? b0 + kHistChunk : L;
    const VC_GLOBAL uint8_t *pa = gmem(A.data);
    const VC_GLOBAL uint8_t *pb = gmem(fb[f].data);
    uint32_t s[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) s[i] = 0;
    static_assert(kHistThreads % 3 == 1, "the channel update below assumes a stride of 1 mod 3");
    uint32_t c = static_cast<uint32_t>((b0 + threadIdx.x) % 3);
    for (uint64_t b = b0 + threadIdx.x; b < b1; b += kHistThreads, c = (c == 2) ? 0 : c + 1) {
        const uint32_t x = pa[b], y = pb[b];
        const uint32_t d = x > y ? x - y : y - x;
        // select by channel without dynamic register indexing
#pragma unroll
        for (uint32_t ch = 0; ch < 3; ++ch) {
            const bool on = (ch == c);
            s[4 * ch + 0] += on ? (d != 0) : 0u;
            s[4 * ch + 1] += on ? d : 0u;
            s[4 * ch + 2] += on ? d * d : 0u;
            s[4 * ch + 3] += on ? static_cast<uint32_t>(__popc(x ^ y)) : 0u;
        }
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        uint32_t v = s[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(&acc[i], static_cast<unsigned long long>(v));
    }
    __syncthreads();
    if (threadIdx.x < 12 && acc[threadIdx.x]) atomicAdd(&out[12ull * f + threadIdx.x], acc[threadIdx.x]);
}

// Streaming reference for the HBM ceiling of the confusion kernels: one
// 16-byte word per thread, out = a (KIND 0) or out = a ^ b (KIND 1).
typedef uint32_t u32x4_s __attribute__((ext_vector_type(4)));
template <int KIND>
__global__ __launch_bounds__(256) void stream_probe(const u32x4_s *__restrict__ a, const u32x4_s *__restrict__ b,
                                                    u32x4_s *__restrict__ out, uint64_t n16) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n16) return;
    const VC_GLOBAL u32x4_s *ga = gmem(a);
    VC_GLOBAL u32x4_s *go = gmem(out);
    if (KIND == 0) go[i] = ga[i];
    else go[i] = ga[i] ^ gmem(b)[i];
}

}  // namespace

hipError_t launch_stream_probe(int kind, const uint8_t *a, const uint8_t *b, uint8_t *out, uint64_t bytes,
                               hipStream_t s) {
    const uint64_t n16 = bytes / 16, groups = (n16 + 255) / 256;
    if (groups == 0) return hipSuccess;
    if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const auto *a4 = reinterpret_cast<const u32x4_s *>(a);
    const auto *b4 = reinterpret_cast<const u32x4_s *>(b);
    auto *o4 = reinterpret_cast<u32x4_s *>(out);
    if (kind == 0)
        hipLaunchKernelGGL(stream_probe<0>, dim3(static_cast<uint32_t>(groups)), dim3(256), 0, s, a4, b4, o4, n16);
    else
        hipLaunchKernelGGL(stream_probe<1>, dim3(static_cast<uint32_t>(groups)), dim3(256), 0, s, a4, b4, o4, n16);
    return hipGetLastError();
}

hipError_t launch_frame_diff(const StatFrame *d_a, const StatFrame *d_b, uint32_t count, uint64_t max_bytes,
                             unsigned long long *d_out, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint64_t chunks = (max_bytes + kHistChunk - 1) / kHistChunk;
    if (chunks * count > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(frame_diff, dim3(static_cast<uint32_t>(chunks * count)), dim3(kHistThreads), 0, s, d_a, d_b,
                       static_cast<uint32_t>(chunks), d_out);
    return hipGetLastError();
}

hipError_t launch_frame_histograms(const StatFrame *d_frames, uint32_t count, uint64_t max_bytes, uint32_t *d_hist,
                                   hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint64_t chunks = (max_bytes + kHistChunk - 1) / kHistChunk;
    if (chunks * count > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(frame_histograms, dim3(static_cast<uint32_t>(chunks * count)), dim3(kHistThreads), 0, s,
                       d_frames, static_cast<uint32_t>(chunks), d_hist);
    return hipGetLastError();
}

hipError_t launch_block_histograms(const StatFrame *d_frames, uint32_t count, uint32_t blocks, uint32_t bw,
                                   uint32_t bh, const uint32_t *d_origins, uint32_t *d_hist, hipStream_t s) {
    if (count == 0 || blocks == 0) return hipSuccess;
    if (static_cast<uint64_t>(blocks) * count > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(block_histograms, dim3(count * blocks), dim3(kHistThreads), 0, s, d_frames, blocks, bw, bh,
                       d_origins, d_hist);
    return hipGetLastError();
}

hipError_t launch_pair_moments(const StatFrame *d_frames, uint32_t count, uint64_t max_positions, uint32_t npos,
                               const uint32_t *d_positions, unsigned long long *d_moments, hipStream_t s) {
    if (count == 0 || max_positions == 0) return hipSuccess;
    const uint64_t groups = (max_positions + kMomPerGroup - 1) / kMomPerGroup;
    if (groups * count > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pair_moments, dim3(static_cast<uint32_t>(groups * count)), dim3(kMomThreads), 0, s, d_frames,
                       static_cast<uint32_t>(groups), npos, d_positions, d_moments);
    return hipGetLastError();
}

}  // namespace vc
