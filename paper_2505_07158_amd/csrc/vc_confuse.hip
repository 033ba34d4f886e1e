// vc_confuse.hip -- bit-level confusion fused with one XOR round (Sec. II-C
// of arXiv 2505.07158: Eq. 2 row shifts, Eq. 3 column shifts, Algs. 3-7) and
// its exact inverse, on gfx950.
//
// The paper keeps an 8w x h bit matrix per channel and runs five kernels
// (bit extraction, H-shift, V-shift, XOR, packing) with full-matrix copies
// in between.  Here the bits never leave byte form.  For output byte
// (i, j, c) (row i, pixel column j, channel c), with d_h = D[c*h + r] and
// d_v = D[3h + c*w + j]:
//     r = (i - d_v mod h) mod h,     s = (8j - d_h mod 8w) mod 8w,
//     C[i][j][c] = bits s..s+7 of source row r, channel c  xor  B[i][j][c]
// where "bits s..s+7" is the funnel shift of pixels s/8 and s/8+1 (mod w),
// least significant bit first (Algs. 3 and 7).
//
// Tiling: a workgroup owns a full-height strip of WT pixel columns (all
// three channels) of one frame.  A column shift stays inside the strip, and
// a row shift maps the strip to one contiguous window of WT+1 pixels of each
// source row, so
//   phase 1: for every source row r and channel c, funnel-shift its window
//            into LDS (one 16-byte global load per four output bytes),
//   phase 2: every output row of the strip gathers its bytes from the LDS
//            rows (i - d_v) mod h, xors B and stores C with coalesced dword
//            accesses.
// Decryption mirrors it: coalesced loads of C and B into LDS with the column
// shift undone, then the row funnel shift scattered to the plaintext rows.
// Workgroups are mapped so that all strips of one frame run on one XCD and
// share its L2 (the row windows of neighbouring strips overlap).
#include <algorithm>

#include "vc_internal.hpp"

namespace vc {
namespace {

typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

// Workgroup -> (frame within the launch, strip).  With xcd_map the
// hardware's round-robin placement of consecutive workgroups over the 8 XCDs
// is undone: XCD x (workgroups g with g % 8 == x) gets frames x, x+8, ...,
// each frame's strips consecutively.
__device__ __forceinline__ void map_workgroup(uint32_t g, uint32_t nstrips, int xcd_map, uint32_t &fl,
                                              uint32_t &strip) {
    if (xcd_map) {
        const uint32_t x = g & 7, l = g >> 3;
        const uint32_t slot = l / nstrips;
        strip = l - slot * nstrips;
        fl = slot * 8 + x;
    } else {
        fl = g / nstrips;
        strip = g - fl * nstrips;
    }
}

// LDS layout of both kernels: the strip S (h rows of RS bytes), then the
// row distances d_h mod 8w (3h words), then the strip's column distances
// d_v mod h (3 x (WT + 4) words).
__host__ __device__ constexpr uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

template <int WT>
struct EncLayout {
    static constexpr uint32_t RS = 3 * WT;
    __host__ __device__ static uint32_t dh_off(uint32_t h) { return align16(h * RS); }
    __host__ __device__ static uint32_t dv_off(uint32_t h) { return dh_off(h) + 4 * 3 * h; }
    __host__ __device__ static uint32_t bytes(uint32_t h) { return dv_off(h) + 4 * 3 * (WT + 4); }
};
template <int WT>
struct DecLayout {
    static constexpr uint32_t CS = WT + 4;  // columns k = 0..WT (the last one is the next strip's first)
    static constexpr uint32_t RS = 3 * CS;
    __host__ __device__ static uint32_t dh_off(uint32_t h) { return align16(h * RS); }
    __host__ __device__ static uint32_t dv_off(uint32_t h) { return dh_off(h) + 4 * 3 * h; }
    __host__ __device__ static uint32_t bytes(uint32_t h) { return dv_off(h) + 4 * 3 * (WT + 4); }
};

// Rows of the coalesced phase prefetched into registers per thread: as
// many as keep the 1024-thread kernel within 96 VGPRs without spills, so
// that a workgroup still fits on a CU beside one wave of the latency-bound
// kernels (4 x 96 + 128 <= 512 VGPRs per SIMD).
template <int WT>
constexpr uint32_t prefetch_rows() {
    return WT <= 16 ? 16 : 20;
}

// Funnel output of four consecutive strip columns k..k+3 of source row r,
// channel c: the 40-bit little-endian run of pixels q..q+4 (mod w) shifted
// right by t.  `row` points at byte c of row r.
__device__ __forceinline__ uint32_t window4_slow(const VC_GLOBAL uint8_t *row, uint32_t q, uint32_t w,
                                                 uint32_t t) {
    uint32_t X = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        X |= static_cast<uint32_t>(row[3 * q]) << (8 * m);
        q = (q + 1 == w) ? 0 : q + 1;
    }
    return __builtin_amdgcn_alignbit(static_cast<uint32_t>(row[3 * q]), X, t);
}

// Same from a 16-byte vector loaded at the dword boundary at or below
// byte 3q (sh = misalignment): bytes sh + {0, 3, 6, 9, 12}.
__device__ __forceinline__ uint32_t window4_fast(const u32x4_a4 &v, uint32_t sh, uint32_t t) {
    const uint32_t e0 = __builtin_amdgcn_alignbyte(v.y, v.x, sh);
    const uint32_t e1 = __builtin_amdgcn_alignbyte(v.z, v.y, sh);
    const uint32_t e2 = __builtin_amdgcn_alignbyte(v.w, v.z, sh);
    const uint32_t X = (e0 & 0xFFu) | ((e0 >> 16) & 0xFF00u) | (e1 & 0xFF0000u) | ((e2 << 16) & 0xFF000000u);
    const uint32_t b4 = (v.w >> (8 * sh)) & 0xFFu;
    return __builtin_amdgcn_alignbit(b4, X, t);
}

// ----------------------------------------------------------------------
// Encryption
// ----------------------------------------------------------------------
template <int WT, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(5, 8))) void confuse_xor_enc(
    const FrameDesc *__restrict__ desc, uint32_t first, uint32_t nframes, Geometry geo, uint32_t nstrips, int xcd_map,
    int aligned) {
    extern __shared__ __align__(16) uint8_t smem[];
    using Lay = EncLayout<WT>;
    constexpr uint32_t RS = Lay::RS;           // LDS row: channel c at c*WT + k
    constexpr uint32_t KG = WT / 4;            // 4-byte groups per (row, channel)
    constexpr uint32_t KPL = KG < 4 ? KG : 4;  // groups per item
    constexpr uint32_t LPG = KG / KPL;         // items per (row, channel)
    constexpr uint32_t GPR = 3 * WT / 4;       // dwords per full strip row
    constexpr uint32_t RP = NT / GPR;          // rows per pass of the coalesced phase
    constexpr uint32_t kPrefetchRows = prefetch_rows<WT>();

    uint32_t fl, strip;
    map_workgroup(blockIdx.x, nstrips, xcd_map, fl, strip);
    if (fl >= nframes) return;
    const FrameDesc d = desc[first + fl];
    const uint32_t w = geo.w, h = geo.h, W8 = geo.W8, row_bytes = geo.row_bytes;
    const uint32_t j0 = strip * WT;
    const uint32_t wt = (w - j0 < static_cast<uint32_t>(WT)) ? w - j0 : WT;
    const VC_GLOBAL uint8_t *__restrict__ P = gmem(d.in);
    const VC_GLOBAL uint16_t *__restrict__ D = gmem(d.D);
    uint8_t *S = smem;
    uint32_t *dhS = reinterpret_cast<uint32_t *>(smem + Lay::dh_off(h));
    uint32_t *dvS = reinterpret_cast<uint32_t *>(smem + Lay::dv_off(h));
    VC_GLOBAL uint8_t *__restrict__ outp = gmem(d.out) + 3 * j0;
    const VC_GLOBAL uint8_t *__restrict__ Bp = gmem(d.B) + 3 * j0;

    // The keystream is read in the coalesced phase; start those loads now.
    const uint32_t g = threadIdx.x % GPR, i0 = threadIdx.x / GPR;
    const bool p2 = aligned && i0 < RP && g < 3 * wt / 4 && i0 < h;
    uint32_t bpre[kPrefetchRows];
    if (p2) {
#pragma unroll
        for (uint32_t k = 0; k < kPrefetchRows; ++k) {
            const uint32_t i = i0 + k * RP;
            if (i < h)
                bpre[k] = *reinterpret_cast<const VC_GLOBAL uint32_t *>(Bp + static_cast<uint64_t>(i) * row_bytes + 4 * g);
        }
    }

    // Phase 0: distances, reduced once.
    for (uint32_t it = threadIdx.x; it < 3 * h; it += NT) dhS[it] = mod_u16(D[it], geo.mod_W8);
    for (uint32_t it = threadIdx.x; it < 3 * wt; it += NT) {
        const uint32_t c = it / wt, k = it - c * wt;
        dvS[c * WT + k] = mod_u16(D[3 * h + c * w + j0 + k], geo.mod_h);
    }
    __syncthreads();

    // Phase 1: S[r][c][k] = bits (8(j0+k) - d_h(c,r)) .. +7 of row r, channel
    // c.  Two items per thread are in flight at a time.
    const uint32_t items1 = h * 3 * LPG;
    for (uint32_t base = threadIdx.x; base < items1; base += 2 * NT) {
        uint32_t qv[2], tv[2], sh[2];
        const VC_GLOBAL uint8_t *rowv[2];
        uint8_t *dstv[2];
        bool valid[2];
        u32x4_a4 v[2][KPL];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint32_t it0 = base + e * NT;
            valid[e] = it0 < items1;
            const uint32_t it = valid[e] ? it0 : base;
            const uint32_t kl = it % LPG, rc = it / LPG;
            const uint32_t r = rc / 3, c = rc - 3 * r;
            uint32_t s0 = 8 * j0 + W8 - dhS[c * h + r];
            if (s0 >= W8) s0 -= W8;
            tv[e] = s0 & 7;
            uint32_t q = (s0 >> 3) + 4 * KPL * kl;
            if (q >= w) q -= w;
            qv[e] = q;
            rowv[e] = P + static_cast<uint64_t>(r) * row_bytes + c;
            dstv[e] = S + r * RS + c * WT + 4 * KPL * kl;
            // 16-byte loads for the groups that do not wrap around the row
            // end; the others are computed byte by byte below.
            const uintptr_t sa = reinterpret_cast<uintptr_t>(rowv[e] + 3 * q);
            sh[e] = static_cast<uint32_t>(sa & 3);
#pragma unroll
            for (uint32_t u = 0; u < KPL; ++u) {
                uint32_t qu = q + 4 * u;
                if (qu >= w) qu -= w;
                const bool fast = aligned && qu + 4 < w;
                v[e][u] = fast ? *reinterpret_cast<const VC_GLOBAL u32x4_a4 *>(
                                     reinterpret_cast<uintptr_t>(rowv[e] + 3 * qu) - sh[e])
                               : u32x4_a4{0, 0, 0, 0};
            }
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (!valid[e]) continue;
#pragma unroll
            for (uint32_t u = 0; u < KPL; ++u) {
                uint32_t qu = qv[e] + 4 * u;
                if (qu >= w) qu -= w;
                const bool fast = aligned && qu + 4 < w;
                const uint32_t o = fast ? window4_fast(v[e][u], sh[e], tv[e]) : window4_slow(rowv[e], qu, w, tv[e]);
                *reinterpret_cast<uint32_t *>(dstv[e] + 4 * u) = o;
            }
        }
    }
    __syncthreads();

    // Phase 2: C[i][j0+k][c] = S[(i - d_v(c, j0+k)) mod h][c][k] ^ B.
    if (aligned) {
        if (p2) {
            uint32_t addr[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const uint32_t p = 4 * g + m, k = p / 3, c = p - 3 * k;
                const uint32_t dv = dvS[c * WT + k];
                const uint32_t r = (i0 >= dv) ? i0 - dv : i0 + h - dv;
                addr[m] = r * RS + c * WT + k;
            }
            const uint32_t step = RP % h;
            const uint32_t stepA = step * RS, wrapA = h * RS;
            const uint64_t offstep = static_cast<uint64_t>(RP) * row_bytes;
            uint64_t off = static_cast<uint64_t>(i0) * row_bytes + 4 * g;
            auto gather = [&]() {
                const uint32_t v = static_cast<uint32_t>(S[addr[0]]) | (static_cast<uint32_t>(S[addr[1]]) << 8) |
                                   (static_cast<uint32_t>(S[addr[2]]) << 16) |
                                   (static_cast<uint32_t>(S[addr[3]]) << 24);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    addr[m] += stepA;
                    if (addr[m] >= wrapA) addr[m] -= wrapA;
                }
                return v;
            };
#pragma unroll
            for (uint32_t k = 0; k < kPrefetchRows; ++k) {
                if (i0 + k * RP < h) {
                    *reinterpret_cast<VC_GLOBAL uint32_t *>(outp + off) = gather() ^ bpre[k];
                    off += offstep;
                }
            }
            for (uint32_t i = i0 + kPrefetchRows * RP; i < h; i += RP) {
                *reinterpret_cast<VC_GLOBAL uint32_t *>(outp + off) =
                    gather() ^ *reinterpret_cast<const VC_GLOBAL uint32_t *>(Bp + off);
                off += offstep;
            }
        }
    } else {
        const uint32_t rowlen = 3 * wt;
        const uint32_t items2 = h * rowlen;
        for (uint32_t it = threadIdx.x; it < items2; it += NT) {
            const uint32_t i = it / rowlen, p = it - i * rowlen;
            const uint32_t k = p / 3, c = p - 3 * k;
            const uint32_t dv = dvS[c * WT + k];
            const uint32_t r = (i >= dv) ? i - dv : i + h - dv;
            const uint64_t off = static_cast<uint64_t>(i) * row_bytes + p;
            outp[off] = S[r * RS + c * WT + k] ^ Bp[off];
        }
    }
}

// ----------------------------------------------------------------------
// Decryption
// ----------------------------------------------------------------------
template <int WT, int NT>
__global__ __launch_bounds__(NT) void confuse_xor_dec(const FrameDesc *__restrict__ desc, uint32_t first,
                                                      uint32_t nframes, Geometry geo, uint32_t nstrips,
                                                      int xcd_map, int aligned) {
    extern __shared__ __align__(16) uint8_t smem[];
    using Lay = DecLayout<WT>;
    constexpr uint32_t CS = Lay::CS;
    constexpr uint32_t RS = Lay::RS;
    constexpr uint32_t GPR = 3 * WT / 4;
    constexpr uint32_t RP = NT / GPR;
    constexpr uint32_t kPrefetchRows = 32;  // C ^ B words in flight per thread

    uint32_t fl, strip;
    map_workgroup(blockIdx.x, nstrips, xcd_map, fl, strip);
    if (fl >= nframes) return;
    const FrameDesc d = desc[first + fl];
    const uint32_t w = geo.w, h = geo.h, W8 = geo.W8, row_bytes = geo.row_bytes;
    const uint32_t j0 = strip * WT;
    const uint32_t wt = (w - j0 < static_cast<uint32_t>(WT)) ? w - j0 : WT;
    const uint32_t je = (j0 + wt == w) ? 0 : j0 + wt;  // column after the strip
    const VC_GLOBAL uint16_t *__restrict__ D = gmem(d.D);
    const VC_GLOBAL uint8_t *__restrict__ Cp = gmem(d.in) + 3 * j0;
    const VC_GLOBAL uint8_t *__restrict__ Bp = gmem(d.B) + 3 * j0;
    VC_GLOBAL uint8_t *__restrict__ Pout = gmem(d.out);
    uint8_t *S = smem;
    uint32_t *dhS = reinterpret_cast<uint32_t *>(smem + Lay::dh_off(h));
    uint32_t *dvS = reinterpret_cast<uint32_t *>(smem + Lay::dv_off(h));

    // Start the coalesced loads of C and B.
    const uint32_t g = threadIdx.x % GPR, i0 = threadIdx.x / GPR;
    const bool p1 = aligned && i0 < RP && g < 3 * wt / 4 && i0 < h;
    uint32_t ypre[kPrefetchRows];
    if (p1) {
#pragma unroll
        for (uint32_t k = 0; k < kPrefetchRows; ++k) {
            const uint32_t i = i0 + k * RP;
            if (i < h) {
                const uint64_t off = static_cast<uint64_t>(i) * row_bytes + 4 * g;
                ypre[k] = *reinterpret_cast<const VC_GLOBAL uint32_t *>(Cp + off) ^
                          *reinterpret_cast<const VC_GLOBAL uint32_t *>(Bp + off);
            }
        }
    }

    // Phase 0: distances (column distances for k = 0..wt, the last being
    // column je).
    for (uint32_t it = threadIdx.x; it < 3 * h; it += NT) dhS[it] = mod_u16(D[it], geo.mod_W8);
    for (uint32_t it = threadIdx.x; it < 3 * (wt + 1); it += NT) {
        const uint32_t c = it / (wt + 1), k = it - c * (wt + 1);
        const uint32_t j = (k < wt) ? j0 + k : je;
        dvS[c * CS + k] = mod_u16(D[3 * h + c * w + j], geo.mod_h);
    }
    __syncthreads();

    // Phase 1: Y = C ^ B; undo Eq. 3: S[(i - d_v) mod h][c][k] = Y[i][j0+k][c].
    if (aligned) {
        if (p1) {
            uint32_t addr[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const uint32_t p = 4 * g + m, k = p / 3, c = p - 3 * k;
                const uint32_t dv = dvS[c * CS + k];
                const uint32_t r = (i0 >= dv) ? i0 - dv : i0 + h - dv;
                addr[m] = r * RS + c * CS + k;
            }
            const uint32_t step = RP % h;
            const uint32_t stepA = step * RS, wrapA = h * RS;
            auto scatter = [&](uint32_t y) {
                S[addr[0]] = static_cast<uint8_t>(y);
                S[addr[1]] = static_cast<uint8_t>(y >> 8);
                S[addr[2]] = static_cast<uint8_t>(y >> 16);
                S[addr[3]] = static_cast<uint8_t>(y >> 24);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    addr[m] += stepA;
                    if (addr[m] >= wrapA) addr[m] -= wrapA;
                }
            };
#pragma unroll
            for (uint32_t k = 0; k < kPrefetchRows; ++k)
                if (i0 + k * RP < h) scatter(ypre[k]);
            for (uint32_t i = i0 + kPrefetchRows * RP; i < h; i += RP) {
                const uint64_t off = static_cast<uint64_t>(i) * row_bytes + 4 * g;
                scatter(*reinterpret_cast<const VC_GLOBAL uint32_t *>(Cp + off) ^
                        *reinterpret_cast<const VC_GLOBAL uint32_t *>(Bp + off));
            }
        }
    } else {
        const uint32_t rowlen = 3 * wt;
        const uint32_t items = h * rowlen;
        for (uint32_t it = threadIdx.x; it < items; it += NT) {
            const uint32_t i = it / rowlen, p = it - i * rowlen;
            const uint32_t k = p / 3, c = p - 3 * k;
            const uint32_t dv = dvS[c * CS + k];
            const uint32_t r = (i >= dv) ? i - dv : i + h - dv;
            const uint64_t off = static_cast<uint64_t>(i) * row_bytes + p;
            S[r * RS + c * CS + k] = Cp[off] ^ Bp[off];
        }
    }
    {   // the column after the strip, stored at k = wt
        const VC_GLOBAL uint8_t *Ce = gmem(d.in) + 3 * je;
        const VC_GLOBAL uint8_t *Be = gmem(d.B) + 3 * je;
        for (uint32_t it = threadIdx.x; it < 3 * h; it += NT) {
            const uint32_t i = it / 3, c = it - 3 * i;
            const uint32_t dv = dvS[c * CS + wt];
            const uint32_t r = (i >= dv) ? i - dv : i + h - dv;
            const uint64_t off = static_cast<uint64_t>(i) * row_bytes + c;
            S[r * RS + c * CS + wt] = Ce[off] ^ Be[off];
        }
    }
    __syncthreads();

    // Phase 2: undo Eq. 2.  With a = (d_h mod 8w) >> 3 and t = d_h & 7,
    // plaintext pixel q = (j0 + k - a) mod w of row r, channel c is the
    // funnel shift of strip columns k and k+1 by t.  One byte per lane, so
    // the lanes of a wave store adjacent pixels of one row.
    const uint32_t items2 = h * 3 * WT;
    for (uint32_t it = threadIdx.x; it < items2; it += NT) {
        const uint32_t k = it % WT, rc = it / WT;
        if (k >= wt) continue;
        const uint32_t r = rc / 3, c = rc - 3 * r;
        const uint32_t dh = dhS[c * h + r];
        const uint32_t a = dh >> 3, t = dh & 7;
        uint32_t q = j0 + k + w - a;
        if (q >= w) q -= w;
        const uint8_t *src = S + r * RS + c * CS + k;
        const uint32_t X = static_cast<uint32_t>(src[0]) | (static_cast<uint32_t>(src[1]) << 8);
        Pout[static_cast<uint64_t>(r) * row_bytes + 3 * q + c] = static_cast<uint8_t>(X >> t);
    }
}

constexpr uint32_t kStrips[] = {4, 8, 16, 32, 64};
constexpr uint32_t kThreads[] = {256, 512, 1024};

template <int WT, int NT>
hipError_t launch_one(int decrypt, const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g,
                      bool aligned, int xcd_map, hipStream_t s) {
    const uint32_t nstrips = (g.w + WT - 1) / WT;
    const uint64_t groups =
        xcd_map ? 8ull * ((count + 7) / 8) * nstrips : static_cast<uint64_t>(count) * nstrips;
    if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const uint32_t lds = confuse_lds_bytes(decrypt, g.h, WT);
    if (decrypt)
        hipLaunchKernelGGL((confuse_xor_dec<WT, NT>), dim3(static_cast<uint32_t>(groups)), dim3(NT), lds, s,
                           d_desc, first, count, g, nstrips, xcd_map, aligned ? 1 : 0);
    else
        hipLaunchKernelGGL((confuse_xor_enc<WT, NT>), dim3(static_cast<uint32_t>(groups)), dim3(NT), lds, s,
                           d_desc, first, count, g, nstrips, xcd_map, aligned ? 1 : 0);
    return hipGetLastError();
}

template <int WT>
hipError_t launch_wt(int decrypt, const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g,
                     bool aligned, const ConfuseTuning &t, hipStream_t s) {
    switch (t.threads) {
    case 256: return launch_one<WT, 256>(decrypt, d_desc, first, count, g, aligned, t.xcd_map, s);
    case 1024: return launch_one<WT, 1024>(decrypt, d_desc, first, count, g, aligned, t.xcd_map, s);
    default: return launch_one<WT, 512>(decrypt, d_desc, first, count, g, aligned, t.xcd_map, s);
    }
}

template <int WT, int NT>
hipError_t set_lds_attr(uint32_t limit) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&confuse_xor_enc<WT, NT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(limit));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&confuse_xor_dec<WT, NT>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(limit));
}

template <int WT>
hipError_t set_lds_attr_wt(uint32_t limit) {
    hipError_t e = set_lds_attr<WT, 256>(limit);
    if (e == hipSuccess) e = set_lds_attr<WT, 512>(limit);
    if (e == hipSuccess) e = set_lds_attr<WT, 1024>(limit);
    return e;
}

}  // namespace

uint32_t confuse_lds_bytes(int decrypt, uint32_t h, uint32_t strip) {
    switch (strip) {
    case 4: return decrypt ? DecLayout<4>::bytes(h) : EncLayout<4>::bytes(h);
    case 8: return decrypt ? DecLayout<8>::bytes(h) : EncLayout<8>::bytes(h);
    case 16: return decrypt ? DecLayout<16>::bytes(h) : EncLayout<16>::bytes(h);
    case 32: return decrypt ? DecLayout<32>::bytes(h) : EncLayout<32>::bytes(h);
    case 64: return decrypt ? DecLayout<64>::bytes(h) : EncLayout<64>::bytes(h);
    default: return 0xFFFFFFFFu;
    }
}

uint32_t confuse_max_strip(int decrypt, uint32_t h, uint32_t lds_bytes) {
    uint32_t best = 0;
    for (uint32_t wt : kStrips)
        if (static_cast<uint64_t>(confuse_lds_bytes(decrypt, h, wt)) <= lds_bytes) best = wt;
    return best;
}

hipError_t confuse_configure(uint32_t lds_limit) {
    hipError_t e = set_lds_attr_wt<4>(lds_limit);
    if (e == hipSuccess) e = set_lds_attr_wt<8>(lds_limit);
    if (e == hipSuccess) e = set_lds_attr_wt<16>(lds_limit);
    if (e == hipSuccess) e = set_lds_attr_wt<32>(lds_limit);
    if (e == hipSuccess) e = set_lds_attr_wt<64>(lds_limit);
    return e;
}

hipError_t launch_confuse(int decrypt, const FrameDesc *d_desc, uint32_t first, uint32_t count, uint32_t w,
                          uint32_t h, bool aligned, const ConfuseTuning &t, hipStream_t s) {
    if (count == 0) return hipSuccess;
    Geometry g;
    g.w = w;
    g.h = h;
    g.W8 = 8 * w;
    g.row_bytes = 3 * w;
    g.mod_h = mod_magic(h);
    g.mod_W8 = mod_magic(g.W8);
    switch (t.strip) {
    case 4: return launch_wt<4>(decrypt, d_desc, first, count, g, aligned, t, s);
    case 8: return launch_wt<8>(decrypt, d_desc, first, count, g, aligned, t, s);
    case 16: return launch_wt<16>(decrypt, d_desc, first, count, g, aligned, t, s);
    case 32: return launch_wt<32>(decrypt, d_desc, first, count, g, aligned, t, s);
    case 64: return launch_wt<64>(decrypt, d_desc, first, count, g, aligned, t, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace vc
