// vc_shift.hip -- the confusion of Sec. II-C (Eq. 2 row shifts, Eq. 3 column
// shifts) fused with the XOR round, and its exact inverse, as two passes
// that each touch HBM only with coalesced, aligned accesses:
//
//   encrypt:  S = rows of P shifted by d_h          (row pass,    6 B/px)
//             C = columns of S shifted by d_v, ^ B  (column pass, 9 B/px)
//   decrypt:  T = columns of (C ^ B) unshifted      (column pass, 9 B/px)
//             P = rows of T unshifted               (row pass,    6 B/px)
//
// For output byte (i, j, c) (row i, pixel column j, channel c) with
// d_h = D[c*h + r] mod 8w and d_v = D[3h + c*w + j] mod h:
//     S[r][j][c] = bits s..s+7 of row r, channel c, s = (8j - d_h) mod 8w
//     C[i][j][c] = S[(i - d_v) mod h][j][c] ^ B[i][j][c]
// where "bits s..s+7" is the funnel shift of pixels s/8 and s/8+1 (mod w),
// least significant bit first (Algs. 3 and 7).  The inverse undoes the
// column rotation (row (r + d_v) mod h) and then the row rotation
// (s = (8j + d_h) mod 8w).
//
// A row shift needs a whole row and a column shift a whole column, so a
// single pass must fetch a randomly placed window of every source row per
// channel (encrypt) or scatter bytes of three channels to random places of
// every output row (decrypt, partial-line writes).  Two passes move 15 B/px
// instead of the 9 B/px minimum but never fetch or write a partial line.
#include "vc_internal.hpp"

namespace vc {
namespace {

__device__ __forceinline__ uint32_t mod16(uint32_t x, uint32_t m, float inv_m) {
    const uint32_t q = static_cast<uint32_t>(static_cast<float>(x) * inv_m);
    int32_t r = static_cast<int32_t>(x) - static_cast<int32_t>(q * m);
    if (r < 0) r += static_cast<int32_t>(m);
    if (r >= static_cast<int32_t>(m)) r -= static_cast<int32_t>(m);
    return static_cast<uint32_t>(r);
}

// Workgroup -> (frame within the launch, strip), all strips of a frame on
// one XCD (the hardware places consecutive workgroups round-robin on the 8
// XCDs), so that neighbouring strips' partial cache lines meet in one L2.
__device__ __forceinline__ void map_strip(uint32_t g, uint32_t nstrips, int xcd_map, uint32_t &fl, uint32_t &strip) {
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

// ----------------------------------------------------------------------
// Row pass
// ----------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kRowThreads = 256;
constexpr uint32_t kRowsPerGroup = 4;
constexpr uint32_t kRowShiftTable = 16 * kRowsPerGroup;  // LDS bytes of the rows' shift amounts

// Four output bytes (pixels 4m..4m+3) of one channel: bits s..s+31 of the
// channel's bit row, from source pixels q..q+4 (mod w).  `row` is the source
// row (LDS or global), byte c of pixel 0.
template <typename Ptr>
__device__ __forceinline__ uint32_t shifted4(Ptr row, uint32_t s, uint32_t w) {
    const uint32_t q = s >> 3, t = s & 7;
    uint32_t b[5];
    if (q + 4 < w) {
#pragma unroll
        for (int k = 0; k < 5; ++k) b[k] = row[3 * (q + k)];
    } else {
        uint32_t qq = q;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            b[k] = row[3 * qq];
            qq = (qq + 1 == w) ? 0 : qq + 1;
        }
    }
    const uint32_t X = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
    return __builtin_amdgcn_alignbit(b[4], X, t);
}

// Pixels 4m..4m+3 of all three channels of one row: twelve bytes (pixel k,
// channel c at byte 3k + c), stored as three dwords when aligned.
template <typename Ptr>
__device__ __forceinline__ void shift_group(Ptr row, VC_GLOBAL uint8_t *piece, const uint32_t sh[3], uint32_t m,
                                            uint32_t w, uint32_t W8, int aligned) {
    uint32_t o[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        uint32_t s = 32 * m + sh[c];  // 32m < 8w, sh < 8w
        if (s >= W8) s -= W8;
        o[c] = shifted4(row + c, s, w);
    }
    const uint32_t d0 = (o[0] & 0xFFu) | ((o[1] & 0xFFu) << 8) | ((o[2] & 0xFFu) << 16) | (o[0] << 16 & 0xFF000000u);
    const uint32_t d1 = ((o[1] >> 8) & 0xFFu) | (o[2] & 0xFF00u) | (o[0] & 0xFF0000u) | ((o[1] << 8) & 0xFF000000u);
    const uint32_t d2 = ((o[2] >> 16) & 0xFFu) | ((o[0] >> 16) & 0xFF00u) | ((o[1] >> 8) & 0xFF0000u) | (o[2] & 0xFF000000u);
    if (aligned && 4 * m + 4 <= w) {
        VC_GLOBAL uint32_t *q4 = reinterpret_cast<VC_GLOBAL uint32_t *>(piece);
        q4[0] = d0;
        q4[1] = d1;
        q4[2] = d2;
    } else {
        const uint32_t dw[3] = {d0, d1, d2};
        const uint32_t nb = 3 * ((w - 4 * m < 4) ? w - 4 * m : 4);
        for (uint32_t b = 0; b < nb; ++b) piece[b] = static_cast<uint8_t>(dw[b >> 2] >> (8 * (b & 3)));
    }
}

__device__ __forceinline__ void row_shifts(const VC_GLOBAL uint16_t *D, uint32_t r, uint32_t h, const Geometry &geo,
                                           bool inv, uint32_t sh[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const uint32_t dh = mod16(D[c * h + r], geo.W8, geo.inv_W8);
        sh[c] = inv ? dh : (dh ? geo.W8 - dh : 0);
    }
}

// One workgroup shifts kRowsPerGroup rows of one frame.  Output byte j of
// channel c takes bits s..s+7 with s = 8j + sh[c] (mod 8w), sh = 8w - d_h
// (forward) or d_h (inverse).  A thread produces pixels 4m..4m+3 of all
// three channels (twelve bytes) at a time.  With STAGE all rows of the
// workgroup are first copied to LDS at once (16-byte loads when rows and
// pointers allow, so that many bytes are in flight), then shifted from
// there; otherwise (rows too long for LDS) bytes are read from global
// memory row by row.
template <bool INV, bool STAGE>
__global__ __launch_bounds__(kRowThreads) void row_shift(const FrameDesc *__restrict__ desc, uint32_t first,
                                                       uint32_t nframes, Geometry geo, uint32_t groups_per_frame,
                                                       int aligned, uint32_t lds_row) {
    extern __shared__ __align__(16) uint8_t rowbuf[];
    const uint32_t fl = blockIdx.x / groups_per_frame, grp = blockIdx.x - fl * groups_per_frame;
    if (fl >= nframes) return;
    const FrameDesc d = desc[first + fl];
    const uint32_t w = geo.w, h = geo.h, W8 = geo.W8, rb = geo.row_bytes;
    const VC_GLOBAL uint8_t *__restrict__ src = gmem(INV ? d.X : d.in);
    VC_GLOBAL uint8_t *__restrict__ dst = gmem(INV ? d.out : d.X);
    const VC_GLOBAL uint16_t *__restrict__ D = gmem(d.D);
    const uint32_t ngroups = (w + 3) / 4;
    const uint32_t r0 = grp * kRowsPerGroup;
    const uint32_t nr = (h - r0 < kRowsPerGroup) ? h - r0 : kRowsPerGroup;
    if (STAGE) {
        // the rows' shift amounts sit after the rows
        uint32_t(*shS)[3] = reinterpret_cast<uint32_t(*)[3]>(rowbuf + kRowsPerGroup * lds_row);
        if (threadIdx.x < nr) row_shifts(D, r0 + threadIdx.x, h, geo, INV, shS[threadIdx.x]);
        // strip-major X (the host sets it only for aligned rows whose width
        // is a multiple of the strip): decryption reads T from the strips'
        // runs of nr rows, encryption writes S to them
        const uint32_t xs = d.xstrip, RSx = 3 * xs;
        const bool x_sm = xs != 0;
        if (INV && x_sm) {
            const uint32_t nstr = w / xs;
            const uint64_t run0 = static_cast<uint64_t>(r0) * RSx;
            if (RSx % 16 == 0) {
                const uint32_t per = RSx / 16, per_strip = nr * per, n16 = nstr * per_strip;
                for (uint32_t k = threadIdx.x; k < n16; k += kRowThreads) {
                    const uint32_t st = k / per_strip, within = k - st * per_strip;
                    const uint32_t rr = within / per, e = within - rr * per;
                    const uint64_t goff = static_cast<uint64_t>(st) * h * RSx + run0 + static_cast<uint64_t>(within) * 16;
                    *reinterpret_cast<u32x4 *>(rowbuf + rr * lds_row + st * RSx + 16 * e) =
                        *reinterpret_cast<const VC_GLOBAL u32x4 *>(src + goff);
                }
            } else {
                const uint32_t per = RSx / 4, per_strip = nr * per, n4 = nstr * per_strip;
                for (uint32_t k = threadIdx.x; k < n4; k += kRowThreads) {
                    const uint32_t st = k / per_strip, within = k - st * per_strip;
                    const uint32_t rr = within / per, e = within - rr * per;
                    const uint64_t goff = static_cast<uint64_t>(st) * h * RSx + run0 + static_cast<uint64_t>(within) * 4;
                    *reinterpret_cast<uint32_t *>(rowbuf + rr * lds_row + st * RSx + 4 * e) =
                        *reinterpret_cast<const VC_GLOBAL uint32_t *>(src + goff);
                }
            }
        } else {
            const VC_GLOBAL uint8_t *s0 = src + static_cast<uint64_t>(r0) * rb;
            const bool v16 = aligned && (rb % 16 == 0) && ((reinterpret_cast<uintptr_t>(src) & 15) == 0);
            if (v16) {
                // the rows are contiguous: nr * rb / 16 uint4, row k at LDS offset k * lds_row
                const uint32_t per = rb / 16, n16 = nr * per;
                for (uint32_t k = threadIdx.x; k < n16; k += kRowThreads) {
                    const uint32_t rr = k / per, e = k - rr * per;
                    reinterpret_cast<u32x4 *>(rowbuf + rr * lds_row)[e] =
                        reinterpret_cast<const VC_GLOBAL u32x4 *>(s0)[k];
                }
            } else if (aligned) {
                const uint32_t per = rb / 4, n4 = nr * per;
                for (uint32_t k = threadIdx.x; k < n4; k += kRowThreads) {
                    const uint32_t rr = k / per, e = k - rr * per;
                    reinterpret_cast<uint32_t *>(rowbuf + rr * lds_row)[e] =
                        reinterpret_cast<const VC_GLOBAL uint32_t *>(s0)[k];
                }
            } else {
                const uint32_t n1 = nr * rb;
                for (uint32_t k = threadIdx.x; k < n1; k += kRowThreads) {
                    const uint32_t rr = k / rb, e = k - rr * rb;
                    rowbuf[rr * lds_row + e] = s0[k];
                }
            }
        }
        __syncthreads();
        if (!INV && x_sm) {
            // lanes in output order: strip, row, 12-byte piece, so that a wave
            // writes whole runs of nr rows of consecutive strips
            const uint32_t pps = xs / 4, per_strip = nr * pps, nt = (w / xs) * per_strip;
            for (uint32_t t = threadIdx.x; t < nt; t += kRowThreads) {
                const uint32_t st = t / per_strip, within = t - st * per_strip;
                const uint32_t rr = within / pps, kk = within - rr * pps;
                const uint32_t sh[3] = {shS[rr][0], shS[rr][1], shS[rr][2]};
                VC_GLOBAL uint8_t *piece = dst + static_cast<uint64_t>(st) * h * RSx +
                                           static_cast<uint64_t>(r0 + rr) * RSx + 12 * kk;
                shift_group(rowbuf + rr * lds_row, piece, sh, st * pps + kk, w, W8, aligned);
            }
        } else {
            for (uint32_t k = threadIdx.x; k < nr * ngroups; k += kRowThreads) {
                const uint32_t rr = k / ngroups, m = k - rr * ngroups;
                const uint32_t sh[3] = {shS[rr][0], shS[rr][1], shS[rr][2]};
                shift_group(rowbuf + rr * lds_row, dst + static_cast<uint64_t>(r0 + rr) * rb + 12 * m, sh, m, w, W8,
                            aligned);
            }
        }
    } else {
        for (uint32_t rr = 0; rr < nr; ++rr) {
            const uint32_t r = r0 + rr;
            uint32_t sh[3];
            row_shifts(D, r, h, geo, INV, sh);
            const VC_GLOBAL uint8_t *srow = src + static_cast<uint64_t>(r) * rb;
            VC_GLOBAL uint8_t *drow = dst + static_cast<uint64_t>(r) * rb;
            for (uint32_t m = threadIdx.x; m < ngroups; m += kRowThreads)
                shift_group(srow, drow + 12 * m, sh, m, w, W8, aligned);
        }
    }
}

// ----------------------------------------------------------------------
// Column pass
// ----------------------------------------------------------------------
// LDS: the strip (h rows of 3*WT bytes), then the strip's column distances
// d_v mod h (3 x WT words).
template <int WT>
struct ColLayout {
    static constexpr uint32_t RS = 3 * WT;
    __host__ __device__ static uint32_t dv_off(uint32_t h) { return (h * RS + 15u) & ~15u; }
    __host__ __device__ static uint32_t bytes(uint32_t h) { return dv_off(h) + 4 * 3 * WT; }
};

// One workgroup owns a full-height strip of WT pixel columns (all three
// channels) of one frame.  Forward: stage S, then C[i] = S[(i - d_v) mod h]
// ^ B[i].  Inverse: stage C ^ B, then T[r] = (C ^ B)[(r + d_v) mod h].
// Aligned path: dword loads and stores (w % 4 == 0, 4-byte aligned frames);
// otherwise bytes.
template <int WT, int NT, bool INV>
__global__ __launch_bounds__(NT) void col_shift(const FrameDesc *__restrict__ desc, uint32_t first, uint32_t nframes,
                                                Geometry geo, uint32_t nstrips, int xcd_map, int aligned) {
    extern __shared__ __align__(16) uint8_t smem[];
    using Lay = ColLayout<WT>;
    constexpr uint32_t RS = Lay::RS;
    constexpr uint32_t GPR = 3 * WT / 4;  // dwords per full strip row
    constexpr uint32_t RP = NT / GPR;     // rows per pass
    constexpr uint32_t kUnroll = 8;       // staging passes in flight per thread

    uint32_t fl, strip;
    map_strip(blockIdx.x, nstrips, xcd_map, fl, strip);
    if (fl >= nframes) return;
    const FrameDesc d = desc[first + fl];
    const uint32_t w = geo.w, h = geo.h, rb = geo.row_bytes;
    const uint32_t j0 = strip * WT;
    const uint32_t wt = (w - j0 < static_cast<uint32_t>(WT)) ? w - j0 : WT;
    // Each operand is addressed as base + row * stride: row-major (the
    // strip's columns of each frame row) or, for the intermediate image X,
    // strip-major (the strip's rows contiguous, stride 3*WT; the host sets
    // that layout only when its strip width is this kernel's WT and the rows
    // are aligned).
    const bool x_sm = d.xstrip != 0;
    const uint64_t sm_base = static_cast<uint64_t>(strip) * h * RS;
    const VC_GLOBAL uint8_t *__restrict__ in =
        INV ? gmem(d.in) + 3 * j0 : gmem(d.X) + (x_sm ? sm_base : 3 * j0);
    const uint32_t in_stride = (!INV && x_sm) ? RS : rb;
    const VC_GLOBAL uint8_t *__restrict__ Bp = gmem(d.B) + 3 * j0;
    const uint32_t b_stride = rb;
    VC_GLOBAL uint8_t *__restrict__ out = INV ? gmem(d.X) + (x_sm ? sm_base : 3 * j0) : gmem(d.out) + 3 * j0;
    const uint32_t out_stride = (INV && x_sm) ? RS : rb;
    const VC_GLOBAL uint16_t *__restrict__ D = gmem(d.D);
    uint8_t *S = smem;
    uint32_t *dvS = reinterpret_cast<uint32_t *>(smem + Lay::dv_off(h));

    for (uint32_t it = threadIdx.x; it < 3 * wt; it += NT) {
        const uint32_t c = it / wt, k = it - c * wt;
        const uint32_t dv = mod16(D[3 * h + c * w + j0 + k], h, geo.inv_h);
        dvS[c * WT + k] = INV ? (dv ? h - dv : 0) : dv;  // source row = (i + h - dvS) mod h, forward and inverse
    }

    const uint32_t g = threadIdx.x % GPR, i0 = threadIdx.x / GPR;
    const bool lane_on = aligned && i0 < RP && g < 3 * wt / 4;
    if (aligned) {
        if (!INV && x_sm && (static_cast<uint64_t>(h) * RS) % 16 == 0) {
            // the strip of S is h*RS contiguous bytes, 16-byte aligned: a
            // linear copy into LDS by every thread
            const uint32_t n16 = h * RS / 16;
            const VC_GLOBAL u32x4 *in4 = reinterpret_cast<const VC_GLOBAL u32x4 *>(in);
            u32x4 *S4 = reinterpret_cast<u32x4 *>(S);
            for (uint32_t k0 = threadIdx.x; k0 < n16; k0 += 4 * NT) {
                u32x4 v[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u)
                    if (k0 + u * NT < n16) v[u] = in4[k0 + u * NT];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u)
                    if (k0 + u * NT < n16) S4[k0 + u * NT] = v[u];
            }
        } else if (lane_on) {
            // stage: S row i, dword g  <-  in[i][g] (^ B[i][g] when inverse)
            for (uint32_t base = i0; base < h; base += kUnroll * RP) {
                uint32_t v[kUnroll], b[kUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    const uint32_t i = base + u * RP;
                    if (i < h) {
                        v[u] = *reinterpret_cast<const VC_GLOBAL uint32_t *>(in + static_cast<uint64_t>(i) * in_stride +
                                                                              4 * g);
                        if (INV)
                            b[u] = *reinterpret_cast<const VC_GLOBAL uint32_t *>(
                                Bp + static_cast<uint64_t>(i) * b_stride + 4 * g);
                    }
                }
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    const uint32_t i = base + u * RP;
                    if (i < h) reinterpret_cast<uint32_t *>(S + i * RS)[g] = INV ? (v[u] ^ b[u]) : v[u];
                }
            }
        }
        __syncthreads();
        if (lane_on) {
            uint32_t addr[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const uint32_t p = 4 * g + m, k = p / 3, c = p - 3 * k;
                const uint32_t dv = dvS[c * WT + k];
                const uint32_t r = (i0 >= dv) ? i0 - dv : i0 + h - dv;
                addr[m] = r * RS + p;  // the strip is staged in frame byte order
            }
            const uint32_t stepA = (RP % h) * RS, wrapA = h * RS;
            const uint64_t bstep = static_cast<uint64_t>(RP) * b_stride, ostep = static_cast<uint64_t>(RP) * out_stride;
            uint64_t boff = static_cast<uint64_t>(i0) * b_stride + 4 * g;
            uint64_t ooff = static_cast<uint64_t>(i0) * out_stride + 4 * g;
            for (uint32_t base = i0; base < h; base += kUnroll * RP) {
                uint32_t b[kUnroll];
                if (!INV) {
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u)
                        if (base + u * RP < h)
                            b[u] = *reinterpret_cast<const VC_GLOBAL uint32_t *>(Bp + boff + u * bstep);
                }
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    if (base + u * RP < h) {
                        uint32_t v = static_cast<uint32_t>(S[addr[0]]) | (static_cast<uint32_t>(S[addr[1]]) << 8) |
                                     (static_cast<uint32_t>(S[addr[2]]) << 16) |
                                     (static_cast<uint32_t>(S[addr[3]]) << 24);
                        if (!INV) v ^= b[u];
                        *reinterpret_cast<VC_GLOBAL uint32_t *>(out + ooff + u * ostep) = v;
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            addr[m] += stepA;
                            if (addr[m] >= wrapA) addr[m] -= wrapA;
                        }
                    }
                }
                boff += kUnroll * bstep;
                ooff += kUnroll * ostep;
            }
        }
    } else {
        const uint32_t rowlen = 3 * wt;
        for (uint32_t it = threadIdx.x; it < h * rowlen; it += NT) {
            const uint32_t i = it / rowlen, p = it - i * rowlen;
            const uint8_t v = in[static_cast<uint64_t>(i) * in_stride + p];
            S[i * RS + p] = INV ? (v ^ Bp[static_cast<uint64_t>(i) * b_stride + p]) : v;
        }
        __syncthreads();
        for (uint32_t it = threadIdx.x; it < h * rowlen; it += NT) {
            const uint32_t i = it / rowlen, p = it - i * rowlen;
            const uint32_t k = p / 3, c = p - 3 * k;
            const uint32_t dv = dvS[c * WT + k];
            const uint32_t r = (i >= dv) ? i - dv : i + h - dv;
            const uint8_t v = S[r * RS + p];
            out[static_cast<uint64_t>(i) * out_stride + p] =
                INV ? v : static_cast<uint8_t>(v ^ Bp[static_cast<uint64_t>(i) * b_stride + p]);
        }
    }
}

constexpr uint32_t kColStrips[] = {4, 8, 16, 32, 64};

template <int WT, int NT, bool INV>
hipError_t launch_col_one(const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g, bool aligned,
                          int xcd_map, hipStream_t s) {
    const uint32_t nstrips = (g.w + WT - 1) / WT;
    const uint64_t groups =
        xcd_map ? 8ull * ((count + 7) / 8) * nstrips : static_cast<uint64_t>(count) * nstrips;
    if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((col_shift<WT, NT, INV>), dim3(static_cast<uint32_t>(groups)), dim3(NT),
                       ColLayout<WT>::bytes(g.h), s, d_desc, first, count, g, nstrips, xcd_map, aligned ? 1 : 0);
    return hipGetLastError();
}

template <int WT, bool INV>
hipError_t launch_col_wt(const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g, bool aligned,
                         const ConfuseTuning &t, hipStream_t s) {
    switch (t.threads) {
    case 256: return launch_col_one<WT, 256, INV>(d_desc, first, count, g, aligned, t.xcd_map, s);
    case 512: return launch_col_one<WT, 512, INV>(d_desc, first, count, g, aligned, t.xcd_map, s);
    default: return launch_col_one<WT, 1024, INV>(d_desc, first, count, g, aligned, t.xcd_map, s);
    }
}

template <bool INV>
hipError_t launch_col(const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g, bool aligned,
                      const ConfuseTuning &t, hipStream_t s) {
    switch (t.strip) {
    case 4: return launch_col_wt<4, INV>(d_desc, first, count, g, aligned, t, s);
    case 8: return launch_col_wt<8, INV>(d_desc, first, count, g, aligned, t, s);
    case 16: return launch_col_wt<16, INV>(d_desc, first, count, g, aligned, t, s);
    case 32: return launch_col_wt<32, INV>(d_desc, first, count, g, aligned, t, s);
    case 64: return launch_col_wt<64, INV>(d_desc, first, count, g, aligned, t, s);
    default: return hipErrorInvalidValue;
    }
}

template <bool INV>
hipError_t launch_row(const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g, bool aligned,
                      uint32_t lds_limit, hipStream_t s) {
    const uint32_t per_frame = (g.h + kRowsPerGroup - 1) / kRowsPerGroup;
    const uint64_t groups = static_cast<uint64_t>(count) * per_frame;
    if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const uint32_t lds_row = (g.row_bytes + 15u) & ~15u;
    const uint64_t lds = static_cast<uint64_t>(kRowsPerGroup) * lds_row + kRowShiftTable;
    if (lds <= lds_limit)
        hipLaunchKernelGGL((row_shift<INV, true>), dim3(static_cast<uint32_t>(groups)), dim3(kRowThreads),
                           static_cast<uint32_t>(lds), s, d_desc, first, count, g, per_frame, aligned ? 1 : 0,
                           lds_row);
    else
        hipLaunchKernelGGL((row_shift<INV, false>), dim3(static_cast<uint32_t>(groups)), dim3(kRowThreads), 0, s,
                           d_desc, first, count, g, per_frame, aligned ? 1 : 0, lds_row);
    return hipGetLastError();
}

template <int WT, int NT>
hipError_t set_col_attr(uint32_t limit) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&col_shift<WT, NT, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(limit));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&col_shift<WT, NT, true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(limit));
}

template <int WT>
hipError_t set_col_attr_wt(uint32_t limit) {
    hipError_t e = set_col_attr<WT, 256>(limit);
    if (e == hipSuccess) e = set_col_attr<WT, 512>(limit);
    if (e == hipSuccess) e = set_col_attr<WT, 1024>(limit);
    return e;
}

}  // namespace

uint32_t shift_col_lds_bytes(uint32_t h, uint32_t strip) {
    switch (strip) {
    case 4: return ColLayout<4>::bytes(h);
    case 8: return ColLayout<8>::bytes(h);
    case 16: return ColLayout<16>::bytes(h);
    case 32: return ColLayout<32>::bytes(h);
    case 64: return ColLayout<64>::bytes(h);
    default: return 0xFFFFFFFFu;
    }
}

bool shift_rows_staged(uint32_t w, uint32_t lds_bytes) {
    const uint64_t lds_row = (3ull * w + 15u) & ~15ull;
    return kRowsPerGroup * lds_row + kRowShiftTable <= lds_bytes;
}

uint32_t shift_max_strip(uint32_t h, uint32_t lds_bytes) {
    uint32_t best = 0;
    for (uint32_t wt : kColStrips)
        if (static_cast<uint64_t>(shift_col_lds_bytes(h, wt)) <= lds_bytes) best = wt;
    return best;
}

hipError_t shift_configure(uint32_t lds_limit) {
    hipError_t e = set_col_attr_wt<4>(lds_limit);
    if (e == hipSuccess) e = set_col_attr_wt<8>(lds_limit);
    if (e == hipSuccess) e = set_col_attr_wt<16>(lds_limit);
    if (e == hipSuccess) e = set_col_attr_wt<32>(lds_limit);
    if (e == hipSuccess) e = set_col_attr_wt<64>(lds_limit);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&row_shift<false, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_limit));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&row_shift<true, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_limit));
    return e;
}

hipError_t launch_shift(int decrypt, int pass, const FrameDesc *d_desc, uint32_t first, uint32_t count, uint32_t w,
                        uint32_t h, bool aligned, const ConfuseTuning &t, uint32_t lds_limit, hipStream_t s) {
    if (count == 0) return hipSuccess;
    Geometry g;
    g.w = w;
    g.h = h;
    g.W8 = 8 * w;
    g.row_bytes = 3 * w;
    g.inv_h = 1.0f / static_cast<float>(h);
    g.inv_W8 = 1.0f / static_cast<float>(g.W8);
    // encrypt: pass 0 = rows, pass 1 = columns; decrypt: pass 0 = columns, pass 1 = rows
    const bool rows = decrypt ? pass == 1 : pass == 0;
    if (rows)
        return decrypt ? launch_row<true>(d_desc, first, count, g, aligned, lds_limit, s)
                       : launch_row<false>(d_desc, first, count, g, aligned, lds_limit, s);
    return decrypt ? launch_col<true>(d_desc, first, count, g, aligned, t, s)
                   : launch_col<false>(d_desc, first, count, g, aligned, t, s);
}

}  // namespace vc
