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
//
// The column rotation moves each byte column k = 3j + c of the 3w-byte rows
// on its own (by d_v(c, j)); it does not care where pixels begin.  So the
// column pass cuts the rows into strips of SB bytes (a power of two, up to
// 128 = one cache line), not of whole pixels: with rows of a multiple of 16
// bytes, every row segment of the frame, of B and of the output is then
// whole 16-byte words, and at SB = 128 (1080p: a full-height strip is
// 1080 x 128 bytes of LDS) every HBM access of both passes covers whole
// 128-byte lines.  The intermediate image is stored strip-major in those
// strips (FrameDesc::xstrip), so the column pass stages (encrypt) or writes
// (decrypt) a strip as one contiguous block.
#include "vc_internal.hpp"

namespace vc {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

// Workgroup -> (frame within the launch, strip), all strips of a frame on
// one XCD (the hardware places consecutive workgroups round-robin on the 8
// XCDs), so that neighbouring strips' accesses meet in one L2.
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
constexpr uint32_t kRowThreads = 256;
constexpr uint32_t kRowsPerGroup = 4;
constexpr uint32_t kRowShiftTable = 16 * kRowsPerGroup;  // LDS bytes of the rows' shift amounts
constexpr uint32_t kStageLoads = 6;  // staging loads in flight per thread (4 1080p rows: 5.6 per thread)

// Copies n16 16-byte words into LDS, kStageLoads loads in flight per
// thread: src(k) is the global address of word k, dst(k) its LDS address.
template <typename Src, typename Dst>
__device__ __forceinline__ void stage16(uint32_t n16, Src src, Dst dst) {
    for (uint32_t k0 = threadIdx.x; k0 < n16; k0 += kStageLoads * kRowThreads) {
        u32x4 v[kStageLoads];
#pragma unroll
        for (uint32_t u = 0; u < kStageLoads; ++u)
            if (k0 + u * kRowThreads < n16) v[u] = *src(k0 + u * kRowThreads);
#pragma unroll
        for (uint32_t u = 0; u < kStageLoads; ++u)
            if (k0 + u * kRowThreads < n16) *dst(k0 + u * kRowThreads) = v[u];
    }
}

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
// channel c at byte 3k + c), as three dwords.
template <typename Ptr>
__device__ __forceinline__ void shift12(Ptr row, const uint32_t sh[3], uint32_t m, uint32_t w, uint32_t W8,
                                        uint32_t dw[3]) {
    uint32_t o[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        uint32_t s = 32 * m + sh[c];  // 32m < 8w, sh < 8w
        if (s >= W8) s -= W8;
        o[c] = shifted4(row + c, s, w);
    }
    dw[0] = (o[0] & 0xFFu) | ((o[1] & 0xFFu) << 8) | ((o[2] & 0xFFu) << 16) | (o[0] << 16 & 0xFF000000u);
    dw[1] = ((o[1] >> 8) & 0xFFu) | (o[2] & 0xFF00u) | (o[0] & 0xFF0000u) | ((o[1] << 8) & 0xFF000000u);
    dw[2] = ((o[2] >> 16) & 0xFFu) | ((o[0] >> 16) & 0xFF00u) | ((o[1] >> 8) & 0xFF0000u) | (o[2] & 0xFF000000u);
}

// Stores the twelve bytes of pixels 4m..4m+3 at `piece` (row-major):
// three dwords when aligned, else the bytes that lie inside the row.
__device__ __forceinline__ void store12(VC_GLOBAL uint8_t *piece, const uint32_t dw[3], uint32_t m, uint32_t w,
                                        int aligned) {
    if (aligned && 4 * m + 4 <= w) {
        VC_GLOBAL uint32_t *q4 = reinterpret_cast<VC_GLOBAL uint32_t *>(piece);
        q4[0] = dw[0];
        q4[1] = dw[1];
        q4[2] = dw[2];
    } else {
        const uint32_t nb = 3 * ((w - 4 * m < 4) ? w - 4 * m : 4);
        for (uint32_t b = 0; b < nb; ++b) piece[b] = static_cast<uint8_t>(dw[b >> 2] >> (8 * (b & 3)));
    }
}

__device__ __forceinline__ void row_shifts(const VC_GLOBAL uint16_t *D, uint32_t r, uint32_t h, const Geometry &geo,
                                           bool inv, uint32_t sh[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const uint32_t dh = mod_u16(D[c * h + r], geo.mod_W8);
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
// memory row by row.  The intermediate X is row-major or strip-major
// (FrameDesc::xstrip; only with STAGE and 16-byte rows).
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
        const uint32_t xs = d.xstrip;
        const bool x_sm = xs != 0;
        const uint32_t sl = x_sm ? static_cast<uint32_t>(__builtin_ctz(xs)) : 0;
        if (INV && x_sm) {
            // T is strip-major: rows r0 .. r0+nr-1 of a strip are one
            // contiguous run of 16-byte words, read in memory order (every
            // strip but the last has nr * SB / 16 of them)
            const uint32_t ns = (rb + xs - 1) >> sl, cps = nr * (xs / 16), n16 = nr * (rb / 16);
            // word k: strip st, position `within` of the strip's run of nr rows
            auto strip_of = [&](uint32_t k) { return k / cps < ns - 1 ? k / cps : ns - 1; };
            stage16(
                n16,
                [&](uint32_t k) {
                    const uint32_t st = strip_of(k), k0 = st << sl, sbw = (rb - k0 < xs) ? rb - k0 : xs;
                    return reinterpret_cast<const VC_GLOBAL u32x4 *>(
                        src + static_cast<uint64_t>(k0) * h + static_cast<uint64_t>(r0) * sbw + 16 * (k - st * cps));
                },
                [&](uint32_t k) {
                    const uint32_t st = strip_of(k), k0 = st << sl, sbw = (rb - k0 < xs) ? rb - k0 : xs;
                    const uint32_t within = k - st * cps, q16 = sbw / 16;
                    const uint32_t rr = within / q16, e = within - rr * q16;
                    return reinterpret_cast<u32x4 *>(rowbuf + rr * lds_row + k0 + 16 * e);
                });
        } else {
            const VC_GLOBAL uint8_t *s0 = src + static_cast<uint64_t>(r0) * rb;
            const bool v16 = aligned && (rb % 16 == 0) && ((reinterpret_cast<uintptr_t>(src) & 15) == 0);
            if (v16) {
                // the rows are contiguous: nr * rb / 16 uint4, row k at LDS offset k * lds_row
                const uint32_t per = rb / 16, n16 = nr * per;
                stage16(
                    n16, [&](uint32_t k) { return reinterpret_cast<const VC_GLOBAL u32x4 *>(s0) + k; },
                    [&](uint32_t k) {
                        const uint32_t rr = k / per, e = k - rr * per;
                        return reinterpret_cast<u32x4 *>(rowbuf + rr * lds_row) + e;
                    });
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
            // S is strip-major (w % 16 == 0, so every 12-byte piece lies in
            // the row).  Lanes are ordered strip, row, piece, so that a wave
            // writes rows r0 .. r0+nr-1 of a strip -- one contiguous run of
            // whole lines -- together; a piece that straddles two strips is
            // made by a lane of each, and each stores its own strip's dwords.
            const uint32_t slots = (xs + 11) / 12 + 1;  // pieces that can touch one strip row
            const uint32_t per_strip = nr * slots, total = ((rb + xs - 1) >> sl) * per_strip;
            for (uint32_t t = threadIdx.x; t < total; t += kRowThreads) {
                const uint32_t st = t / per_strip, within = t - st * per_strip;
                const uint32_t rr = within / slots, slot = within - rr * slots;
                const uint32_t k0 = st << sl, sbw = (rb - k0 < xs) ? rb - k0 : xs;
                const uint32_t m = k0 / 12 + slot;
                if (12 * m >= k0 + sbw) continue;  // past the strip's last piece
                const uint32_t sh[3] = {shS[rr][0], shS[rr][1], shS[rr][2]};
                uint32_t dw[3];
                shift12(rowbuf + rr * lds_row, sh, m, w, W8, dw);
                VC_GLOBAL uint8_t *run = dst + static_cast<uint64_t>(k0) * h + static_cast<uint64_t>(r0 + rr) * sbw;
                if (12 * m >= k0 && 12 * m + 12 <= k0 + sbw) {
                    VC_GLOBAL uint32_t *q4 = reinterpret_cast<VC_GLOBAL uint32_t *>(run + (12 * m - k0));
                    q4[0] = dw[0];
                    q4[1] = dw[1];
                    q4[2] = dw[2];
                } else {
#pragma unroll
                    for (uint32_t e = 0; e < 3; ++e) {
                        const uint32_t k = 12 * m + 4 * e;
                        if (k >= k0 && k < k0 + sbw) *reinterpret_cast<VC_GLOBAL uint32_t *>(run + (k - k0)) = dw[e];
                    }
                }
            }
        } else {
            for (uint32_t k = threadIdx.x; k < nr * ngroups; k += kRowThreads) {
                const uint32_t rr = k / ngroups, m = k - rr * ngroups;
                const uint32_t sh[3] = {shS[rr][0], shS[rr][1], shS[rr][2]};
                uint32_t dw[3];
                shift12(rowbuf + rr * lds_row, sh, m, w, W8, dw);
                store12(dst + static_cast<uint64_t>(r0 + rr) * rb + 12 * m, dw, m, w, aligned);
            }
        }
    } else {
        for (uint32_t rr = 0; rr < nr; ++rr) {
            const uint32_t r = r0 + rr;
            uint32_t sh[3];
            row_shifts(D, r, h, geo, INV, sh);
            const VC_GLOBAL uint8_t *srow = src + static_cast<uint64_t>(r) * rb;
            VC_GLOBAL uint8_t *drow = dst + static_cast<uint64_t>(r) * rb;
            for (uint32_t m = threadIdx.x; m < ngroups; m += kRowThreads) {
                uint32_t dw[3];
                shift12(srow, sh, m, w, W8, dw);
                store12(drow + 12 * m, dw, m, w, aligned);
            }
        }
    }
}

// ----------------------------------------------------------------------
// Planar row pass (rows of a multiple of 16 pixels, frames and outputs
// 16-byte aligned).  The byte-wise form above spends most of its time on
// per-byte LDS reads and index arithmetic; here one item is 16 pixels (48
// bytes) of one row:
//   1. the item's 48 bytes are loaded, split into the three channels with
//      byte permutes and stored as LDS channel planes (w bytes each,
//      followed by a copy of the plane's first 16 bytes, so that a window
//      that runs past the end of the row continues at its start);
//   2. the item makes its 16 output bytes of each channel c: they are bits
//      s .. s+127 of the channel's bit row, s = (128 g + sh_c) mod 8w for
//      item g, i.e. four v_alignbit of five plane dwords from byte
//      (s >> 3) & ~3 on, at bit offset s mod 32; byte permutes interleave
//      the channels again and the item stores 48 bytes.
// ----------------------------------------------------------------------
constexpr uint32_t kPlanePad = 16;

__host__ __device__ inline uint32_t plane_stride(uint32_t w) { return w + kPlanePad; }
// LDS of a planar workgroup of R rows: one buffer that holds in turn the
// rows, their channel planes and the shifted rows, then the shift table.
constexpr uint32_t kPlanarItems = 4;  // items per thread at most (registers across barriers)
__host__ __device__ inline uint64_t planar_lds_bytes(uint32_t w, uint32_t R) {
    return 3ull * R * plane_stride(w) + kRowShiftTable;
}
// Rows per planar workgroup: the most (4, 2 or 1) whose items fit the
// threads' registers and whose LDS fits lds_limit; 0 if none.
__host__ __device__ inline uint32_t planar_rows(uint32_t w, uint32_t lds_limit) {
    for (uint32_t R = kRowsPerGroup; R >= 1; R /= 2)
        if (static_cast<uint64_t>(R) * (w / 16) <= kRowThreads * kPlanarItems && planar_lds_bytes(w, R) <= lds_limit)
            return R;
    return 0;
}

// Byte permutes with compile-time selectors: dword k of the result is byte
// B_k of the little-endian 12-dword array s.  v_perm_b32 picks from the
// 64-bit pair (first operand : second operand); 0x0C gives a zero byte.
constexpr int first_other(int a, int b, int c, int d, int x, int y) {
    return (a != x && a != y) ? a : (b != x && b != y) ? b : (c != x && c != y) ? c : (d != x && d != y) ? d : -1;
}
constexpr uint32_t sel_two(const int (&B)[4], int lo, int hi) {
    uint32_t sel = 0;
    for (int k = 0; k < 4; ++k) {
        const int dw = B[k] / 4, by = B[k] % 4;
        const uint32_t v = dw == lo ? by : dw == hi ? 4 + by : 0x0C;
        sel |= v << (8 * k);
    }
    return sel;
}
constexpr uint32_t sel_third(const int (&B)[4], int third) {
    uint32_t sel = 0;
    for (int k = 0; k < 4; ++k) {
        const int dw = B[k] / 4, by = B[k] % 4;
        const uint32_t v = dw == third ? 4 + by : k;
        sel |= v << (8 * k);
    }
    return sel;
}
template <int B0, int B1, int B2, int B3>
__device__ __forceinline__ uint32_t gather4(const uint32_t (&s)[12]) {
    constexpr int B[4] = {B0, B1, B2, B3};
    constexpr int d0 = B0 / 4;
    constexpr int d1r = first_other(B0 / 4, B1 / 4, B2 / 4, B3 / 4, d0, d0);
    constexpr int d1 = d1r < 0 ? d0 : d1r;
    constexpr int d2 = first_other(B0 / 4, B1 / 4, B2 / 4, B3 / 4, d0, d1);
    uint32_t r = __builtin_amdgcn_perm(s[d1], s[d0], sel_two(B, d0, d1));
    if constexpr (d2 >= 0) r = __builtin_amdgcn_perm(s[d2], r, sel_third(B, d2));
    return r;
}

// 48 interleaved bytes (pixel p, channel c at byte 3p + c) -> three planes
// of 16 bytes (plane c dword m = channel c of pixels 4m .. 4m+3), and back.
template <int C, int M>
__device__ __forceinline__ uint32_t plane_dword(const uint32_t (&s)[12]) {
    return gather4<12 * M + C, 12 * M + C + 3, 12 * M + C + 6, 12 * M + C + 9>(s);
}
template <int M>
__device__ __forceinline__ uint32_t pixel_dword(const uint32_t (&p)[12]) {
    // byte b = 4M + x is pixel b / 3, channel b % 3: plane dword 4c + pixel / 4
    constexpr int b0 = 4 * M, b1 = b0 + 1, b2 = b0 + 2, b3 = b0 + 3;
    return gather4<4 * (4 * (b0 % 3) + b0 / 12) + (b0 / 3) % 4, 4 * (4 * (b1 % 3) + b1 / 12) + (b1 / 3) % 4,
                   4 * (4 * (b2 % 3) + b2 / 12) + (b2 / 3) % 4, 4 * (4 * (b3 % 3) + b3 / 12) + (b3 / 3) % 4>(p);
}
__device__ __forceinline__ void to_planes(const uint32_t (&s)[12], uint32_t (&p)[12]) {
    p[0] = plane_dword<0, 0>(s); p[1] = plane_dword<0, 1>(s); p[2] = plane_dword<0, 2>(s); p[3] = plane_dword<0, 3>(s);
    p[4] = plane_dword<1, 0>(s); p[5] = plane_dword<1, 1>(s); p[6] = plane_dword<1, 2>(s); p[7] = plane_dword<1, 3>(s);
    p[8] = plane_dword<2, 0>(s); p[9] = plane_dword<2, 1>(s); p[10] = plane_dword<2, 2>(s); p[11] = plane_dword<2, 3>(s);
}
__device__ __forceinline__ void to_pixels(const uint32_t (&p)[12], uint32_t (&s)[12]) {
    s[0] = pixel_dword<0>(p); s[1] = pixel_dword<1>(p); s[2] = pixel_dword<2>(p); s[3] = pixel_dword<3>(p);
    s[4] = pixel_dword<4>(p); s[5] = pixel_dword<5>(p); s[6] = pixel_dword<6>(p); s[7] = pixel_dword<7>(p);
    s[8] = pixel_dword<8>(p); s[9] = pixel_dword<9>(p); s[10] = pixel_dword<10>(p); s[11] = pixel_dword<11>(p);
}

// 16-byte word k of the run of rows r0 .. r0+nr-1 of X, in memory order:
// its byte offset in X and in an LDS copy of those rows (row-major, rows
// of rb bytes).  Row-major X: the rows are one run.  Strip-major X (strips
// of xs = 2^sl bytes, ns of them): strip s holds the rows' segments of sbw
// bytes as one run of nr * sbw bytes (every strip but the last has nr *
// xs / 16 words).
struct XRun {
    uint32_t rb, h, r0, nr, xs, sl, ns, cps, cps_shift;
    __device__ __forceinline__ XRun(uint32_t rb_, uint32_t h_, uint32_t r0_, uint32_t nr_, uint32_t xs_)
        : rb(rb_), h(h_), r0(r0_), nr(nr_), xs(xs_) {
        sl = xs ? static_cast<uint32_t>(__builtin_ctz(xs)) : 0;
        ns = xs ? (rb + xs - 1) >> sl : 1;
        cps = xs ? nr * (xs / 16) : 0;
        // a power of two when nr is (every workgroup but a frame's last)
        cps_shift = (cps && (cps & (cps - 1)) == 0) ? static_cast<uint32_t>(__builtin_ctz(cps)) : 32;
    }
    __device__ __forceinline__ void word(uint32_t k, uint64_t &x, uint32_t &lds) const {
        if (!xs) {
            x = static_cast<uint64_t>(r0) * rb + 16 * k;
            lds = 16 * k;
            return;
        }
        uint32_t st = cps_shift < 32 ? k >> cps_shift : k / cps;
        st = st < ns - 1 ? st : ns - 1;
        const uint32_t k0 = st << sl, sbw = (rb - k0 < xs) ? rb - k0 : xs;
        const uint32_t within = k - st * cps;
        uint32_t rr, e;
        if (sbw == xs) {
            rr = within >> (sl - 4);
            e = within & (xs / 16 - 1);
        } else {
            rr = within / (sbw / 16);
            e = within - rr * (sbw / 16);
        }
        x = static_cast<uint64_t>(k0) * h + static_cast<uint64_t>(r0) * sbw + 16 * within;
        lds = rr * rb + k0 + 16 * e;
    }
};

// One workgroup shifts R = rpg rows (at most kRowsPerGroup; 256 threads,
// at most NI items each, NI <= kPlanarItems: fewer registers when rows are
// short); one LDS buffer serves every phase:
//   A. the rows are staged (row-major, 16-byte loads in memory order of the
//      source, six in flight per thread);
//   B. each item (16 pixels of a row) takes its 48 bytes into registers;
//      after a barrier they are split into the channel planes, written over
//      the rows;
//   C. each item shifts its 16 bytes per channel out of the planes and
//      interleaves them in registers; after a barrier they are written back
//      as rows;
//   D. the shifted rows are copied out in memory order of the destination
//      (16-byte stores, whole runs of rpg rows of each strip when X is
//      strip-major).
template <bool INV, uint32_t NI>
__global__ __launch_bounds__(kRowThreads) void row_shift_planar(const FrameDesc *__restrict__ desc, uint32_t first,
                                                              uint32_t nframes, Geometry geo,
                                                              uint32_t groups_per_frame, uint32_t rpg) {
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t fl = blockIdx.x / groups_per_frame, grp = blockIdx.x - fl * groups_per_frame;
    if (fl >= nframes) return;
    const FrameDesc d = desc[first + fl];
    const uint32_t w = geo.w, h = geo.h, W8 = geo.W8, rb = geo.row_bytes;
    const uint32_t G = w / 16, ps = plane_stride(w);
    const uint32_t r0 = grp * rpg;
    const uint32_t nr = (h - r0 < rpg) ? h - r0 : rpg;
    const uint32_t items = nr * G, n16 = nr * (rb / 16);
    uint8_t *rows = lds;    // row rr at rr * rb
    uint8_t *planes = lds;  // plane (rr, c) at (3 rr + c) * ps
    uint32_t(*shS)[3] = reinterpret_cast<uint32_t(*)[3]>(lds + 3 * rpg * ps);
    if (threadIdx.x < nr) row_shifts(gmem(d.D), r0 + threadIdx.x, h, geo, INV, shS[threadIdx.x]);
    const VC_GLOBAL uint8_t *__restrict__ src = gmem(INV ? d.X : d.in);
    VC_GLOBAL uint8_t *__restrict__ dst = gmem(INV ? d.out : d.X);
    const XRun xr(rb, h, r0, nr, d.xstrip);
    // A. stage
    if (INV) {
        stage16(
            n16,
            [&](uint32_t k) {
                uint64_t x;
                uint32_t l;
                xr.word(k, x, l);
                return reinterpret_cast<const VC_GLOBAL u32x4 *>(src + x);
            },
            [&](uint32_t k) {
                uint64_t x;
                uint32_t l;
                xr.word(k, x, l);
                return reinterpret_cast<u32x4 *>(rows + l);
            });
    } else {
        const VC_GLOBAL u32x4 *s0 = reinterpret_cast<const VC_GLOBAL u32x4 *>(src + static_cast<uint64_t>(r0) * rb);
        stage16(
            n16, [&](uint32_t k) { return s0 + k; }, [&](uint32_t k) { return reinterpret_cast<u32x4 *>(rows) + k; });
    }
    __syncthreads();
    // item j of this thread: it = threadIdx.x + j * kRowThreads, row rr, 16-pixel group g
    uint32_t rrj[NI], gj[NI];
#pragma unroll
    for (uint32_t j = 0; j < NI; ++j) {
        const uint32_t it = threadIdx.x + j * kRowThreads;
        rrj[j] = static_cast<uint32_t>(it >= G) + (it >= 2 * G) + (it >= 3 * G);
        gj[j] = it - rrj[j] * G;
    }
    u32x4 v[NI][3];
    // B. rows -> registers -> channel planes
#pragma unroll
    for (uint32_t j = 0; j < NI; ++j)
        if (threadIdx.x + j * kRowThreads < items) {
            const u32x4 *q = reinterpret_cast<const u32x4 *>(rows + rrj[j] * rb + 48 * gj[j]);
            v[j][0] = q[0];
            v[j][1] = q[1];
            v[j][2] = q[2];
        }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < NI; ++j)
        if (threadIdx.x + j * kRowThreads < items) {
            uint32_t sw[12], p[12];
#pragma unroll
            for (uint32_t i = 0; i < 3; ++i) {
                sw[4 * i] = v[j][i].x; sw[4 * i + 1] = v[j][i].y; sw[4 * i + 2] = v[j][i].z; sw[4 * i + 3] = v[j][i].w;
            }
            to_planes(sw, p);
#pragma unroll
            for (uint32_t c = 0; c < 3; ++c) {
                uint8_t *pl = planes + (3 * rrj[j] + c) * ps;
                const u32x4 x{p[4 * c], p[4 * c + 1], p[4 * c + 2], p[4 * c + 3]};
                *reinterpret_cast<u32x4 *>(pl + 16 * gj[j]) = x;
                if (gj[j] == 0) *reinterpret_cast<u32x4 *>(pl + w) = x;  // the wrap-around copy
            }
        }
    __syncthreads();
    // C. shift out of the planes and interleave -> registers -> rows
#pragma unroll
    for (uint32_t j = 0; j < NI; ++j)
        if (threadIdx.x + j * kRowThreads < items) {
            const uint32_t rr = rrj[j], g = gj[j];
            uint32_t p[12], o[12];
#pragma unroll
            for (uint32_t c = 0; c < 3; ++c) {
                uint32_t s = 128 * g + shS[rr][c];  // 128 g < 8w, sh < 8w
                if (s >= W8) s -= W8;
                const uint32_t *a = reinterpret_cast<const uint32_t *>(planes + (3 * rr + c) * ps) + (s >> 5);
                const uint32_t a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3], a4 = a[4];
                const uint32_t t = s & 31;
                p[4 * c] = __builtin_amdgcn_alignbit(a1, a0, t);
                p[4 * c + 1] = __builtin_amdgcn_alignbit(a2, a1, t);
                p[4 * c + 2] = __builtin_amdgcn_alignbit(a3, a2, t);
                p[4 * c + 3] = __builtin_amdgcn_alignbit(a4, a3, t);
            }
            to_pixels(p, o);
#pragma unroll
            for (uint32_t i = 0; i < 3; ++i) v[j][i] = u32x4{o[4 * i], o[4 * i + 1], o[4 * i + 2], o[4 * i + 3]};
        }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < NI; ++j)
        if (threadIdx.x + j * kRowThreads < items) {
            u32x4 *q = reinterpret_cast<u32x4 *>(rows + rrj[j] * rb + 48 * gj[j]);
            q[0] = v[j][0];
            q[1] = v[j][1];
            q[2] = v[j][2];
        }
    __syncthreads();
    // D. copy out
    if (INV) {
        VC_GLOBAL u32x4 *d0 = reinterpret_cast<VC_GLOBAL u32x4 *>(dst + static_cast<uint64_t>(r0) * rb);
        stage16(
            n16, [&](uint32_t k) { return reinterpret_cast<const u32x4 *>(rows) + k; }, [&](uint32_t k) { return d0 + k; });
    } else {
        stage16(
            n16,
            [&](uint32_t k) {
                uint64_t x;
                uint32_t l;
                xr.word(k, x, l);
                return reinterpret_cast<const u32x4 *>(rows + l);
            },
            [&](uint32_t k) {
                uint64_t x;
                uint32_t l;
                xr.word(k, x, l);
                return reinterpret_cast<VC_GLOBAL u32x4 *>(dst + x);
            });
    }
}

// ----------------------------------------------------------------------
// Column pass
// ----------------------------------------------------------------------
// LDS: the strip (h rows of at most SB bytes), then the strip's column
// distances (SB words: the source-row offset of each byte column).
// Strips of 16 bytes or more keep each staged row at a stride of SB + 4
// bytes (an odd number of dwords), so that the gather's lanes, which read
// the same byte column of consecutive rows, fall in different LDS banks.
__host__ __device__ constexpr uint32_t col_row_stride(uint32_t SB) { return SB >= 16 ? SB + 4 : SB; }
__host__ __device__ inline uint32_t col_dv_off(uint32_t h, uint32_t SB) { return align16(h * col_row_stride(SB)); }
__host__ __device__ inline uint32_t col_lds_bytes(uint32_t h, uint32_t SB) { return col_dv_off(h, SB) + 4 * SB; }

// Byte columns k0 .. k0 + sb - 1 of the strip: dvS[kk] = d_v mod h of the
// column (forward: the output row i takes source row (i - dvS) mod h) or
// h - d_v mod h (inverse: row r of T takes row (r + d_v) mod h of C ^ B);
// both read (i + h - dvS) mod h.
__device__ __forceinline__ void col_distances(const VC_GLOBAL uint16_t *D, const Geometry &geo, uint32_t k0,
                                              uint32_t sb, bool inv, uint32_t *dvS, uint32_t nt) {
    const uint32_t h = geo.h, w = geo.w;
    for (uint32_t kk = threadIdx.x; kk < sb; kk += nt) {
        const uint32_t k = k0 + kk, j = k / 3, c = k - 3 * j;
        const uint32_t dv = mod_u16(D[3 * h + c * w + j], geo.mod_h);
        dvS[kk] = inv ? (dv ? h - dv : 0) : dv;
    }
}

// A 16-byte word to a 4-byte aligned LDS address (the padded staged rows).
__device__ __forceinline__ void put16(uint8_t *p, const u32x4 &v) {
    uint32_t *q = reinterpret_cast<uint32_t *>(p);
    q[0] = v.x;
    q[1] = v.y;
    q[2] = v.z;
    q[3] = v.w;
}

// 16-byte column pass: rows of a multiple of 16 bytes, frames, outputs and
// keystream 16-byte aligned, X strip-major with strips of SB bytes.  One
// workgroup owns a full-height strip of one frame; thread t handles the
// 16-byte word q = t % nq of rows i0, i0 + RP, ... (i0 = t / nq).
//   forward: stage the strip of S (one contiguous block of X) with
//            B's first rows already in flight, then
//            C[i][word] = gather of S rows (i - d_v) mod h ^ B[i][word];
//   inverse: stage C ^ B (16-byte words of every row), then
//            T[r][word] = gather of rows (r + d_v) mod h, stored to the
//            strip's contiguous block of X.
template <int SB, int NT, bool INV>
__global__ __launch_bounds__(NT) void col_shift_v(const FrameDesc *__restrict__ desc, uint32_t first, uint32_t nframes,
                                                  Geometry geo, uint32_t nstrips, int xcd_map) {
    extern __shared__ __align__(16) uint8_t smem[];
    constexpr uint32_t U = NT >= 1024 ? 2 : 4;  // rows in flight per thread (1024 threads: within 56 VGPRs)
    uint32_t fl, strip;
    map_strip(blockIdx.x, nstrips, xcd_map, fl, strip);
    if (fl >= nframes) return;
    const FrameDesc d = desc[first + fl];
    const uint32_t h = geo.h, rb = geo.row_bytes;
    const uint32_t k0 = strip * SB;
    const uint32_t sb = (rb - k0 < static_cast<uint32_t>(SB)) ? rb - k0 : SB;  // a multiple of 16
    const uint32_t nq = sb >> 4, sbp = sb + 4;  // staged row stride: col_row_stride
    const uint32_t RP = NT / nq;  // rows per pass
    const uint32_t q = threadIdx.x % nq, i0 = threadIdx.x / nq;
    const uint32_t np = (i0 < RP && i0 < h) ? (h - i0 + RP - 1) / RP : 0;  // rows of this thread
    uint8_t *S = smem;
    uint32_t *dvS = reinterpret_cast<uint32_t *>(smem + col_dv_off(h, SB));
    VC_GLOBAL uint8_t *Xs = gmem(d.X) + static_cast<uint64_t>(k0) * h;  // the strip's block of X
    const VC_GLOBAL uint8_t *Bq = gmem(d.B) + k0 + 16 * q;
    col_distances(gmem(d.D), geo, k0, sb, INV, dvS, NT);

    u32x4 b[U];
    if (!INV) {
        // B of the first U rows in flight while the strip is staged
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
            if (u < np) b[u] = *reinterpret_cast<const VC_GLOBAL u32x4 *>(Bq + static_cast<uint64_t>(i0 + u * RP) * rb);
        // word q of rows i0, i0 + RP, ...: a wave reads a contiguous run of X
        const VC_GLOBAL u32x4 *X4 = reinterpret_cast<const VC_GLOBAL u32x4 *>(Xs) + q;
        for (uint32_t p0 = 0; p0 < np; p0 += 4) {
            u32x4 v[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u)
                if (p0 + u < np) v[u] = X4[(i0 + (p0 + u) * RP) * nq];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u)
                if (p0 + u < np) put16(S + (i0 + (p0 + u) * RP) * sbp + 16 * q, v[u]);
        }
    } else {
        const VC_GLOBAL uint8_t *Cq = gmem(d.in) + k0 + 16 * q;
        for (uint32_t p0 = 0; p0 < np; p0 += U) {
            u32x4 c[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                if (p0 + u < np) {
                    const uint64_t off = static_cast<uint64_t>(i0 + (p0 + u) * RP) * rb;
                    c[u] = *reinterpret_cast<const VC_GLOBAL u32x4 *>(Cq + off);
                    b[u] = *reinterpret_cast<const VC_GLOBAL u32x4 *>(Bq + off);
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                if (p0 + u < np)
                    put16(S + (i0 + (p0 + u) * RP) * sbp + 16 * q, c[u] ^ b[u]);
        }
    }
    __syncthreads();
    if (np == 0) return;

    // LDS byte address of each of the thread's 16 byte columns in its
    // current row, stepped by RP rows (mod h) per pass
    uint32_t a[16];
#pragma unroll
    for (uint32_t m = 0; m < 16; ++m) {
        const uint32_t kk = 16 * q + m, dv = dvS[kk];
        const uint32_t r = (i0 >= dv) ? i0 - dv : i0 + h - dv;
        a[m] = r * sbp + kk;
    }
    const uint32_t stepA = (RP % h) * sbp, wrapA = h * sbp;
    VC_GLOBAL uint8_t *Oq = INV ? Xs + 16 * q : gmem(d.out) + k0 + 16 * q;
    const uint32_t ostride = INV ? sb : rb;
    for (uint32_t p0 = 0; p0 < np; p0 += U) {
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t p = p0 + u;
            if (p < np) {
                u32x4 v;
#pragma unroll
                for (uint32_t e = 0; e < 4; ++e)
                    v[e] = static_cast<uint32_t>(S[a[4 * e]]) | (static_cast<uint32_t>(S[a[4 * e + 1]]) << 8) |
                           (static_cast<uint32_t>(S[a[4 * e + 2]]) << 16) |
                           (static_cast<uint32_t>(S[a[4 * e + 3]]) << 24);
                const uint32_t i = i0 + p * RP;
                if (!INV) {
                    v ^= b[u];
                    if (p + U < np)
                        b[u] = *reinterpret_cast<const VC_GLOBAL u32x4 *>(
                            Bq + static_cast<uint64_t>(i0 + (p + U) * RP) * rb);
                }
                *reinterpret_cast<VC_GLOBAL u32x4 *>(Oq + static_cast<uint64_t>(i) * ostride) = v;
#pragma unroll
                for (uint32_t m = 0; m < 16; ++m) {
                    a[m] += stepA;
                    if (a[m] >= wrapA) a[m] -= wrapA;
                }
            }
        }
    }
}

// Column pass for any frame (X row-major): the same strips, staged and
// gathered in units of G bytes (G = 4 when rows and pointers are 4-byte
// aligned, else 1).
template <int SB, int NT, bool INV, int G>
__global__ __launch_bounds__(NT) void col_shift_g(const FrameDesc *__restrict__ desc, uint32_t first, uint32_t nframes,
                                                  Geometry geo, uint32_t nstrips, int xcd_map) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t fl, strip;
    map_strip(blockIdx.x, nstrips, xcd_map, fl, strip);
    if (fl >= nframes) return;
    const FrameDesc d = desc[first + fl];
    const uint32_t h = geo.h, rb = geo.row_bytes;
    const uint32_t k0 = strip * SB;
    const uint32_t sb = (rb - k0 < static_cast<uint32_t>(SB)) ? rb - k0 : SB;
    const uint32_t ng = sb / G;  // units per strip row
    uint8_t *S = smem;           // row stride SB
    uint32_t *dvS = reinterpret_cast<uint32_t *>(smem + col_dv_off(h, SB));
    const VC_GLOBAL uint8_t *in = gmem(INV ? d.in : d.X) + k0;
    VC_GLOBAL uint8_t *out = gmem(INV ? d.X : d.out) + k0;
    const VC_GLOBAL uint8_t *Bp = gmem(d.B) + k0;
    col_distances(gmem(d.D), geo, k0, sb, INV, dvS, NT);
    const uint32_t total = h * ng;
    for (uint32_t it = threadIdx.x; it < total; it += NT) {
        const uint32_t i = it / ng, g = it - i * ng;
        const uint64_t off = static_cast<uint64_t>(i) * rb + G * g;
        if (G == 4) {
            uint32_t v = *reinterpret_cast<const VC_GLOBAL uint32_t *>(in + off);
            if (INV) v ^= *reinterpret_cast<const VC_GLOBAL uint32_t *>(Bp + off);
            *reinterpret_cast<uint32_t *>(S + i * SB + 4 * g) = v;
        } else {
            uint8_t v = in[off];
            if (INV) v ^= Bp[off];
            S[i * SB + g] = v;
        }
    }
    __syncthreads();
    for (uint32_t it = threadIdx.x; it < total; it += NT) {
        const uint32_t i = it / ng, g = it - i * ng;
        const uint64_t off = static_cast<uint64_t>(i) * rb + G * g;
        uint32_t v = 0;
#pragma unroll
        for (uint32_t m = 0; m < static_cast<uint32_t>(G); ++m) {
            const uint32_t kk = G * g + m, dv = dvS[kk];
            const uint32_t r = (i >= dv) ? i - dv : i + h - dv;
            v |= static_cast<uint32_t>(S[r * SB + kk]) << (8 * m);
        }
        if (G == 4) {
            if (!INV) v ^= *reinterpret_cast<const VC_GLOBAL uint32_t *>(Bp + off);
            *reinterpret_cast<VC_GLOBAL uint32_t *>(out + off) = v;
        } else {
            if (!INV) v ^= Bp[off];
            out[off] = static_cast<uint8_t>(v);
        }
    }
}

constexpr uint32_t kColStrips[] = {4, 8, 16, 32, 64, 128};

template <int SB, int NT, bool INV>
hipError_t launch_col_one(const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g, int align,
                          bool vec, int xcd_map, hipStream_t s) {
    const uint32_t nstrips = (g.row_bytes + SB - 1) / SB;
    const uint64_t groups =
        xcd_map ? 8ull * ((count + 7) / 8) * nstrips : static_cast<uint64_t>(count) * nstrips;
    if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const dim3 grid(static_cast<uint32_t>(groups)), block(NT);
    const uint32_t lds = col_lds_bytes(g.h, SB);
    if constexpr (SB >= 16) {
        if (vec) {
            hipLaunchKernelGGL((col_shift_v<SB, NT, INV>), grid, block, lds, s, d_desc, first, count, g, nstrips,
                               xcd_map);
            return hipGetLastError();
        }
    }
    if (align >= 1)
        hipLaunchKernelGGL((col_shift_g<SB, NT, INV, 4>), grid, block, lds, s, d_desc, first, count, g, nstrips,
                           xcd_map);
    else
        hipLaunchKernelGGL((col_shift_g<SB, NT, INV, 1>), grid, block, lds, s, d_desc, first, count, g, nstrips,
                           xcd_map);
    return hipGetLastError();
}

template <int SB, bool INV>
hipError_t launch_col_sb(const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g, int align,
                         bool vec, const ConfuseTuning &t, hipStream_t s) {
    switch (t.threads) {
    case 256: return launch_col_one<SB, 256, INV>(d_desc, first, count, g, align, vec, t.xcd_map, s);
    case 512: return launch_col_one<SB, 512, INV>(d_desc, first, count, g, align, vec, t.xcd_map, s);
    default: return launch_col_one<SB, 1024, INV>(d_desc, first, count, g, align, vec, t.xcd_map, s);
    }
}

template <bool INV>
hipError_t launch_col(const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g, int align, bool vec,
                      const ConfuseTuning &t, hipStream_t s) {
    switch (t.strip) {
    case 4: return launch_col_sb<4, INV>(d_desc, first, count, g, align, vec, t, s);
    case 8: return launch_col_sb<8, INV>(d_desc, first, count, g, align, vec, t, s);
    case 16: return launch_col_sb<16, INV>(d_desc, first, count, g, align, vec, t, s);
    case 32: return launch_col_sb<32, INV>(d_desc, first, count, g, align, vec, t, s);
    case 64: return launch_col_sb<64, INV>(d_desc, first, count, g, align, vec, t, s);
    case 128: return launch_col_sb<128, INV>(d_desc, first, count, g, align, vec, t, s);
    default: return hipErrorInvalidValue;
    }
}

template <bool INV>
hipError_t launch_row(const FrameDesc *d_desc, uint32_t first, uint32_t count, const Geometry &g, int align,
                      uint32_t lds_limit, hipStream_t s) {
    const bool aligned = align >= 1;
    if (shift_rows_planar(g.w, align, lds_limit)) {
        const uint32_t R = planar_rows(g.w, lds_limit);
        const uint32_t per_frame = (g.h + R - 1) / R;
        const uint64_t groups = static_cast<uint64_t>(count) * per_frame;
        if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
        const uint32_t lds = static_cast<uint32_t>(planar_lds_bytes(g.w, R));
        if (R * (g.w / 16) <= 2 * kRowThreads)
            hipLaunchKernelGGL((row_shift_planar<INV, 2>), dim3(static_cast<uint32_t>(groups)), dim3(kRowThreads), lds,
                               s, d_desc, first, count, g, per_frame, R);
        else
            hipLaunchKernelGGL((row_shift_planar<INV, kPlanarItems>), dim3(static_cast<uint32_t>(groups)),
                               dim3(kRowThreads), lds, s, d_desc, first, count, g, per_frame, R);
        return hipGetLastError();
    }
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

template <typename K>
hipError_t set_lds(K kernel, uint32_t limit) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(limit));
}

template <int SB, int NT>
hipError_t set_col_attr(uint32_t limit) {
    hipError_t e = set_lds(&col_shift_g<SB, NT, false, 4>, limit);
    if (e == hipSuccess) e = set_lds(&col_shift_g<SB, NT, true, 4>, limit);
    if (e == hipSuccess) e = set_lds(&col_shift_g<SB, NT, false, 1>, limit);
    if (e == hipSuccess) e = set_lds(&col_shift_g<SB, NT, true, 1>, limit);
    if constexpr (SB >= 16) {
        if (e == hipSuccess) e = set_lds(&col_shift_v<SB, NT, false>, limit);
        if (e == hipSuccess) e = set_lds(&col_shift_v<SB, NT, true>, limit);
    }
    return e;
}

template <int SB>
hipError_t set_col_attr_sb(uint32_t limit) {
    hipError_t e = set_col_attr<SB, 256>(limit);
    if (e == hipSuccess) e = set_col_attr<SB, 512>(limit);
    if (e == hipSuccess) e = set_col_attr<SB, 1024>(limit);
    return e;
}

}  // namespace

uint32_t shift_col_lds_bytes(uint32_t h, uint32_t strip) {
    for (uint32_t sb : kColStrips)
        if (sb == strip) return col_lds_bytes(h, strip);
    return 0xFFFFFFFFu;
}

bool shift_rows_staged(uint32_t w, uint32_t lds_bytes) {
    const uint64_t lds_row = (3ull * w + 15u) & ~15ull;
    return kRowsPerGroup * lds_row + kRowShiftTable <= lds_bytes;
}

bool shift_rows_planar(uint32_t w, int align, uint32_t lds_bytes) {
    return align >= 2 && w >= 16 && w % 16 == 0 && planar_rows(w, lds_bytes) > 0;
}

uint32_t shift_max_strip(uint32_t h, uint32_t lds_bytes) {
    uint32_t best = 0;
    for (uint32_t sb : kColStrips)
        if (static_cast<uint64_t>(col_lds_bytes(h, sb)) <= lds_bytes) best = sb;
    return best;
}

hipError_t shift_configure(uint32_t lds_limit) {
    hipError_t e = set_col_attr_sb<4>(lds_limit);
    if (e == hipSuccess) e = set_col_attr_sb<8>(lds_limit);
    if (e == hipSuccess) e = set_col_attr_sb<16>(lds_limit);
    if (e == hipSuccess) e = set_col_attr_sb<32>(lds_limit);
    if (e == hipSuccess) e = set_col_attr_sb<64>(lds_limit);
    if (e == hipSuccess) e = set_col_attr_sb<128>(lds_limit);
    if (e == hipSuccess) e = set_lds(&row_shift<false, true>, lds_limit);
    if (e == hipSuccess) e = set_lds(&row_shift<true, true>, lds_limit);
    if (e == hipSuccess) e = set_lds(&row_shift_planar<false, 2>, lds_limit);
    if (e == hipSuccess) e = set_lds(&row_shift_planar<true, 2>, lds_limit);
    if (e == hipSuccess) e = set_lds(&row_shift_planar<false, kPlanarItems>, lds_limit);
    if (e == hipSuccess) e = set_lds(&row_shift_planar<true, kPlanarItems>, lds_limit);
    return e;
}

uint32_t shift_xstrip(uint32_t w, uint32_t strip, int align, uint32_t lds_limit) {
    if (align < 2 || strip < 16 || (3ull * w) % 16 != 0 ||
        !(shift_rows_staged(w, lds_limit) || shift_rows_planar(w, align, lds_limit)))
        return 0;
    for (uint32_t sb : kColStrips)
        if (sb == strip) return strip;
    return 0;
}

hipError_t launch_shift(int decrypt, int pass, const FrameDesc *d_desc, uint32_t first, uint32_t count, uint32_t w,
                        uint32_t h, int align, const ConfuseTuning &t, uint32_t lds_limit, hipStream_t s) {
    if (count == 0) return hipSuccess;
    Geometry g;
    g.w = w;
    g.h = h;
    g.W8 = 8 * w;
    g.row_bytes = 3 * w;
    g.mod_h = mod_magic(h);
    g.mod_W8 = mod_magic(g.W8);
    // encrypt: pass 0 = rows, pass 1 = columns; decrypt: pass 0 = columns, pass 1 = rows
    const bool rows = decrypt ? pass == 1 : pass == 0;
    if (rows)
        return decrypt ? launch_row<true>(d_desc, first, count, g, align, lds_limit, s)
                       : launch_row<false>(d_desc, first, count, g, align, lds_limit, s);
    // the 16-byte kernels read or write X strip-major in this launch's
    // strips; the host lays X out so exactly when shift_xstrip says so
    const bool vec = shift_xstrip(w, t.strip, align, lds_limit) != 0;
    return decrypt ? launch_col<true>(d_desc, first, count, g, align, vec, t, s)
                   : launch_col<false>(d_desc, first, count, g, align, vec, t, s);
}

}  // namespace vc
