// vc_internal.hpp -- types shared by the kernels and the C-ABI layer of
// libvcipher (gfx950).  Not installed; the public interface is vcipher.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vcipher.h"

namespace vc {

// Pointers read out of descriptors are generic (flat) to the compiler;
// casting them to the global address space turns flat loads and stores
// (which also count against the LDS wait counter) into global ones.
#define VC_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ VC_GLOBAL T *gmem(T *p) {
    return (VC_GLOBAL T *)p;
}

// Per-frame work descriptor, packed on the host for every batch chunk and
// read by all kernels (uniform per workgroup, so it lands in SGPRs).
struct FrameDesc {
    const uint8_t *in;   // plaintext (encrypt) or ciphertext (decrypt), h*w*3
    uint8_t *out;        // output frame, h*w*3
    uint8_t *hash;       // 32-byte frame hash H
    double *IR;          // 2n x 4 LHCS_m iterates
    uint16_t *D;         // 3h + 3w shift distances
    uint8_t *B;          // 3wh keystream bytes
    uint8_t *X;          // 3wh intermediate of the two-pass confusion (S or T)
    uint32_t w, h;
    uint64_t L;          // 3wh
    // Layout of X: 0 = row-major (the frame's own layout), else strip-major
    // with strips of SB = xstrip bytes of each row (the column pass's strip
    // width, a power of two >= 16; rows of 3w bytes, a multiple of 16): byte
    // k of row r lies in strip s = k / SB, at s*SB*h + r*sb + k % SB, where
    // sb = min(SB, 3w - s*SB) is the strip's width (only the last strip can
    // be narrower), so that a strip's rows are contiguous and the column
    // pass reads (encrypt) or writes (decrypt) them linearly.
    uint32_t xstrip;
    uint32_t pad;
};

// One stream's frames inside a part, in sequence order: chain records
// rec[first .. first+count).
struct StreamRun {
    uint32_t slot;       // chain-state slot
    uint32_t first;
    uint32_t count;
    uint32_t pad;
};

// The chain's view of one frame, in sequence order within a run.
struct ChainRec {
    const uint8_t *hash;  // 32-byte frame hash H
    double *IR;           // 2n x 4 LHCS_m iterates
};

enum KernelId {
    K_SHA = 0,
    K_CHAIN = 1,
    K_KEYGEN = 2,
    K_ENC = 3,       // single-pass confusion + XOR
    K_DEC = 4,       // single-pass inverse
    K_ROW_ENC = 5,   // two-pass: row shift
    K_COL_ENC = 6,   // two-pass: column shift + XOR
    K_COL_DEC = 7,   // two-pass: XOR + inverse column shift
    K_ROW_DEC = 8,   // two-pass: inverse row shift
    K_COUNT = 9
};

// x mod m for a 16-bit x and 1 <= m < 2^20, by multiplication only:
// with M = ceil(2^48 / m) and e = M*m - 2^48 (0 <= e < m),
// x*M / 2^48 = x/m + x*e / (m * 2^48), and x*e < 2^36, so the second term
// stays below 1/m and floor(x*M / 2^48) is the exact quotient.  x*M fits
// in 64 bits (M <= 2^48).
struct ModMagic {
    uint32_t m, pad;
    uint64_t M;
};
__host__ __device__ inline ModMagic mod_magic(uint32_t m) {
    return ModMagic{m, 0, ((uint64_t(1) << 48) + m - 1) / m};
}
__device__ __forceinline__ uint32_t mod_u16(uint32_t x, const ModMagic &g) {
    const uint32_t q = static_cast<uint32_t>((static_cast<uint64_t>(x) * g.M) >> 48);
    return x - q * g.m;
}

// Frame geometry of a confusion launch (all frames of a launch share it).
struct Geometry {
    uint32_t w, h, W8, row_bytes;  // W8 = 8w bits per channel row, row_bytes = 3w
    ModMagic mod_h, mod_W8;        // for the distance reductions d mod h, d mod 8w
};

struct ConfuseTuning {
    // two-pass form: bytes of a row per column-pass strip (4..128, a power
    // of two); single-pass form: pixels per strip (4..64)
    uint32_t strip;
    uint32_t threads;    // 256, 512 or 1024
    int xcd_map;         // keep all strips of a frame on one XCD
};

// Device flag bits (int at d_flags[0]).
enum { FLAG_NONFINITE = 1 };

// A frame for the statistics kernels (uint8, h x w x 3).
struct StatFrame {
    const uint8_t *data;
    uint32_t w, h;
};

// Launchers (each in the translation unit of its kernel).
hipError_t launch_sha256_subframes(const FrameDesc *d_desc, uint32_t count, uint32_t n,
                                   hipStream_t s);
hipError_t launch_lhcs_chain(const StreamRun *d_runs, const ChainRec *d_rec, uint32_t nruns,
                             double *d_state, uint32_t n, double gamma, int *d_flags, hipStream_t s);
hipError_t launch_lhcs_keygen(const FrameDesc *d_desc, uint32_t count, uint32_t n,
                              double gamma, int *d_flags, hipStream_t s);
// Frames [first, first + count) of d_desc all have shape (w, h).
hipError_t launch_confuse(int decrypt, const FrameDesc *d_desc, uint32_t first, uint32_t count,
                          uint32_t w, uint32_t h, bool aligned, const ConfuseTuning &t,
                          hipStream_t s);
// Largest strip width the LDS holds for height h (0 if none), given the
// per-workgroup LDS budget.
uint32_t confuse_max_strip(int decrypt, uint32_t h, uint32_t lds_bytes);
uint32_t confuse_lds_bytes(int decrypt, uint32_t h, uint32_t strip);
hipError_t confuse_configure(uint32_t lds_limit);
// Two-pass confusion (vc_shift.hip).  pass 0 then pass 1: encrypt = rows,
// then columns + XOR; decrypt = XOR + columns, then rows.  Reads and writes
// FrameDesc::X as the intermediate.  `align` is what every frame of the
// launch satisfies: 0 nothing, 1 rows and frame pointers 4-byte aligned
// (w % 4 == 0), 2 rows and pointers (frames, output, keystream) 16-byte
// aligned (w % 16 == 0); the 16-byte column kernels run only for align 2
// with a strip-major X of the launch's strip width.
hipError_t launch_shift(int decrypt, int pass, const FrameDesc *d_desc, uint32_t first, uint32_t count, uint32_t w,
                        uint32_t h, int align, const ConfuseTuning &t, uint32_t lds_limit, hipStream_t s);
// Widest column-pass strip (bytes) whose full-height staging fits lds_bytes
// for height h, 0 if none.
uint32_t shift_max_strip(uint32_t h, uint32_t lds_bytes);
// True when the row pass stages its rows in LDS for frames of width w (the
// forms that read or write the strip-major intermediate image).
bool shift_rows_staged(uint32_t w, uint32_t lds_bytes);
// True when the row pass runs in its planar form (16 pixels per item, the
// rows split into channel planes in LDS): alignment class 2, w a multiple
// of 16, and one row with its planes fits lds_bytes.  Either staged form
// reads and writes the strip-major intermediate image.
bool shift_rows_planar(uint32_t w, int align, uint32_t lds_bytes);
// Layout of the intermediate image for frames of width w whose column pass
// uses strips of `strip` bytes under alignment class `align`: the strip
// width when X is strip-major (FrameDesc::xstrip), else 0 (row-major).
// launch_shift picks its column kernel by the same rule.
uint32_t shift_xstrip(uint32_t w, uint32_t strip, int align, uint32_t lds_limit);
uint32_t shift_col_lds_bytes(uint32_t h, uint32_t strip);
hipError_t shift_configure(uint32_t lds_limit);
// Statistics (vc_stats.hip).  hist: count x 3 x 256 (frame) or count x
// blocks x 3 x 256 (blocks), uint32; moments: count x 3 directions x 3
// channels x 5 sums, uint64.  Frame histograms and moments are added to
// their outputs (zero them first).
hipError_t launch_frame_histograms(const StatFrame *d_frames, uint32_t count, uint64_t max_bytes, uint32_t *d_hist,
                                   hipStream_t s);
hipError_t launch_block_histograms(const StatFrame *d_frames, uint32_t count, uint32_t blocks, uint32_t bw,
                                   uint32_t bh, const uint32_t *d_origins, uint32_t *d_hist, hipStream_t s);
hipError_t launch_pair_moments(const StatFrame *d_frames, uint32_t count, uint64_t max_positions, uint32_t npos,
                               const uint32_t *d_positions, unsigned long long *d_moments, hipStream_t s);
hipError_t launch_frame_diff(const StatFrame *d_a, const StatFrame *d_b, uint32_t count, uint64_t max_bytes,
                             unsigned long long *d_out, hipStream_t s);
// out = a (kind 0) or a ^ b (kind 1) over `bytes` (a multiple of 16,
// 16-byte aligned pointers), one 16-byte word per thread.
hipError_t launch_stream_probe(int kind, const uint8_t *a, const uint8_t *b, uint8_t *out, uint64_t bytes,
                               hipStream_t s);

// A library call (encrypt_frames, encrypt_frames_hashed, decrypt_frames or
// vc_hash_frames) with a 32-byte hash buffer of its own for every frame
// instead of one contiguous array; for the serving core, whose requests
// each carry their own hash buffer.  Same validation and errors.
// Device-addressable buffer check (vc_pointer_reachable).
bool reachable(const void *p, size_t bytes);
enum class CallKind { Encrypt, EncryptHashed, Decrypt, Hash };
int call_frames(vc_cipher *ctx, CallKind kind, size_t count, const uint8_t *const *frames, const vc_shape *shapes,
                uint8_t *const *hash_ptrs, uint8_t *const *out, hipStream_t stream);

// A wave of SHA-256 compression or of the key-stream integrator issues an
// instruction almost every cycle, so two such waves on one SIMD each run at
// about half speed while other SIMDs may hold none.  Claiming more than half
// of a SIMD's 512 registers per lane (256 VGPRs + 8 AGPRs) for every wave of
// those kernels keeps any two of them off the same SIMD; the bandwidth-bound
// confusion waves (at most 248 registers) still fit beside one.  Only for
// kernels of at most four waves per workgroup (one per SIMD of a CU).  The
// empty asm emits no instruction.
__device__ __forceinline__ void claim_half_simd() { asm volatile("" ::: "v255", "a7"); }

}  // namespace vc
