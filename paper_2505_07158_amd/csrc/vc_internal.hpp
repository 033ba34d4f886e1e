// vc_internal.hpp -- types shared by the kernels and the C-ABI layer of
// libvcipher (gfx950).  Not installed; the public interface is vcipher.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
    // with strips of that many pixels (WT, a power of two that divides w;
    // the column pass's strip width): byte c of row r lies in strip
    // s = c / 3WT at s*h*3WT + r*3WT + c % 3WT, so that a strip's rows are
    // contiguous and the column pass reads (encrypt) or writes (decrypt)
    // them linearly.
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

// Frame geometry of a confusion launch (all frames of a launch share it).
struct Geometry {
    uint32_t w, h, W8, row_bytes;  // W8 = 8w bits per channel row, row_bytes = 3w
    float inv_h, inv_W8;           // reciprocals for the distance reductions
};

struct ConfuseTuning {
    uint32_t strip;      // pixels per strip (multiple of 4)
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
// FrameDesc::X as the intermediate.
hipError_t launch_shift(int decrypt, int pass, const FrameDesc *d_desc, uint32_t first, uint32_t count, uint32_t w,
                        uint32_t h, bool aligned, const ConfuseTuning &t, uint32_t lds_limit, hipStream_t s);
uint32_t shift_max_strip(uint32_t h, uint32_t lds_bytes);
// True when the row pass stages its rows in LDS for frames of width w (the
// only form that reads or writes the strip-major intermediate image).
bool shift_rows_staged(uint32_t w, uint32_t lds_bytes);
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
