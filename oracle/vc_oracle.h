/*
 * vc_oracle.h -- CPU oracle of the diffusion-free video cipher (arXiv 2505.07158).
 *
 * TEST INFRASTRUCTURE ONLY.  This header and vc_oracle.c are a plain, slow,
 * scalar C99 statement of what the cipher computes.  They exist so that the
 * GPU library can be checked against them; only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load them.  They share
 * no code, header, table or constant generator with the GPU library.
 *
 * Build: gcc -O2 -std=gnu99 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (SSE2 scalar doubles on x86-64; never x87; no fused multiply-add).
 *
 * Notation follows the paper: a frame is h rows by w columns by 3 channels,
 * stored row-major with interleaved channels, L = 3*w*h bytes.  n is the
 * number of worker threads of the paper's protocol (sub-frames and worker
 * LHCS pairs); ND = 3*h + 3*w is the number of shift distances.
 */
#ifndef VC_ORACLE_H
#define VC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* SHA-256 of len bytes (FIPS 180-4, sections 5.1.1, 6.2). */
void vco_sha256(const uint8_t *msg, uint64_t len, uint8_t out[32]);

/* Frame hash of Sec. II-A: H = h_1 xor ... xor h_n, h_i the SHA-256 of the
 * i-th contiguous byte range [floor(i*L/n), floor((i+1)*L/n)). */
void vco_frame_hash(const uint8_t *frame, uint64_t L, uint32_t n, uint8_t H[32]);

/* 32 key bytes -> the four user initial conditions (x0, y0, z0, w0). */
void vco_key_from_bytes(const uint8_t K[32], double ic[4]);

/* Initial-condition reconstruction of Sec. II-A (Fig. 1a, described in
 * prose): base (the user key, or the previous frame's x_2n..w_2n) and the
 * frame hash H -> the new initial condition of LHCS_m. */
void vco_reconstruct(const double base[4], const uint8_t H[32], double ic[4]);

/* One classical Runge-Kutta step (h = 0.01) of the LHCS of Eq. 1 with
 * sigma = 10, rho = 28, beta = 8/3 and control parameter gamma.  In place.
 * Returns 0, or -1 when a component became non-finite. */
int vco_rk4_step(double s[4], double gamma);

/* Right-hand side of Eq. 1 (for tests). */
void vco_lhcs_rhs(const double s[4], double gamma, double ds[4]);

/* LHCS_m iteration of Sec. II-A / Alg. 1: IR[m-1] = state after m steps,
 * m = 1..2n, from ic.  IR holds 2n*4 doubles (x, y, z, w per step). */
int vco_chain(const double ic[4], double gamma, uint32_t n, double *IR);

/* Worker data generation of Sec. II-B / Alg. 2: IR -> shift distances
 * D (ND uint16) and keystream bytes B (L bytes). */
int vco_keystream(const double *IR, double gamma, uint32_t n, uint32_t w,
                  uint32_t h, uint16_t *D, uint8_t *B);

/* One worker's raw byte stream (for tests): nbytes bytes of worker i. */
int vco_worker_stream(const double *IR, double gamma, uint32_t i,
                      uint64_t nbytes, uint8_t *out);

/* Bit-level confusion + XOR of Sec. II-C, closed per-byte form. */
void vco_confuse_enc(const uint8_t *P, uint32_t w, uint32_t h,
                     const uint16_t *D, const uint8_t *B, uint8_t *C);
/* Its exact inverse. */
void vco_confuse_dec(const uint8_t *C, uint32_t w, uint32_t h,
                     const uint16_t *D, const uint8_t *B, uint8_t *P);
/* The same two transforms computed on the 8w x h bit matrices of Alg. 3,
 * stage by stage (Alg. 3, Eq. 2, Eq. 3, Alg. 6, Alg. 7), each permutation
 * in gather form (slow; small frames). Return -1 on allocation failure. */
int vco_confuse_enc_literal(const uint8_t *P, uint32_t w, uint32_t h,
                            const uint16_t *D, const uint8_t *B, uint8_t *C);
int vco_confuse_dec_literal(const uint8_t *C, uint32_t w, uint32_t h,
                            const uint16_t *D, const uint8_t *B, uint8_t *P);

/* Whole frame, Alg. 1: base[4] is the stream's chain state (user key for
 * the first frame) and is advanced to x_2n..w_2n.  Returns 0 or -1. */
int vco_encrypt_frame(double base[4], double gamma, uint32_t n,
                      const uint8_t *P, uint32_t w, uint32_t h,
                      uint8_t *C, uint8_t H[32]);
int vco_decrypt_frame(double base[4], double gamma, uint32_t n,
                      const uint8_t *C, uint32_t w, uint32_t h,
                      const uint8_t H[32], uint8_t *P);

/* Same as vco_encrypt_frame, with the sub-frame hashes and the n workers
 * spread over `threads` POSIX threads the way the paper's worker threads
 * share them (Alg. 1, Alg. 2).  Output is identical to the serial form. */
int vco_encrypt_frame_mt(double base[4], double gamma, uint32_t n,
                         const uint8_t *P, uint32_t w, uint32_t h,
                         uint8_t *C, uint8_t H[32], uint32_t threads);

#ifdef __cplusplus
}
#endif
#endif
