/*
 * vcipher.h -- C ABI of the MI355X (gfx950) implementation of the
 * diffusion-free per-frame video cipher of arXiv 2505.07158, "Real-Time
 * Bit-Level Encryption of Full High-Definition Video Without Diffusion".
 *
 * One call of encrypt_frames runs, for every frame, the whole per-frame path
 * of the paper on the GPU:
 *   1. the frame hash H, the xor of the SHA-256 digests of n contiguous
 *      sub-frames (Sec. II-A; Alg. 1, Alg. 2);
 *   2. reconstruction of the LHCS_m initial condition from the stream's
 *      chain state and H, then 2n iterations of the hyperchaotic Lorenz
 *      system of Eq. 1 (Sec. II-A; Alg. 1);
 *   3. the n worker LHCS pairs that turn those iterates into shift
 *      distances D and keystream bytes B (Sec. II-B; Alg. 2);
 *   4. bit-level circular row shifts (Eq. 2, Alg. 4) and column shifts
 *      (Eq. 3, Alg. 5) fused with one XOR against B (Alg. 6), i.e. Algs. 3-7
 *      in one pass.
 * decrypt_frames runs steps 2-4 with the exact inverse of step 4 (Sec. II-D
 * states that decryption inverts encryption).
 *
 * Conventions for every function below:
 *  - Return value: VC_OK (0) or a negative vc_status.  No function throws,
 *    aborts or prints.
 *  - Frames are uint8, h rows x w columns x 3 channels, row-major with
 *    interleaved channels (L = 3*w*h bytes, byte (i*w + j)*3 + c), resident
 *    in device memory of the context's GPU.  The caller owns every frame,
 *    output and hash buffer and keeps them alive until the work completes.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    GPU work is enqueued asynchronously on it; host-side validation happens
 *    before anything is enqueued, so a call that fails enqueues nothing and
 *    leaves the chain states untouched.
 *  - Calls on one context are serialised internally (a mutex); chain-state
 *    updates and scratch reuse are ordered by the library in call order, so
 *    consecutive calls may use different streams.  Inputs must be ready on
 *    the stream a call is given (the caller orders its own producers).
 *  - Protocol readings where the paper is silent (integrator, step, byte
 *    order, partitions, layouts) are frozen as protocol version 1; see
 *    vc_protocol_version.
 */
#ifndef VCIPHER_H
#define VCIPHER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VC_OK = 0,
    VC_EINVAL = -1,      /* bad argument, shape, key, alignment or aliasing  */
    VC_ENOMEM = -2,      /* a frame does not fit the context's scratch, or an
                            allocation failed                               */
    VC_EDEVICE = -3,     /* a HIP runtime call failed                        */
    VC_EORDER = -4,      /* frames of a stream out of sequence               */
    VC_ENONFINITE = -5,  /* an LHCS trajectory left the finite range
                            (reported by cipher_status)                      */
    VC_EBUSY = -6        /* the serving loop has work pending (reset,
                            trace replay)                                   */
} vc_status;

/* The user key of Alg. 1 (Require): initial conditions x0, y0, z0, w0 and
 * the control parameter gamma of Eq. 1 (hyperchaotic for
 * -1.52 <= gamma <= -0.06, Sec. II-A), plus n, the worker count of Alg. 2,
 * which the decryptor must match (Sec. V).  1 <= n <= 1024. */
typedef struct {
    double x0, y0, z0, w0;
    double gamma;
    uint32_t n;
} vc_key;

/* Shape and position of one frame.  c must be 3; w, h >= 1; w <= 65535,
 * h <= vc_max_frame_height(ctx) (40956 on MI355X with the default two-pass
 * confusion, whose column pass holds a full-height strip of at least 4
 * bytes per row in one workgroup's LDS); n <= 3*w*h.  `stream` selects a chain (0 <= stream <
 * max_streams of cipher_init); `seq` must equal the stream's next sequence
 * number (0 after cipher_init or cipher_stream_reset), and frames of one
 * stream inside a call appear in increasing seq order. */
typedef struct {
    uint32_t w, h, c;
    uint32_t stream;
    uint64_t seq;
} vc_shape;

/* Opaque context: device-resident chain states, scratch for IR, D and B,
 * descriptor staging. */
typedef struct vc_cipher vc_cipher;

/* Protocol version of the readings this library implements (1). */
uint32_t vc_protocol_version(void);

/* Static description of a status code. Never NULL. */
const char *vc_strerror(int status);

/* Derive x0..w0 from 32 key bytes.  The paper's key is the user inputs x0,
 * y0, z0, w0 and gamma (Sec. II-A, the inputs of Alg. 1) and gives no byte
 * encoding; this is the library's reading (protocol version 1), which
 * takes the key bytes the way Sec. II-A's reconstruction takes the 32 hash
 * bytes: bytes 8k..8k+7 give variable k, integer part = (big-endian u16 of
 * the first two bytes) mod 32 (the upper bound u of Sec. II-A), fraction =
 * the big-endian u48 of the next six bytes times 2^-48 (exact).  gamma and n
 * are copied.  Host only.  VC_EINVAL on NULL pointers, gamma outside
 * [-1.52, -0.06] (the hyperchaotic range of Sec. II-A) or n outside
 * [1, 1024]. */
int vc_key_from_bytes(const uint8_t key32[32], double gamma, uint32_t n, vc_key *out);

/* Create a context on the current HIP device.  max_streams >= 1 chains are
 * set to the key.  scratch_bytes sizes the device scratch for IR, D and B
 * (0 = 2 GiB); larger batches are processed in chunks that fit.  VC_EINVAL
 * for a non-finite x0..w0, gamma outside [-1.52, -0.06], n outside
 * [1, 1024], max_streams == 0 or out == NULL; VC_ENOMEM / VC_EDEVICE on
 * allocation or runtime failure.  *out is NULL on error. */
int cipher_init(const vc_key *key, uint32_t max_streams, size_t scratch_bytes, vc_cipher **out);

/* Release every resource of the context (synchronises its device first).
 * NULL is a no-op. */
void cipher_destroy(vc_cipher *ctx);

/* Encrypt `count` frames.  frames[f] (device, L bytes) is the plaintext,
 * out[f] (device, L bytes) receives the ciphertext, hashes (count*32 bytes)
 * receives each frame's H in FIPS 180-4 digest byte order; the receiver
 * needs H to decrypt (Sec. V: hashes travel with the frames).  Hash buffers
 * here and below may be device memory or pinned host memory
 * (hipHostMalloc): the kernels write and read them in place; any other host
 * memory is rejected with VC_EINVAL (vc_pointer_reachable).
 * out[f] must not overlap frames[f] (the permutation is a gather).
 * Errors: VC_EINVAL (shape, NULL, overlap, hash buffer), VC_EORDER (seq),
 * VC_ENOMEM (frame larger than the scratch), VC_EDEVICE. */
int encrypt_frames(vc_cipher *ctx, size_t count, const uint8_t *const *frames,
                   const vc_shape *shapes, uint8_t *hashes, uint8_t *const *out,
                   void *stream);

/* Decrypt `count` frames with the sender's hashes (count*32 bytes).
 * frames[f] is ciphertext, out[f] receives the plaintext.  Same errors and
 * ordering rules as encrypt_frames. */
int decrypt_frames(vc_cipher *ctx, size_t count, const uint8_t *const *frames,
                   const vc_shape *shapes, const uint8_t *hashes,
                   uint8_t *const *out, void *stream);

/* Size of the fixed device array (one per GPU the library runs on, held
 * until the process ends) that encrypt_frames_noalloc works in. */
#define VC_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc:
 * encrypt_frames (same arguments, same output bytes, hashes and chain
 * updates) without any allocation.  The buffers a call needs beyond the
 * caller's frames, outputs and hashes -- its frame descriptors (the first
 * 1 MiB) and, per frame, the LHCS_m iterates, distances, keystream and the
 * two-pass intermediate image -- live in one fixed array of
 * VC_NOALLOC_SCRATCH_BYTES on the context's GPU instead of the context's
 * scratch; descriptors are staged through a pinned buffer that cipher_init
 * set aside.  The call allocates no device or pinned memory and creates no
 * stream or event; every stage (hash, chain, keystream, confusion) runs on
 * `stream`, in order, without the chain/keystream overlap of
 * encrypt_frames.  Frames are taken in spans that fit the array.
 * Errors, before anything is enqueued: VC_ENOMEM if one frame needs more
 * than VC_NOALLOC_SCRATCH_BYTES - 1 MiB (vc_scratch_per_frame; every frame
 * up to 3840x2160 fits), VC_EINVAL if the descriptors of `count` frames
 * exceed 1 MiB (more than about 9,000 frames), and the errors of
 * encrypt_frames.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (no part of it needs to start at zero:
 * each kernel writes what it later reads): calls that overlap in time on
 * one GPU -- on different streams, from other contexts or threads -- race
 * and give wrong results, so the caller serialises them.  Calls of the same
 * context are ordered with its other calls through events created at
 * cipher_init.  Profiling (vc_profile_enable) does not time its kernels. */
int encrypt_frames_noalloc(vc_cipher *ctx, size_t count, const uint8_t *const *frames,
                           const vc_shape *shapes, uint8_t *hashes, uint8_t *const *out, void *stream);

/* encrypt_frames with the frame hashes already computed (by
 * vc_hash_frames on the same plaintext, possibly on another stream): runs
 * the key schedule and the confusion + XOR only.  hashes (count*32 bytes)
 * is read.  This lets a sender hash batch k+1 while batch k
 * is being encrypted.  If a hash is not the one of Sec. II-A for its frame,
 * the receiver can still decrypt with it, but the output no longer follows
 * the paper's protocol.  Same errors and ordering rules as encrypt_frames. */
int encrypt_frames_hashed(vc_cipher *ctx, size_t count, const uint8_t *const *frames,
                          const vc_shape *shapes, const uint8_t *hashes, uint8_t *const *out,
                          void *stream);

/* Frame hash H of Sec. II-A for each frame (n sub-frames of the context's
 * key), without encrypting and without touching chain states. Only w, h, c
 * of shapes are read. */
int vc_hash_frames(vc_cipher *ctx, size_t count, const uint8_t *const *frames,
                   const vc_shape *shapes, uint8_t *hashes, void *stream);

/* Set a stream's chain back to the key (next seq 0).  Enqueued on the
 * context's last-used stream; synchronous with respect to the host. */
int cipher_stream_reset(vc_cipher *ctx, uint32_t stream);

/* Read / write a stream's chain state: the four LHCS_m values that seed the
 * next frame (x_2n..w_2n of the previous frame, Sec. II-A) and the next
 * sequence number.  Both synchronise the device.  set_state rejects
 * non-finite values (VC_EINVAL). */
int cipher_stream_get_state(vc_cipher *ctx, uint32_t stream, double st[4], uint64_t *next_seq);
int cipher_stream_set_state(vc_cipher *ctx, uint32_t stream, const double st[4], uint64_t next_seq);

/* Synchronise `stream` and report device-side errors raised since the last
 * call: VC_ENONFINITE if an LHCS trajectory became non-finite.  Clears the
 * flag. */
int cipher_status(vc_cipher *ctx, void *stream);

/* Per-kernel timing with HIP events recorded on the launch stream around
 * every kernel launch.  Kernel ids: 0 sha256_subframes, 1 lhcs_chain,
 * 2 lhcs_keygen, 3 confuse_xor_enc, 4 confuse_xor_dec (single-pass
 * confusion), 5 row_shift_enc, 6 col_shift_xor_enc, 7 col_shift_xor_dec,
 * 8 row_shift_dec (two-pass confusion).  vc_profile_read
 * synchronises pending events and returns the summed milliseconds and the
 * launch count since profiling was enabled (or last reset). */
int vc_profile_enable(vc_cipher *ctx, int enable);
int vc_profile_read(vc_cipher *ctx, int kernel_id, double *total_ms, uint64_t *launches);
int vc_profile_reset(vc_cipher *ctx);
const char *vc_kernel_name(int kernel_id);

/* Overlap of the LHCS_m chain with keygen and confusion.  Every chain step
 * of a context runs on one context-owned stream, in call order, after the
 * caller's stream has reached the call.  The scratch is split into
 * `scratch_slots` equal slots (1..4); each span of frames whose IR, D and B
 * fit a slot takes the next slot once its previous user is done.  Each span
 * is cut into `parts` sub-batches in call order (1..64); keygen and
 * confusion of part k run on side stream k mod side_streams (0..8; 0 = on
 * the chain stream), after the chain of part k.  The caller's stream waits
 * for the call's side work before its later work, so results are
 * stream-ordered as usual; a caller that issues consecutive calls on
 * different streams lets the chain of one call overlap the keygen and
 * confusion of the previous one.  Defaults: 3 parts, 3 side streams,
 * 2 slots.  A process whose streams outnumber the device's hardware queues
 * (GPU_MAX_HW_QUEUES, 4 by default in HIP) shares queues between streams,
 * which serialises their work; size the queue count to the streams in use.
 * Changing the slot count waits for the device.  Never changes output
 * bytes.  VC_EINVAL for out-of-range arguments. */
int vc_set_overlap(vc_cipher *ctx, uint32_t parts, uint32_t side_streams, uint32_t scratch_slots);

/* How the confusion + XOR of Sec. II-C (Eqs. 2-3, Algs. 3-7) runs:
 * passes = 2 (default): a row pass (the d_h bit-row rotations, whole rows)
 * and a column pass (the d_v rotations and the XOR with B, full-height
 * strips), through an intermediate image in the scratch -- 15 bytes of
 * HBM traffic per pixel, every access a whole aligned word of a coalesced
 * run; passes = 1: one fused pass per strip (9 bytes per pixel at best, but
 * randomly placed per-channel row windows, and byte-granular scattered
 * writes when decrypting).  Both give identical bytes.  VC_EINVAL unless
 * passes is 1 or 2. */
int vc_set_confusion_passes(vc_cipher *ctx, uint32_t passes);

/* Device scratch one w x h frame needs with worker count n (keystream B,
 * distances D, iterates IR and the two-pass intermediate, each 256-byte
 * aligned): a context's scratch_bytes / scratch_slots should hold the
 * frames of the largest call (else calls are split into spans). */
size_t vc_scratch_per_frame(uint32_t w, uint32_t h, uint32_t n);

/* Autotuner: time the strip-tiled confusion pass (the column pass of the
 * two-pass form, or the single pass) for w x h frames, `frames` per launch
 * (1..4096), over every strip width the LDS holds (see vc_set_tuning) and
 * 256/512/1024 threads, on buffers it allocates and frees itself (contents arbitrary:
 * the kernels are data-oblivious), and remember the fastest for this
 * shape, direction (decrypt 0/1) and pass count.  Later calls use it unless
 * vc_set_tuning fixed a tiling.  Writes the choice to *strip_out and
 * *threads_out when not NULL.  Synchronous.  VC_EINVAL for an unsupported
 * shape, VC_ENOMEM / VC_EDEVICE on device failures. */
int vc_autotune(vc_cipher *ctx, int decrypt, uint32_t w, uint32_t h, uint32_t frames, uint32_t *strip_out,
                uint32_t *threads_out);

/* Strip width of the confusion kernels (0 = automatic; else a power of two
 * from 4 to 128): for the two-pass form, bytes of a row per column-pass
 * strip (the column rotation of Eq. 3 moves each byte column on its own, so
 * strips need not hold whole pixels; 128 bytes = one cache line); for the
 * single-pass form, pixels (at most 64).  A width the LDS cannot hold for a
 * frame's height, or wider than the form allows, falls back to the
 * automatic choice.  threads per workgroup: 256, 512 or 1024 (0 =
 * automatic).  xcd_map: map workgroups so that all strips of one frame run
 * on one XCD.  Tuning never changes output bytes.  VC_EINVAL for other
 * values. */
int vc_set_tuning(vc_cipher *ctx, uint32_t strip_width, uint32_t threads, int xcd_map);

/* Testing entry point: run the confusion + XOR kernels (decrypt = 0) or
 * their inverse (decrypt = 1) on caller-supplied distances D[f] (device,
 * 3h+3w uint16) and keystream B[f] (device, L bytes), with no hash or key
 * schedule.  Same kernels as encrypt_frames / decrypt_frames. */
int vc_debug_confuse(vc_cipher *ctx, int decrypt, size_t count, const uint8_t *const *in,
                     const vc_shape *shapes, const uint16_t *const *D,
                     const uint8_t *const *B, uint8_t *const *out, void *stream);

/* Testing entry point: run the key schedule (steps 2 and 3) for frames with
 * the given hashes, advancing the chains as decrypt_frames would, and write
 * each frame's LHCS_m iterates IR[f] (device, 2n*4 doubles: x,y,z,w of
 * iterations 1..2n), distances D[f] and keystream B[f]. */
int vc_debug_keysched(vc_cipher *ctx, size_t count, const vc_shape *shapes,
                      const uint8_t *hashes, double *const *IR, uint16_t *const *D,
                      uint8_t *const *B, void *stream);

/* Testing entry point: the keystream generation of Sec. II-B (Alg. 2)
 * alone.  For each frame, the n worker LHCS pairs are seeded from the
 * caller's LHCS_m iterates IR[f] (device, 2n x 4 doubles: x, y, z, w of
 * iterations 1..2n) and write distances D[f] (device, 3h+3w uint16) and
 * keystream B[f] (device, L bytes); only w, h, c of shapes are read, and no
 * chain state is read or changed.  A worker trajectory that leaves the
 * finite range raises the device flag that cipher_status reports as
 * VC_ENONFINITE (the outputs are then meaningless but every kernel ends
 * normally).  Same kernel as encrypt_frames. */
int vc_debug_keygen(vc_cipher *ctx, size_t count, const vc_shape *shapes, const double *const *IR,
                    uint16_t *const *D, uint8_t *const *B, void *stream);

/* ---- Statistics of Sec. III (integer reductions; formulas on the host) ----
 * These need no context; each is synchronous (it synchronises `stream`
 * before returning) and uses device memory it allocates and frees itself.
 * Frames follow the conventions above (device, uint8 h x w x 3).
 *
 * vc_frame_histograms: 256-level intensity histogram of every channel of
 * every frame (Sec. III-A, Eqs. 4-5: histogram variance and chi-square;
 * Sec. III-C, Eq. 10: information entropy).  hist: device uint32
 * [count][3][256], overwritten.  VC_EINVAL for bad shapes or NULL pointers. */
int vc_frame_histograms(size_t count, const uint8_t *const *frames, const vc_shape *shapes, uint32_t *hist,
                        void *stream);

/* vc_block_histograms: histograms of `blocks` sub-blocks of block_h x
 * block_w pixels per frame (Sec. III-C, Eq. 11: local Shannon entropy over
 * k randomly chosen non-overlapping blocks of T_B pixels).  origins: HOST
 * uint32 [count][blocks][2] = (row, column) of each block's top-left pixel;
 * every block must lie inside its frame (else VC_EINVAL; overlap is the
 * caller's choice).  hist: device uint32 [count][blocks][3][256]. */
int vc_block_histograms(size_t count, const uint8_t *const *frames, const vc_shape *shapes, uint32_t blocks,
                        uint32_t block_w, uint32_t block_h, const uint32_t *origins, uint32_t *hist, void *stream);

/* vc_pair_moments: exact sums over adjacent pixel pairs (x at (r, c), y its
 * neighbour) of x, y, x^2, y^2 and xy, per direction (0 horizontal (r, c+1),
 * 1 vertical (r+1, c), 2 diagonal (r+1, c+1)) and channel -- the inputs of
 * the correlation coefficient of Sec. III-B, Eqs. 6-9.  positions: HOST
 * uint32 [count][npairs][2] = (r, c) with r < h-1 and c < w-1 (the same
 * positions serve all three directions; else VC_EINVAL), or NULL for every
 * such pixel.  moments: device uint64 [count][3 directions][3 channels][5],
 * overwritten. */
int vc_pair_moments(size_t count, const uint8_t *const *frames, const vc_shape *shapes, uint32_t npairs,
                    const uint32_t *positions, uint64_t *moments, void *stream);

/* vc_max_frame_height: the tallest frame the context accepts under its
 * current confusion form (vc_set_confusion_passes): the column pass keeps a
 * full-height strip of at least 4 bytes per row, the single-pass kernel one
 * of at least 4 pixels, in one workgroup's LDS (Sec. II-C: a column rotation by d_v can move any row to
 * any row).  Taller frames give VC_EINVAL.  0 for a NULL context. */
uint32_t vc_max_frame_height(const vc_cipher *ctx);

/* vc_frame_diff: per channel of each pair of frames a[i], b[i] (both of
 * shapes[i]): the number of differing bytes, the sum of |a - b|, the sum of
 * (a - b)^2 and the number of differing bits -- the counts behind NPCR and
 * UACI (Sec. IV-B, Eqs. 14-16) and behind the PSNR of a frame decrypted
 * after a cropping attack or channel noise (Sec. IV-C).  out: device uint64
 * [count][3 channels][4], overwritten.  Like the statistics calls above it
 * needs no context, synchronises `stream` before returning and allocates
 * and frees its own device memory.  VC_EINVAL for bad shapes or NULL
 * pointers. */
int vc_frame_diff(size_t count, const uint8_t *const *a, const uint8_t *const *b, const vc_shape *shapes,
                  uint64_t *out, void *stream);

/* ---- Prepared batches: launch-only calls for HIP graph capture ----
 * encrypt_frames / decrypt_frames plan every call on the host (shape
 * groups, scratch spans, chain records), stage its descriptors through a
 * pinned ring and fork to the context's streams.  A prepared batch does the
 * planning once: vc_batch_prepare fixes the frames' device buffers, shapes,
 * streams, hash and output buffers, allocates the batch's own scratch and
 * uploads its descriptors to device memory the batch owns.
 * vc_batch_launch then only enqueues kernels on `stream` (the same kernels
 * as encrypt_frames / decrypt_frames, one after another, without the
 * chain/keystream overlap of encrypt_frames) -- no copy, no allocation, no
 * event, no synchronisation -- so one or more launches can be captured in a
 * HIP graph and the graph replayed; a caller overlaps batches by capturing
 * launches of different batches on forked streams.
 *
 * Every launch, and every replay of a graph that captured one, processes
 * the frames then in the batch's input buffers as the next frames of their
 * streams, in the order of `shapes`: the chain states on the device advance
 * (Sec. II-A: each frame's key material starts from the previous frame's
 * iterates).  shapes[f].seq only orders the frames of one stream inside the
 * batch (strictly increasing per stream, else VC_EORDER).  A direct
 * vc_batch_launch advances the context's host-side sequence numbers of the
 * batch's streams (cipher_stream_get_state); a graph replay does not.  The
 * caller orders a context's batch launches with its other calls (they share
 * its chain states), keeps every buffer alive while the batch exists, and
 * must not prepare a batch while another call of the context may be
 * running.  `mode`:
 *   VC_PREP_ENCRYPT: frames are plaintext, hashes (count*32 bytes, device or
 *     pinned host memory) receive H, out the ciphertext (Sec. II, Alg. 1);
 *   VC_PREP_DECRYPT: frames are ciphertext, hashes hold the sender's H;
 *   VC_PREP_HASH: only the frame hash H of each frame (Sec. II-A: the
 *     sub-frame SHA-256 digests xored), into hashes; out may be NULL, the
 *     streams and seqs are not used, no chain advances and the batch holds
 *     no scratch.  H depends on the frame alone, so a caller may hash block
 *     k+1 while block k is encrypted;
 *   VC_PREP_ENCRYPT_HASHED: as VC_PREP_ENCRYPT, with hashes already holding
 *     H of these frames (from a VC_PREP_HASH launch or vc_hash_frames);
 *     the frames are not hashed again.
 * Other values are VC_EINVAL.  Tiling (autotuned or fixed) is taken at
 * prepare time.  Kernel profiling does not time batch launches.  Errors: as
 * encrypt_frames, plus VC_ENOMEM if the batch's scratch cannot be
 * allocated. */
typedef struct vc_batch vc_batch;
enum { VC_PREP_ENCRYPT = 0, VC_PREP_DECRYPT = 1, VC_PREP_HASH = 2, VC_PREP_ENCRYPT_HASHED = 3 };
int vc_batch_prepare(vc_cipher *ctx, int mode, size_t count, const uint8_t *const *frames,
                     const vc_shape *shapes, uint8_t *hashes, uint8_t *const *out, vc_batch **batch);
int vc_batch_launch(vc_batch *batch, void *stream);
/* Frees the batch (synchronises its device first).  NULL is a no-op. */
void vc_batch_destroy(vc_batch *batch);

/* ---- Serving: continuous batching of per-frame requests ----
 * The paper's monitoring system (Sec. V) encrypts every stream frame by frame
 * as frames arrive and reports latency and the delay rate (frames later than
 * one frame interval).  A request is one frame of one stream to encrypt or
 * decrypt.  The scheduler admits requests in arrival order while the device
 * footprint of the requests in flight stays within hbm_budget (a request
 * larger than the whole budget is admitted alone), launches a stream's frame
 * t+1 only with or after frame t (the chain of Sec. II-A is serial per
 * stream) and frames of one stream in one batch in sequence order, forms a
 * batch (one library call) of one class from whatever has arrived whenever
 * fewer than max_inflight batches of its kind and class are in flight, and at
 * most max_batch requests per batch and max_stream_inflight frames of one
 * stream in flight (0 = no limit).  With hash_first an encrypt request is
 * first hashed in a "hash" batch (Sec. II-A's frame hash does not depend on
 * the stream's previous frame), then encrypted in stream order with that
 * hash.  Requests of different kinds are independent (a stream id names a
 * chain of the sender or of the receiver). */
enum { VC_REQ_ENCRYPT = 0, VC_REQ_DECRYPT = 1, VC_BATCH_HASH = 2 };

typedef struct {
    uint64_t tag;          /* the caller's id, returned with the completion */
    int32_t kind;          /* VC_REQ_ENCRYPT or VC_REQ_DECRYPT */
    uint32_t stream;       /* chain of the frame's video stream */
    uint64_t seq;          /* 0, 1, 2, ... per (kind, stream) */
    uint32_t w, h;         /* frame shape (3 channels) */
    uint64_t cls;          /* batch class (vc_sched; the server sets it from w, h) */
    uint64_t nbytes;       /* device bytes held while in flight (server: 0 = input,
                              output and scratch, vc_scratch_per_frame) */
    double arrival;        /* seconds on the caller's clock */
    const uint8_t *frame;  /* device, h*w*3 (server) */
    uint8_t *out;          /* device, h*w*3 (server) */
    uint8_t *hash;         /* 32 bytes (device or pinned host): written when encrypting, read when
                              decrypting (the sender's H) (server) */
} vc_request;

typedef struct {
    uint64_t tag;
    double launched;   /* pump time of the request's first launch */
    double done;       /* pump time at which its batch was seen complete */
    int32_t hashed;    /* went through a hash batch first */
    int32_t status;    /* VC_OK; the status of a batch launch that failed; or
                          VC_EORDER, not launched: an earlier frame of the
                          same stream failed (the stream stays broken until
                          its chain is restarted: vc_server_reset) */
} vc_completion;

typedef struct {
    uint64_t hbm_budget;
    uint32_t max_inflight;         /* per kind and class (0 = 1) */
    uint32_t max_batch;            /* 0 = 512 */
    uint32_t max_stream_inflight;  /* 0 = no limit */
    int32_t hash_first;
    uint32_t max_inflight_hash;    /* hash batches per class (0 = max_inflight): they are
                                      latency-bound and occupy few SIMDs, so a frame that
                                      arrives while one runs need not wait for it */
    uint32_t reserved;             /* 0 */
} vc_sched_config;

typedef struct {
    uint32_t inflight_batches, pending, max_stream_inflight, completed_unpolled;
    uint64_t inflight_bytes, batches_launched;
} vc_sched_stats;

/* The scheduling core over the caller's backend (host only; no device).
 * vc_sched_pump(now): retires batches whose query returns 1 (their requests
 * complete at `now`; hash batches move on to the ordered stage), then calls
 * launch(user, kind, count, tags) for every batch it forms (kind:
 * VC_REQ_ENCRYPT, VC_REQ_DECRYPT or VC_BATCH_HASH; returns a handle >= 0 or a
 * negative status) and returns the number launched (or the first negative
 * status: that batch's requests complete with it, and later frames of their
 * streams complete with VC_EORDER without being launched).  vc_sched_poll returns completions in completion order.  Not
 * thread-safe. */
typedef struct vc_sched vc_sched;
typedef int64_t (*vc_launch_fn)(void *user, int kind, size_t count, const uint64_t *tags);
typedef int (*vc_query_fn)(void *user, int64_t handle);
int vc_sched_create(const vc_sched_config *cfg, vc_sched **out);
int vc_sched_submit(vc_sched *sched, const vc_request *req);
int vc_sched_pump(vc_sched *sched, double now, vc_launch_fn launch, vc_query_fn query, void *user);
size_t vc_sched_poll(vc_sched *sched, vc_completion *out, size_t max);
int vc_sched_get_stats(const vc_sched *sched, vc_sched_stats *stats);
int vc_sched_idle(const vc_sched *sched);
void vc_sched_destroy(vc_sched *sched);

/* The serving loop on the current GPU: the scheduler above with a backend of
 * its own -- per class (one of the `nclasses` resolutions w, h given at
 * creation) a sender and a receiver context (cipher_init with this key,
 * max_streams chains, scratch_bytes of scratch, 0 = hbm_budget / nclasses
 * but at least 1 GiB; vc_set_overlap(parts, side_streams, scratch_slots)
 * when parts > 0), and per kind and class max_inflight (hash batches:
 * max_inflight_hash) device streams used
 * in rotation.  A batch is one call of encrypt_frames (encrypt_frames_hashed
 * after a hash batch), decrypt_frames or vc_hash_frames, with each request's
 * own hash buffer; the key state and scratch stay resident.  The clock is
 * seconds since creation (vc_server_clock).  vc_server_run_trace replays
 * `count` requests sorted by arrival (seconds from the call), submitting each
 * when the clock reaches it and pumping until all are done, and writes
 * done[i] for reqs[i] (times relative to the call); it checks every request
 * (and the order of arrivals) before submitting any, and is VC_EBUSY unless
 * the server is idle with no unpolled completion.  If a launch fails during
 * the replay it returns that status at once: later requests are not
 * submitted, and those already submitted complete through vc_server_poll
 * with their index in reqs as the tag.  vc_server_reset sets
 * every chain back to the key and every stream's next frame back to seq 0
 * (VC_EBUSY unless idle).  Errors: VC_EINVAL for
 * a shape that is not one of the classes, a stream out of range, NULL
 * buffers or a hash buffer that the device cannot reach
 * (vc_pointer_reachable); a failing library call is returned by pump. */
typedef struct vc_server vc_server;
typedef struct {
    vc_sched_config sched;
    uint32_t max_streams;
    uint32_t parts, side_streams, scratch_slots;
    uint64_t scratch_bytes;
} vc_server_config;
int vc_server_create(const vc_key *key, const uint32_t *classes, size_t nclasses, const vc_server_config *cfg,
                     vc_server **out);
double vc_server_clock(const vc_server *server);
int vc_server_submit(vc_server *server, const vc_request *req);
int vc_server_pump(vc_server *server);
size_t vc_server_poll(vc_server *server, vc_completion *out, size_t max);
int vc_server_idle(vc_server *server);
int vc_server_get_stats(vc_server *server, vc_sched_stats *stats);
int vc_server_run_trace(vc_server *server, size_t count, const vc_request *reqs, vc_completion *done);
int vc_server_reset(vc_server *server);
int vc_server_status(vc_server *server);
void vc_server_destroy(vc_server *server);

/* 1 when the kernels can read and write [p, p + bytes) in place: device or
 * managed memory, or pinned host memory that the device addresses at the
 * same address (hipHostMalloc); 0 otherwise (pageable host memory, NULL,
 * bytes == 0, or no device).  The first and the last byte are checked, so
 * the range is expected to lie in one allocation.  The calls above check
 * their hash buffers with it before enqueuing anything.  Host only. */
int vc_pointer_reachable(const void *p, size_t bytes);

/* vc_bandwidth_probe: a measurement helper outside the cipher -- the
 * streaming ceiling that the confusion kernels' HBM rates are compared with.
 * kind 0 copies `bytes` from a to out; kind 1 writes out = a ^ b (two reads
 * and one write per byte, the access mix of the confusion's 9 bytes per
 * pixel).  One 16-byte word per thread, asynchronous on `stream`.  bytes a
 * multiple of 16 and every pointer 16-byte aligned (device memory), else
 * VC_EINVAL. */
int vc_bandwidth_probe(int kind, const uint8_t *a, const uint8_t *b, uint8_t *out, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* VCIPHER_H */
