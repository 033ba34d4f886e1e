/* Test driver in plain C: the library's C ABI used with no Python and no
 * torch.  Device memory comes from hipMalloc, frames from a seeded LCG.
 * Two streams of different shapes (one 16-pixel aligned, one not) are
 * encrypted in one encrypt_frames call, compared byte for byte with the
 * oracle (frame hashes, ciphertext, chain states), decrypted on a second
 * context, and a pageable hash buffer is refused with VC_EINVAL.  Prints
 * "roundtrip ok" and exits 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "vcipher.h"
#include "vc_oracle.h"

#define CHECK(cond, ...)                      \
    do {                                      \
        if (!(cond)) {                        \
            fprintf(stderr, __VA_ARGS__);     \
            fprintf(stderr, "\n");            \
            exit(1);                          \
        }                                     \
    } while (0)

static uint64_t lcg = 0x2505071580ull;
static uint8_t next_byte(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (uint8_t)(lcg >> 56);
}

enum { NF = 5 };

int main(void) {
    const uint32_t n = 8;
    const double gamma = -1.0;
    uint8_t key32[32];
    for (int k = 0; k < 32; ++k) key32[k] = next_byte();
    vc_key key;
    CHECK(vc_key_from_bytes(key32, gamma, n, &key) == VC_OK, "vc_key_from_bytes");

    /* frames 0-2: stream 0, 48x64; frames 3-4: stream 1, 17x23 */
    vc_shape shapes[NF];
    for (int f = 0; f < NF; ++f) {
        const int s = f >= 3;
        shapes[f].w = s ? 23 : 64;
        shapes[f].h = s ? 17 : 48;
        shapes[f].c = 3;
        shapes[f].stream = (uint32_t)s;
        shapes[f].seq = (uint64_t)(s ? f - 3 : f);
    }
    uint8_t *host_p[NF], *host_c[NF], *host_q[NF];
    uint8_t *dev_p[NF], *dev_c[NF], *dev_q[NF];
    size_t L[NF];
    for (int f = 0; f < NF; ++f) {
        L[f] = 3ull * shapes[f].w * shapes[f].h;
        host_p[f] = malloc(L[f]);
        host_c[f] = malloc(L[f]);
        host_q[f] = malloc(L[f]);
        CHECK(host_p[f] && host_c[f] && host_q[f], "malloc");
        for (size_t b = 0; b < L[f]; ++b) host_p[f][b] = next_byte();
        CHECK(hipMalloc((void **)&dev_p[f], L[f]) == hipSuccess, "hipMalloc");
        CHECK(hipMalloc((void **)&dev_c[f], L[f]) == hipSuccess, "hipMalloc");
        CHECK(hipMalloc((void **)&dev_q[f], L[f]) == hipSuccess, "hipMalloc");
        CHECK(hipMemcpy(dev_p[f], host_p[f], L[f], hipMemcpyHostToDevice) == hipSuccess, "hipMemcpy");
    }
    uint8_t *dev_h = NULL;
    CHECK(hipMalloc((void **)&dev_h, 32 * NF) == hipSuccess, "hipMalloc");
    hipStream_t st;
    CHECK(hipStreamCreate(&st) == hipSuccess, "hipStreamCreate");

    vc_cipher *enc = NULL, *dec = NULL;
    CHECK(cipher_init(&key, 2, 0, &enc) == VC_OK, "cipher_init");
    CHECK(cipher_init(&key, 2, 0, &dec) == VC_OK, "cipher_init");

    /* a pageable hash buffer: classified first, then refused before enqueue */
    uint8_t pageable[32 * NF];
    CHECK(vc_pointer_reachable(pageable, sizeof pageable) == 0, "pageable memory classified as reachable");
    CHECK(vc_pointer_reachable(dev_h, 32 * NF) == 1, "device memory classified as unreachable");
    CHECK(encrypt_frames(enc, NF, (const uint8_t *const *)dev_p, shapes, pageable, dev_c, st) == VC_EINVAL,
          "pageable hash buffer accepted");

    CHECK(encrypt_frames(enc, NF, (const uint8_t *const *)dev_p, shapes, dev_h, dev_c, st) == VC_OK,
          "encrypt_frames");
    uint8_t host_h[32 * NF];
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync");
    CHECK(hipMemcpy(host_h, dev_h, sizeof host_h, hipMemcpyDeviceToHost) == hipSuccess, "hipMemcpy");
    for (int f = 0; f < NF; ++f)
        CHECK(hipMemcpy(host_c[f], dev_c[f], L[f], hipMemcpyDeviceToHost) == hipSuccess, "hipMemcpy");
    CHECK(cipher_status(enc, st) == VC_OK, "cipher_status");

    /* the oracle, stream by stream from the key */
    double base[2][4];
    vco_key_from_bytes(key32, base[0]);
    vco_key_from_bytes(key32, base[1]);
    uint8_t *ref = malloc(L[0] > L[3] ? L[0] : L[3]);
    CHECK(ref != NULL, "malloc");
    for (int f = 0; f < NF; ++f) {
        uint8_t H[32];
        const int s = (int)shapes[f].stream;
        CHECK(vco_encrypt_frame(base[s], gamma, n, host_p[f], shapes[f].w, shapes[f].h, ref, H) == 0, "oracle");
        CHECK(memcmp(H, host_h + 32 * f, 32) == 0, "frame %d: hash differs from the oracle", f);
        CHECK(memcmp(ref, host_c[f], L[f]) == 0, "frame %d: ciphertext differs from the oracle", f);
    }
    for (uint32_t s = 0; s < 2; ++s) {
        double state[4];
        uint64_t next = 0;
        CHECK(cipher_stream_get_state(enc, s, state, &next) == VC_OK, "get_state");
        CHECK(memcmp(state, base[s], sizeof state) == 0 && next == (s ? 2u : 3u), "stream %u: chain state", s);
    }

    CHECK(decrypt_frames(dec, NF, (const uint8_t *const *)dev_c, shapes, dev_h, dev_q, st) == VC_OK,
          "decrypt_frames");
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync");
    for (int f = 0; f < NF; ++f) {
        CHECK(hipMemcpy(host_q[f], dev_q[f], L[f], hipMemcpyDeviceToHost) == hipSuccess, "hipMemcpy");
        CHECK(memcmp(host_q[f], host_p[f], L[f]) == 0, "frame %d: decrypt(encrypt(x)) != x", f);
    }
    CHECK(cipher_status(dec, st) == VC_OK, "cipher_status");

    cipher_destroy(enc);
    cipher_destroy(dec);
    (void)hipStreamDestroy(st);
    for (int f = 0; f < NF; ++f) {
        (void)hipFree(dev_p[f]);
        (void)hipFree(dev_c[f]);
        (void)hipFree(dev_q[f]);
        free(host_p[f]);
        free(host_c[f]);
        free(host_q[f]);
    }
    (void)hipFree(dev_h);
    free(ref);
    printf("roundtrip ok\n");
    return 0;
}
