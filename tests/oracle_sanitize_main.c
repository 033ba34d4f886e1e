/*
 * Driver for the sanitizer build of the CPU oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only).  Exercises every entry point
 * of vc_oracle.h over small and ragged shapes and several worker counts, and
 * checks the round trips, so that an out-of-bounds access, a use of
 * uninitialised heap or an undefined shift anywhere in the oracle aborts
 * the run.  Exit status 0 on success.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/vc_oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 11);
}

static int check(int ok, const char *what, uint32_t h, uint32_t w, uint32_t n)
{
    if (!ok) fprintf(stderr, "FAILED %s h=%u w=%u n=%u\n", what, h, w, n);
    return ok ? 0 : 1;
}

int main(void)
{
    static const uint32_t shapes[][2] = {{1, 1}, {1, 4}, {3, 5}, {5, 3}, {17, 5}, {6, 6}, {64, 64}, {33, 100}};
    static const uint32_t ns[] = {1, 2, 3, 6, 32};
    int fails = 0;
    uint8_t digest[32];
    uint8_t msg[300];
    for (int i = 0; i < 300; ++i) msg[i] = (uint8_t)next_u32();
    for (uint64_t len = 0; len <= 300; ++len) vco_sha256(msg, len, digest);

    uint8_t K[32];
    for (int i = 0; i < 32; ++i) K[i] = (uint8_t)next_u32();
    double key[4];
    vco_key_from_bytes(K, key);

    for (size_t si = 0; si < sizeof shapes / sizeof shapes[0]; ++si) {
        const uint32_t h = shapes[si][0], w = shapes[si][1];
        const uint64_t L = 3ull * w * h, ND = 3ull * h + 3ull * w;
        uint8_t *P = malloc(L), *C = malloc(L), *Q = malloc(L), *C2 = malloc(L), *C3 = malloc(L), *Bk = malloc(L);
        uint16_t *D = malloc(2 * ND);
        for (uint64_t k = 0; k < L; ++k) { P[k] = (uint8_t)next_u32(); Bk[k] = (uint8_t)next_u32(); }
        for (uint64_t k = 0; k < ND; ++k) D[k] = (uint16_t)next_u32();
        /* confusion, both forms, both directions */
        vco_confuse_enc(P, w, h, D, Bk, C);
        fails += check(vco_confuse_enc_literal(P, w, h, D, Bk, C2) == 0 && !memcmp(C, C2, L), "literal enc", h, w, 0);
        vco_confuse_dec(C, w, h, D, Bk, Q);
        fails += check(!memcmp(P, Q, L), "closed round trip", h, w, 0);
        fails += check(vco_confuse_dec_literal(C, w, h, D, Bk, Q) == 0 && !memcmp(P, Q, L), "literal round trip", h, w, 0);
        for (size_t ni = 0; ni < sizeof ns / sizeof ns[0]; ++ni) {
            const uint32_t n = ns[ni];
            if (n > L) continue;
            double base[4], base2[4], base3[4], IR[2 * 32 * 4], ic[4], st[4];
            uint8_t H[32], H2[32], H3[32];
            memcpy(base, key, sizeof base);
            memcpy(base2, key, sizeof base2);
            memcpy(base3, key, sizeof base3);
            vco_frame_hash(P, L, n, H);
            vco_reconstruct(base, H, ic);
            memcpy(st, ic, sizeof st);
            fails += check(vco_rk4_step(st, -1.0) == 0, "rk4", h, w, n);
            fails += check(vco_chain(ic, -1.0, n, IR) == 0, "chain", h, w, n);
            fails += check(vco_keystream(IR, -1.0, n, w, h, D, Bk) == 0, "keystream", h, w, n);
            uint8_t ws[100];
            fails += check(vco_worker_stream(IR, -1.0, n - 1, sizeof ws, ws) == 0, "worker stream", h, w, n);
            fails += check(vco_encrypt_frame(base, -1.52, n, P, w, h, C, H2) == 0, "encrypt", h, w, n);
            fails += check(vco_encrypt_frame_mt(base3, -1.52, n, P, w, h, C3, H3, 4) == 0 && !memcmp(C, C3, L) &&
                           !memcmp(H2, H3, 32), "threaded encrypt", h, w, n);
            fails += check(vco_decrypt_frame(base2, -1.52, n, C, w, h, H2, Q) == 0 && !memcmp(P, Q, L) &&
                           !memcmp(base, base2, sizeof base), "decrypt", h, w, n);
        }
        free(P); free(C); free(Q); free(C2); free(C3); free(Bk); free(D);
    }
    if (fails) fprintf(stderr, "%d checks failed\n", fails);
    else printf("sanitized oracle run: all checks passed\n");
    return fails ? 1 : 0;
}
