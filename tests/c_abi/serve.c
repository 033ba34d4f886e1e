/* Test driver in plain C for the library's serving loop (vc_server_*): no
 * Python and no torch.  Four video streams of two resolutions (three
 * encrypt streams, one decrypt stream whose ciphertext comes from a
 * separate sender context), three frames each, submitted out of order to a
 * server with hash-first batches; every served frame is compared with the
 * oracle (frame hashes and ciphertext, each stream's chain from the key) or
 * with the plaintext.  The server is then reset and the same requests are
 * replayed with staggered arrival times through vc_server_run_trace, with
 * the same results.  Prints "serve ok" and exits 0 on success. */
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

static uint64_t lcg = 0x5e7e0c0deull;
static uint32_t next_u32(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(lcg >> 32);
}

enum { S = 4, T = 3, NR = S * T };

static const uint32_t W[S] = {64, 23, 64, 64}, H[S] = {48, 17, 48, 48};
static const int DEC[S] = {0, 0, 0, 1};

static uint8_t *host_p[S][T], *dev_p[S][T], *dev_c[S][T], *dev_out[S][T];
static uint8_t *dev_hash; /* 32 bytes per request */

static size_t frame_bytes(int s) { return 3ull * W[s] * H[s]; }

/* request r = s * T + t: frame t of stream s */
static vc_request make_request(int r, double arrival) {
    const int s = r / T, t = r % T;
    vc_request q;
    memset(&q, 0, sizeof q);
    q.tag = (uint64_t)r;
    q.kind = DEC[s] ? VC_REQ_DECRYPT : VC_REQ_ENCRYPT;
    q.stream = (uint32_t)s;
    q.seq = (uint64_t)t;
    q.w = W[s];
    q.h = H[s];
    q.arrival = arrival;
    q.frame = DEC[s] ? dev_c[s][t] : dev_p[s][t];
    q.out = dev_out[s][t];
    q.hash = dev_hash + 32 * r;
    return q;
}

/* every served frame against the oracle (encrypt) or the plaintext (decrypt) */
static void check_outputs(const uint8_t key32[32], double gamma, uint32_t n, const char *what) {
    uint8_t hashes[32 * NR];
    CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
    CHECK(hipMemcpy(hashes, dev_hash, sizeof hashes, hipMemcpyDeviceToHost) == hipSuccess, "hipMemcpy");
    uint8_t *got = malloc(frame_bytes(0)), *ref = malloc(frame_bytes(0));
    CHECK(got && ref, "malloc");
    for (int s = 0; s < S; ++s) {
        double base[4];
        vco_key_from_bytes(key32, base);
        for (int t = 0; t < T; ++t) {
            const size_t L = frame_bytes(s);
            CHECK(hipMemcpy(got, dev_out[s][t], L, hipMemcpyDeviceToHost) == hipSuccess, "hipMemcpy");
            if (DEC[s]) {
                CHECK(memcmp(got, host_p[s][t], L) == 0, "%s: stream %d frame %d: decrypted frame differs", what,
                      s, t);
                continue;
            }
            uint8_t Href[32];
            CHECK(vco_encrypt_frame(base, gamma, n, host_p[s][t], W[s], H[s], ref, Href) == 0, "oracle");
            CHECK(memcmp(Href, hashes + 32 * (s * T + t), 32) == 0, "%s: stream %d frame %d: hash differs", what, s,
                  t);
            CHECK(memcmp(ref, got, L) == 0, "%s: stream %d frame %d: ciphertext differs", what, s, t);
        }
    }
    free(got);
    free(ref);
}

int main(void) {
    const uint32_t n = 6;
    const double gamma = -0.5;
    uint8_t key32[32];
    for (int k = 0; k < 32; ++k) key32[k] = (uint8_t)next_u32();
    vc_key key;
    CHECK(vc_key_from_bytes(key32, gamma, n, &key) == VC_OK, "vc_key_from_bytes");

    for (int s = 0; s < S; ++s)
        for (int t = 0; t < T; ++t) {
            const size_t L = frame_bytes(s);
            host_p[s][t] = malloc(L);
            CHECK(host_p[s][t] != NULL, "malloc");
            for (size_t b = 0; b < L; ++b) host_p[s][t][b] = (uint8_t)next_u32();
            CHECK(hipMalloc((void **)&dev_p[s][t], L) == hipSuccess, "hipMalloc");
            CHECK(hipMalloc((void **)&dev_c[s][t], L) == hipSuccess, "hipMalloc");
            CHECK(hipMalloc((void **)&dev_out[s][t], L) == hipSuccess, "hipMalloc");
            CHECK(hipMemcpy(dev_p[s][t], host_p[s][t], L, hipMemcpyHostToDevice) == hipSuccess, "hipMemcpy");
        }
    CHECK(hipMalloc((void **)&dev_hash, 32 * NR) == hipSuccess, "hipMalloc");

    /* the decrypt stream's ciphertext and hashes, from a sender context */
    {
        vc_cipher *snd = NULL;
        CHECK(cipher_init(&key, S, 0, &snd) == VC_OK, "cipher_init");
        const int s = 3;
        vc_shape sh[T];
        const uint8_t *in[T];
        uint8_t *out[T];
        for (int t = 0; t < T; ++t) {
            sh[t].w = W[s];
            sh[t].h = H[s];
            sh[t].c = 3;
            sh[t].stream = (uint32_t)s;
            sh[t].seq = (uint64_t)t;
            in[t] = dev_p[s][t];
            out[t] = dev_c[s][t];
        }
        CHECK(encrypt_frames(snd, T, in, sh, dev_hash + 32 * (s * T), out, NULL) == VC_OK, "sender encrypt_frames");
        CHECK(cipher_status(snd, NULL) == VC_OK, "sender status");
        cipher_destroy(snd);
    }

    const uint32_t classes[4] = {64, 48, 23, 17};
    vc_server_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.sched.hbm_budget = 1ull << 28;
    cfg.sched.max_inflight = 2;
    cfg.sched.max_batch = 4;
    cfg.sched.hash_first = 1;
    cfg.max_streams = S;
    cfg.scratch_bytes = 64ull << 20;
    vc_server *srv = NULL;
    CHECK(vc_server_create(&key, classes, 2, &cfg, &srv) == VC_OK, "vc_server_create");

    /* out of order: a fixed shuffle of the requests */
    int order[NR];
    for (int r = 0; r < NR; ++r) order[r] = r;
    for (int r = NR - 1; r > 0; --r) {
        const int j = (int)(next_u32() % (uint32_t)(r + 1));
        const int x = order[r];
        order[r] = order[j];
        order[j] = x;
    }
    vc_completion done[NR];
    int seen[NR] = {0}, got = 0;
    vc_completion buf[16];
    for (int k = 0; k < NR; ++k) {
        vc_request q = make_request(order[k], 0.0);
        CHECK(vc_server_submit(srv, &q) == VC_OK, "vc_server_submit");
        CHECK(vc_server_pump(srv) >= 0, "vc_server_pump");
    }
    const double t0 = vc_server_clock(srv);
    while (got < NR) {
        CHECK(vc_server_clock(srv) - t0 < 60.0, "the server did not finish within 60 s");
        CHECK(vc_server_pump(srv) >= 0, "vc_server_pump");
        const size_t m = vc_server_poll(srv, buf, 16);
        for (size_t i = 0; i < m; ++i) {
            const int r = (int)buf[i].tag;
            CHECK(r >= 0 && r < NR && !seen[r], "unexpected completion %d", r);
            CHECK(buf[i].status == VC_OK, "request %d: status %d", r, buf[i].status);
            seen[r] = 1;
            done[r] = buf[i];
            ++got;
        }
    }
    CHECK(vc_server_idle(srv) == 1, "not idle after every completion");
    for (int r = 0; r < NR; ++r)
        CHECK(done[r].hashed == (DEC[r / T] ? 0 : 1), "request %d: hash-first flag", r);
    check_outputs(key32, gamma, n, "submit/pump/poll");
    vc_sched_stats st;
    CHECK(vc_server_get_stats(srv, &st) == VC_OK, "stats");
    CHECK(st.batches_launched >= 3 && st.inflight_bytes == 0, "stats after the run");

    /* the same requests again from frame 0, replayed by the library's loop */
    CHECK(vc_server_reset(srv) == VC_OK, "vc_server_reset");
    for (int s = 0; s < S; ++s)
        for (int t = 0; t < T; ++t) CHECK(hipMemset(dev_out[s][t], 0, frame_bytes(s)) == hipSuccess, "hipMemset");
    vc_request trace[NR];
    int k = 0;
    for (int t = 0; t < T; ++t) /* sorted by arrival: frame t of every stream at 1 ms * t */
        for (int s = 0; s < S; ++s) trace[k++] = make_request(s * T + t, 0.001 * t);
    vc_completion tdone[NR];
    CHECK(vc_server_run_trace(srv, NR, trace, tdone) == VC_OK, "vc_server_run_trace");
    for (int i = 0; i < NR; ++i)
        CHECK(tdone[i].tag == trace[i].tag && tdone[i].status == VC_OK && tdone[i].done >= tdone[i].launched,
              "trace completion %d", i);
    check_outputs(key32, gamma, n, "run_trace");
    CHECK(vc_server_status(srv) == VC_OK, "vc_server_status");
    vc_server_destroy(srv);

    for (int s = 0; s < S; ++s)
        for (int t = 0; t < T; ++t) {
            (void)hipFree(dev_p[s][t]);
            (void)hipFree(dev_c[s][t]);
            (void)hipFree(dev_out[s][t]);
            free(host_p[s][t]);
        }
    (void)hipFree(dev_hash);
    printf("serve ok\n");
    return 0;
}
