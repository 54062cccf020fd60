/*
 * Sanitizer driver for the host side of the C ABI (include/jiffy.h).
 *
 * The test-suite builds the library's host code under AddressSanitizer and
 * UndefinedBehaviorSanitizer (device code left out) and links this driver.
 * It needs no GPU: it drives every entry point's host logic -- layout and
 * argument checks, worst-case sizes, stream-header parsing, the limits of
 * step contexts -- with seeded valid, invalid and extreme values.  Calls
 * that would reach a device return JIFFY_E_DEVICE here, which is accepted.
 * Any out-of-bounds access, overflow of a signed value, shift past the width
 * or other undefined operation aborts the run; otherwise it prints the case
 * count and exits 0.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/jiffy.h"

static uint64_t g_state = 0xD1B54A32D192ED03ull;
static uint64_t next_u64(void) { /* xorshift64* */
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return g_state * 0x2545F4914F6CDD1Dull;
}

static long g_cases = 0;

static void expect(int ok, const char* what, long a) {
    if (!ok) {
        fprintf(stderr, "sanitize host driver: %s (%ld)\n", what, a);
        exit(2);
    }
    g_cases++;
}

static int status_ok(int rc) { return rc == JIFFY_OK || rc == JIFFY_E_INVALID || rc == JIFFY_E_DEVICE || rc == JIFFY_E_CORRUPT || rc == JIFFY_E_CAPACITY || rc == JIFFY_E_SHAPE || rc == JIFFY_E_SCRATCH; }

static jiffy_layout random_layout(void) {
    jiffy_layout L;
    memset(&L, 0, sizeof L);
    static const uint32_t dims[] = {0, 1, 2, 3, 64, 128, 2048, 4096, 65536, 1u << 20, 0x7FFFFFFFu, 0xFFFFFFFFu};
    L.height = dims[next_u64() % (sizeof dims / sizeof dims[0])];
    L.width = dims[next_u64() % (sizeof dims / sizeof dims[0])];
    L.n_attrs = (uint32_t)(next_u64() % 10);
    for (int a = 0; a < JIFFY_MAX_ATTRS; ++a) {
        static const uint8_t wb[] = {0, 1, 2, 3, 4, 8, 255};
        L.width_bytes[a] = wb[next_u64() % 7];
        static const uint32_t P[] = {0, 1, 2, 10, 1000, 0xFFFFFFFFu};
        L.precision[a] = P[next_u64() % 6];
    }
    return L;
}

int main(void) {
    /* worst-case sizes and the layout checks */
    for (int it = 0; it < 200000; ++it) {
        jiffy_layout L = random_layout();
        uint32_t T = (uint32_t)(next_u64() % 4 ? next_u64() % 300 : next_u64());
        size_t b = jiffy_encode_bound(&L, T);
        size_t sb = jiffy_stream_state_bytes(&L);
        expect(b == 0 || b > 20, "encode bound", (long)b);
        (void)sb;
        jiffy_options opt = {(uint32_t)(next_u64() % 6), (uint32_t)(next_u64() % 5)};
        size_t out_len = 0;
        const void* planes[JIFFY_MAX_ATTRS] = {0};
        int rc = jiffy_encode(&L, &opt, T, planes, NULL, 0, &out_len, NULL, NULL);
        expect(rc == JIFFY_E_INVALID, "encode without planes", rc);
        rc = jiffy_encode_noalloc(&L, &opt, T, planes, NULL, 0, &out_len, NULL, NULL);
        expect(rc == JIFFY_E_INVALID, "noalloc encode without planes", rc);
        uint64_t sizes[JIFFY_ABL_SIZES];
        rc = jiffy_ablate(&L, T, T ? NULL : planes, sizes, NULL);
        expect(status_ok(rc), "ablate status", rc);
        jiffy_stream* st = NULL;
        rc = jiffy_stream_create(&L, &opt, &st);
        expect(status_ok(rc) && (rc != JIFFY_OK || st), "stream create status", rc);
        if (st) jiffy_stream_destroy(st);
    }
    /* stream headers: random, then valid ones with random tables */
    uint8_t buf[4096];
    for (int it = 0; it < 200000; ++it) {
        size_t n = (size_t)(next_u64() % sizeof buf);
        for (size_t i = 0; i < n; ++i) buf[i] = (uint8_t)next_u64();
        if (n >= 20 && it % 2) {
            memcpy(buf, "JFY1", 4);
            buf[4] = 1; buf[5] = 0;
            buf[6] = (uint8_t)(next_u64() % 10); buf[7] = 0;
            if (it % 4 == 1) { /* a small T so that the table fits */
                uint32_t T = (uint32_t)(next_u64() % 8);
                memcpy(buf + 16, &T, 4);
            }
        }
        jiffy_layout L;
        uint32_t T = 0;
        int rc = jiffy_peek(buf, n, &L, &T);
        expect(rc == JIFFY_OK || rc == JIFFY_E_CORRUPT, "peek status", rc);
    }
    /* step contexts: limits */
    static const uint64_t S[] = {0, 1, 1u << 20, 1ull << 40, (1ull << 40) + 1, ~0ull};
    static const uint32_t R[] = {0, 1, 1u << 24, (1u << 24) + 1, 0xFFFFFFFFu};
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 6; ++j) {
            size_t w = jiffy_step_workspace_bytes(R[i], S[j]);
            const int valid = R[i] && S[j] && R[i] <= (1u << 24) && S[j] <= (1ull << 40);
            expect(valid ? w > 0 : w == 0, "step workspace limits", (long)(i * 10 + j));
            jiffy_step* st = NULL;
            int rc = jiffy_step_create(R[i], S[j], &st);
            expect(valid ? status_ok(rc) : rc == JIFFY_E_INVALID, "step create limits", rc);
            if (st) jiffy_step_destroy(st);
        }
    /* the other entry points' argument checks */
    jiffy_grid g;
    memset(&g, 0, sizeof g);
    for (int it = 0; it < 100000; ++it) {
        g.height = (uint32_t)(next_u64() % 3 ? next_u64() % 5000 : next_u64());
        g.width = (uint32_t)(next_u64() % 3 ? next_u64() % 5000 : next_u64());
        g.range_bytes = (uint32_t)(next_u64() % 6);
        g.n_attrs = (uint32_t)(next_u64() % 10);
        for (int a = 0; a < JIFFY_MAX_ATTRS; ++a) g.attr_bytes[a] = (uint8_t)(next_u64() % 6);
        g.elev_lo = (double)(int64_t)(next_u64() % 7) - 3.0;
        g.elev_hi = (double)(int64_t)(next_u64() % 7) - 3.0;
        g.range_unit = (double)(int64_t)(next_u64() % 3) * 0.001;
        int rc = jiffy_standardize(&g, (uint32_t)(next_u64() % 4), (uint32_t)(next_u64() % 1000), NULL, NULL, NULL, NULL,
                                   NULL);
        expect(status_ok(rc), "standardize status", rc);
    }
    /* the many-stream calls' argument checks */
    for (int it = 0; it < 100000; ++it) {
        jiffy_layout L = random_layout();
        const uint32_t n = (uint32_t)(next_u64() % 4), T = (uint32_t)(next_u64() % 3 ? next_u64() % 40 : next_u64());
        const void* pl[JIFFY_MAX_ATTRS] = {0};
        const void* const* planes[4] = {pl, pl, pl, pl};
        void* outs[4] = {0};
        size_t caps[4] = {0}, lens[4] = {0};
        jiffy_options opt = {(uint32_t)(next_u64() % 4), 0};
        int rc = jiffy_encode_many(&L, &opt, n, T, it % 3 ? planes : NULL, outs, caps, lens, NULL, NULL);
        expect(n ? rc == JIFFY_E_INVALID : status_ok(rc), "encode_many without planes", rc);
        const void* ins[4] = {0};
        size_t in_lens[4] = {0};
        void* const* po[4] = {0};
        rc = jiffy_decode_many(&L, n, T, it % 3 ? ins : NULL, in_lens, po, NULL);
        expect(n && T ? rc == JIFFY_E_INVALID : status_ok(rc), "decode_many without streams", rc);
    }
    for (int s = -10; s <= 2; ++s) expect(jiffy_status_string(s) != NULL, "status string", s);
    jiffy_tuning t = {(uint32_t)2, 0};
    expect(jiffy_set_tuning(&t) == JIFFY_E_INVALID, "tuning check", 0);
    t.fused = 0;
    expect(jiffy_set_tuning(&t) == JIFFY_OK, "tuning set", 0);
    expect(jiffy_get_tuning(&t, NULL) == JIFFY_OK, "tuning get", 0);
    printf("sanitize host driver: %ld cases, no finding\n", g_cases);
    return 0;
}
