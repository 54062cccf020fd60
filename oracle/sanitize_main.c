/*
 * Sanitizer driver for the CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Built together with jiffy_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by the test-suite.  It drives every entry point
 * with seeded inputs: whole sequences of several shapes, sample widths,
 * precisions and modes are encoded and decoded (the decode must restore the
 * quantized samples), then every truncation and many byte and bit flips of
 * small streams are decoded (each must return OK or ORC_E_CORRUPT), and the
 * section and frame readers get random bytes.  Any out-of-bounds access or
 * undefined operation aborts the run; otherwise it prints the case count
 * and exits 0.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "jiffy_oracle.h"

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) { /* xorshift64* */
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return g_state * 0x2545F4914F6CDD1Dull;
}

static void fail(const char* what, int a, int b) {
    fprintf(stderr, "sanitize driver: %s (%d, %d)\n", what, a, b);
    exit(2);
}

static uint64_t get(const void* p, unsigned wb, size_t i) {
    if (wb == 1) return ((const uint8_t*)p)[i];
    if (wb == 2) return ((const uint16_t*)p)[i];
    return ((const uint32_t*)p)[i];
}

static long g_cases = 0;

/* encodes a random sequence and checks the decode; returns the stream (caller frees) */
static uint8_t* round_trip(uint32_t H, uint32_t W, uint32_t T, unsigned A, const unsigned* wb, const uint32_t* P,
                           unsigned mode, unsigned zero_pct, size_t* len_out) {
    orc_layout L;
    memset(&L, 0, sizeof L);
    L.height = H;
    L.width = W;
    L.n_attrs = A;
    size_t npx = (size_t)H * W;
    void* planes[ORC_MAX_ATTRS];
    void* outs[ORC_MAX_ATTRS];
    for (unsigned a = 0; a < A; ++a) {
        L.width_bytes[a] = (uint8_t)wb[a];
        L.precision[a] = P[a];
        planes[a] = malloc(npx * T * wb[a]);
        outs[a] = malloc(npx * T * wb[a]);
        uint64_t top = wb[a] == 4 ? 0xFFFFFFFFull : (1ull << (8 * wb[a])) - 1;
        for (size_t i = 0; i < npx * T; ++i) {
            uint64_t v = next_u64();
            uint64_t x = (v % 100 < zero_pct) ? 0 : ((i % 7 == 0) ? (v >> 16) & top : 1000 + (v >> 40) % 50);
            if (x > top) x = top;
            if (wb[a] == 1) ((uint8_t*)planes[a])[i] = (uint8_t)x;
            else if (wb[a] == 2) ((uint16_t*)planes[a])[i] = (uint16_t)x;
            else ((uint32_t*)planes[a])[i] = (uint32_t)x;
        }
    }
    orc_options opt = {mode, 0};
    size_t cap = orc_encode_bound(&L, T);
    uint8_t* out = (uint8_t*)malloc(cap);
    uint8_t* modes = (uint8_t*)malloc((size_t)T * A + 1);
    size_t len = 0;
    int rc = orc_encode(&L, &opt, T, (const void* const*)planes, NULL, out, cap, &len, modes);
    if (rc) fail("encode", rc, (int)mode);
    rc = orc_decode(out, len, outs);
    if (rc) fail("decode", rc, (int)mode);
    for (unsigned a = 0; a < A; ++a) {
        for (size_t i = 0; i < npx * T; ++i) {
            uint64_t want = orc_dequantize(orc_quantize(get(planes[a], wb[a], i), P[a]), P[a], 8 * wb[a]);
            if (get(outs[a], wb[a], i) != want) fail("round trip", (int)a, (int)i);
        }
        free(planes[a]);
        free(outs[a]);
    }
    free(modes);
    g_cases++;
    *len_out = len;
    return out;
}

/* every truncation and a set of byte and bit flips of one stream */
static void mutate(const uint8_t* s, size_t len, uint32_t H, uint32_t W, uint32_t T, unsigned A, const unsigned* wb) {
    size_t npx = (size_t)H * W;
    void* outs[ORC_MAX_ATTRS];
    for (unsigned a = 0; a < A; ++a) outs[a] = malloc(npx * T * wb[a] + 8);
    uint8_t* b = (uint8_t*)malloc(len + 8);
    for (size_t cut = 0; cut < len; ++cut) {
        memcpy(b, s, cut);
        uint8_t* exact = (uint8_t*)malloc(cut ? cut : 1);
        memcpy(exact, b, cut);
        int rc = orc_decode(exact, cut, outs);
        if (rc != ORC_OK && rc != ORC_E_CORRUPT) fail("truncated decode status", rc, (int)cut);
        free(exact);
        g_cases++;
    }
    for (size_t pos = 0; pos < len; ++pos) {
        for (int k = 0; k < 3; ++k) {
            memcpy(b, s, len);
            if (k == 0) b[pos] ^= (uint8_t)(1u << (next_u64() % 8));
            else if (k == 1) b[pos] = (uint8_t)next_u64();
            else b[pos] = 0xFF;
            orc_layout L2;
            uint32_t T2;
            if (orc_peek(b, len, &L2, &T2) == ORC_OK) {
                /* a header flip can change the shape: decode only what fits the buffers */
                size_t need = (size_t)L2.height * L2.width * T2;
                int fits = L2.n_attrs == A;
                for (unsigned a = 0; fits && a < A; ++a) fits = L2.width_bytes[a] <= wb[a] && need <= npx * T;
                if (fits) {
                    int rc = orc_decode(b, len, outs);
                    if (rc != ORC_OK && rc != ORC_E_CORRUPT) fail("flipped decode status", rc, (int)pos);
                }
            }
            g_cases++;
        }
    }
    free(b);
    for (unsigned a = 0; a < A; ++a) free(outs[a]);
}

int main(void) {
    static const uint32_t shapes[][3] = {{1, 1, 2}, {3, 7, 3}, {2, 64, 4}, {16, 40, 3}, {5, 300, 2}};
    static const unsigned widths[][3] = {{4, 2, 1}, {2, 2, 2}, {1, 4, 2}};
    static const uint32_t precs[][3] = {{1, 1, 1}, {10, 3, 1}, {1000, 1, 2}};
    for (unsigned si = 0; si < sizeof shapes / sizeof shapes[0]; ++si) {
        for (unsigned wi = 0; wi < 3; ++wi) {
            for (unsigned mode = 0; mode < 4; ++mode) {
                for (unsigned zp = 0; zp <= 100; zp += 50) {
                    size_t len;
                    const uint32_t H = shapes[si][0], W = shapes[si][1], T = shapes[si][2];
                    uint8_t* s = round_trip(H, W, T, 3, widths[wi], precs[wi], mode, zp, &len);
                    if (si < 3 && zp == 50) mutate(s, len, H, W, T, 3, widths[wi]);
                    free(s);
                }
            }
        }
    }
    /* the section and frame readers on random bytes */
    uint8_t buf[600];
    uint32_t z[1024];
    for (int it = 0; it < 20000; ++it) {
        size_t n = next_u64() % sizeof buf;
        for (size_t i = 0; i < n; ++i) buf[i] = (uint8_t)next_u64();
        if (n >= 4 && it % 2) { buf[0] = (uint8_t)(next_u64() % 300); buf[1] = buf[2] = buf[3] = 0; }
        size_t used;
        unsigned bits = 8u << (next_u64() % 3);
        (void)orc_pfor_decode(buf, n, bits, (uint32_t)(next_u64() % 1024), z, &used);
        uint8_t mask[512];
        if (n >= 4) { buf[0] = 0x28; buf[1] = 0xB5; buf[2] = 0x2F; buf[3] = 0xFD; }
        (void)orc_unframe(buf, n, mask, next_u64() % sizeof mask);
        g_cases++;
    }
    printf("sanitize driver: %ld cases, no finding\n", g_cases);
    return 0;
}
