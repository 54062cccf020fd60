/*
 * Jiffy CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, scalar, deliberately slow reference of the Jiffy LiDAR scan codec
 * (Ford & Ford, "Lossless SIMD Compression of LiDAR Range and Attribute Scan
 * Sequences", arXiv 2209.08196).  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no source,
 * header, table or helper with the GPU library; its types are declared here
 * on their own on purpose.
 *
 * The paper fixes the order of the steps (Sec. III, Fig. 2): quantize
 * (Sec. III-B), zero bitmask (Sec. III-C), I/P choice by trial compression
 * (Sec. III-E), mask XOR for P-scans (Sec. III-D), zero removal, temporal
 * difference for P-scans (Sec. III-D), horizontal delta (Sec. III-C),
 * ZigZag (Eq. 1), patched frame-of-reference packing (Sec. II, III-C).
 * Where the paper leaves a byte layout or a rounding open, the project's
 * reading is used; every such reading is listed with the design notes.
 */
#ifndef JIFFY_ORACLE_H
#define JIFFY_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_ATTRS 8

typedef struct {
    uint32_t height, width, n_attrs;
    uint8_t width_bytes[ORC_MAX_ATTRS]; /* 1, 2 or 4 */
    uint32_t precision[ORC_MAX_ATTRS];  /* quantization step P >= 1 */
} orc_layout;

typedef struct {
    uint32_t mode;       /* 0 auto (trial), 1 I only, 2 P only, 3 brute force (smaller record) */
    uint32_t trial_rows; /* 0 means the default of 4 */
} orc_options;

enum {
    ORC_OK = 0,
    ORC_E_INVALID = -1,
    ORC_E_CAPACITY = -2,
    ORC_E_CORRUPT = -3,
};

/* ---- single steps, exported so that tests can pin each one ---- */
uint64_t orc_quantize(uint64_t x, uint32_t precision);
uint64_t orc_dequantize(uint64_t q, uint32_t precision, unsigned bits);
uint32_t orc_zigzag(uint32_t d, unsigned bits);
uint32_t orc_unzigzag(uint32_t z, unsigned bits);
/* width choice for one frame of 128 values; returns its packed byte cost */
uint32_t orc_pfor_choose(const uint32_t z[128], unsigned* b, unsigned* n_exc, unsigned* max_bits);
/* sum of the frame costs of z[0..n) (the trial-compression measure) */
uint64_t orc_pfor_cost(const uint32_t* z, size_t n);
/* a whole residual section; returns bytes written or needed (out may be NULL) */
size_t orc_pfor_encode(const uint32_t* z, uint32_t n, uint8_t* out, size_t cap);
/* parses a section; *n_out gets the count, z must hold n_max values */
int orc_pfor_decode(const uint8_t* in, size_t len, unsigned bits, uint32_t n_expect, uint32_t* z, size_t* used);
/* mask frame (Zstd frame restricted to Raw and RLE blocks) */
size_t orc_frame(const uint8_t* in, size_t n, uint8_t* out, size_t cap);
int orc_unframe(const uint8_t* in, size_t len, uint8_t* out, size_t n_expect);
/* rows used by the trial compression; returns their count */
unsigned orc_trial_rows(uint32_t height, uint32_t k, uint32_t* rows);

/* ---- whole codec ---- */
size_t orc_encode_bound(const orc_layout* layout, uint32_t n_scans);
/* planes[a] points at n_scans*H*W samples of attribute a (host memory).
 * prev_planes (may be NULL) gives one previous scan per attribute that the
 * first scan may predict from; without it the first scan is an I-scan. */
int orc_encode(const orc_layout* layout, const orc_options* opt, uint32_t n_scans,
               const void* const* planes, const void* const* prev_planes,
               uint8_t* out, size_t cap, size_t* out_len, uint8_t* modes);
int orc_peek(const uint8_t* in, size_t len, orc_layout* layout, uint32_t* n_scans);
int orc_decode(const uint8_t* in, size_t len, void* const* planes_out);

#ifdef __cplusplus
}
#endif
#endif
