/*
 * Jiffy CPU oracle -- TEST INFRASTRUCTURE ONLY (see jiffy_oracle.h).
 *
 * Scalar C99, one sample at a time, no blocking or fusion beyond what the
 * paper's description states.  Section references are to Ford & Ford,
 * arXiv 2209.08196.  Byte layout (stream header, record, residual section,
 * mask frame) is the project's reading of the places where the paper is
 * silent; it is written out once, here, in the order the paper lists the
 * steps.
 */
#include "jiffy_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* growable little-endian byte buffer                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint8_t* p;
    size_t n, cap;
    int oom;
} obuf;

static void ob_reserve(obuf* b, size_t extra) {
    if (b->oom || b->n + extra <= b->cap) return;
    size_t nc = b->cap ? b->cap : 256;
    while (nc < b->n + extra) nc *= 2;
    uint8_t* np = (uint8_t*)realloc(b->p, nc);
    if (!np) { b->oom = 1; return; }
    b->p = np;
    b->cap = nc;
}
static void ob_put(obuf* b, const void* src, size_t n) {
    ob_reserve(b, n);
    if (b->oom) return;
    memcpy(b->p + b->n, src, n);
    b->n += n;
}
static void ob_u8(obuf* b, uint8_t v) { ob_put(b, &v, 1); }
static void ob_u16(obuf* b, uint16_t v) {
    uint8_t t[2] = {(uint8_t)v, (uint8_t)(v >> 8)};
    ob_put(b, t, 2);
}
static void ob_u32(obuf* b, uint32_t v) {
    uint8_t t[4] = {(uint8_t)v, (uint8_t)(v >> 8), (uint8_t)(v >> 16), (uint8_t)(v >> 24)};
    ob_put(b, t, 4);
}
static void ob_pad4(obuf* b) {
    while (b->n % 4) ob_u8(b, 0);
}
static uint32_t rd_u32(const uint8_t* p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static uint16_t rd_u16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }

/* ------------------------------------------------------------------------ */
/* Sec. III-B: quantization to a user precision P                            */
/* ------------------------------------------------------------------------ */

/* Zero is the invalid sentinel (Sec. III-A) and stays zero.  Otherwise the
 * sample goes to the nearest multiple of P, halves rounded up, so the
 * round-trip error is at most floor(P/2) (Sec. III-B, Fig. 4 caption).  A
 * valid sample never becomes the sentinel: it is clamped to 1. */
uint64_t orc_quantize(uint64_t x, uint32_t precision) {
    if (x == 0) return 0;
    uint64_t q = (x + precision / 2) / precision;
    return q == 0 ? 1 : q;
}

/* The stored precision restores the original representation (Sec. III-A);
 * a product beyond the sample width saturates. */
uint64_t orc_dequantize(uint64_t q, uint32_t precision, unsigned bits) {
    uint64_t top = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
    uint64_t x = q * (uint64_t)precision;
    return x > top ? top : x;
}

/* ------------------------------------------------------------------------ */
/* Eq. 1: ZigZag.  The printed case for negative x is garbled; the standard  */
/* map the paper names is used: x >= 0 -> 2x, x < 0 -> 2|x| - 1.             */
/* ------------------------------------------------------------------------ */
static uint64_t low_mask(unsigned bits) { return bits >= 64 ? ~0ull : ((1ull << bits) - 1); }

static int64_t as_signed(uint64_t d, unsigned bits) {
    d &= low_mask(bits);
    if (d >> (bits - 1)) return (int64_t)d - (int64_t)(1ull << bits);
    return (int64_t)d;
}

uint32_t orc_zigzag(uint32_t d, unsigned bits) {
    int64_t x = as_signed(d, bits);
    if (x >= 0) return (uint32_t)(2 * x);
    return (uint32_t)(-2 * x - 1);
}

uint32_t orc_unzigzag(uint32_t z, unsigned bits) {
    int64_t x = (z & 1u) ? -(int64_t)(((uint64_t)z + 1) / 2) : (int64_t)(z / 2);
    return (uint32_t)((uint64_t)x & low_mask(bits));
}

/* ------------------------------------------------------------------------ */
/* Sec. II / III-C: patched frame of reference over frames of 128 values.   */
/* The frame reference is 0 (ZigZag output is non-negative and small);       */
/* values that do not fit in b bits are patched from an exception list.      */
/* ------------------------------------------------------------------------ */
static unsigned bit_width(uint32_t v) {
    unsigned b = 0;
    while (v) { b++; v >>= 1; }
    return b;
}

static int exceeds(uint32_t v, unsigned b) { return b < 32 && (v >> b) != 0; }

uint32_t orc_pfor_choose(const uint32_t z[128], unsigned* b_out, unsigned* n_out, unsigned* B_out) {
    uint32_t mx = 0;
    for (int i = 0; i < 128; ++i) if (z[i] > mx) mx = z[i];
    unsigned B = bit_width(mx);
    uint32_t best = 0xFFFFFFFFu;
    unsigned best_b = 0, best_n = 0;
    for (unsigned b = 0; b <= B; ++b) {
        unsigned n = 0;
        for (int i = 0; i < 128; ++i) n += exceeds(z[i], b);
        /* payload of 128 b-bit slots, one position byte per exception, and
         * the exceptions' high parts at B-b bits each */
        uint32_t cost = 16u * b + (n ? n + (n * (B - b) + 7) / 8 : 0);
        if (cost <= best) { /* ties go to the larger b */
            best = cost;
            best_b = b;
            best_n = n;
        }
    }
    if (b_out) *b_out = best_b;
    if (n_out) *n_out = best_n;
    if (B_out) *B_out = B;
    return best;
}

static void load_frame(const uint32_t* z, size_t n, size_t j, uint32_t f[128]) {
    for (size_t i = 0; i < 128; ++i) {
        size_t k = 128 * j + i;
        f[i] = k < n ? z[k] : 0; /* the last frame is padded with zeros */
    }
}

uint64_t orc_pfor_cost(const uint32_t* z, size_t n) {
    uint64_t total = 0;
    size_t nb = (n + 127) / 128;
    uint32_t f[128];
    for (size_t j = 0; j < nb; ++j) {
        load_frame(z, n, j, f);
        total += orc_pfor_choose(f, NULL, NULL, NULL);
    }
    return total;
}

/* LSB-first bit writer: bit k of the stream is bit (k mod 8) of byte k/8. */
static void put_bits(uint8_t* dst, uint64_t bitpos, uint32_t v, unsigned width) {
    for (unsigned i = 0; i < width; ++i)
        if ((v >> i) & 1u) dst[(bitpos + i) >> 3] |= (uint8_t)(1u << ((bitpos + i) & 7));
}
static uint32_t get_bits(const uint8_t* src, uint64_t bitpos, unsigned width) {
    uint32_t v = 0;
    for (unsigned i = 0; i < width; ++i)
        if ((src[(bitpos + i) >> 3] >> ((bitpos + i) & 7)) & 1u) v |= 1u << i;
    return v;
}

/* Residual section:
 *   u32 N | u8 b[nb] | u8 n_exc[nb] | u8 B[nb] | pad to 4 |
 *   payload (16*b bytes per frame) | exception positions (1 byte each) |
 *   exception high parts (ceil(n*(B-b)/8) bytes per frame)            */
static void pfor_emit(obuf* ob, const uint32_t* z, uint32_t n) {
    size_t nb = (n + 127) / 128;
    unsigned* bb = (unsigned*)calloc(nb ? nb : 1, sizeof(unsigned));
    unsigned* nn = (unsigned*)calloc(nb ? nb : 1, sizeof(unsigned));
    unsigned* BB = (unsigned*)calloc(nb ? nb : 1, sizeof(unsigned));
    if (!bb || !nn || !BB) { ob->oom = 1; free(bb); free(nn); free(BB); return; }
    uint32_t f[128];
    for (size_t j = 0; j < nb; ++j) {
        load_frame(z, n, j, f);
        orc_pfor_choose(f, &bb[j], &nn[j], &BB[j]);
    }
    ob_u32(ob, n);
    for (size_t j = 0; j < nb; ++j) ob_u8(ob, (uint8_t)bb[j]);
    for (size_t j = 0; j < nb; ++j) ob_u8(ob, (uint8_t)nn[j]);
    for (size_t j = 0; j < nb; ++j) ob_u8(ob, (uint8_t)BB[j]);
    ob_pad4(ob);
    /* payload: the low b bits of every slot */
    for (size_t j = 0; j < nb; ++j) {
        uint8_t blk[512];
        memset(blk, 0, sizeof blk);
        load_frame(z, n, j, f);
        uint32_t lowm = bb[j] >= 32 ? 0xFFFFFFFFu : ((1u << bb[j]) - 1);
        for (unsigned i = 0; i < 128; ++i) put_bits(blk, (uint64_t)i * bb[j], f[i] & lowm, bb[j]);
        ob_put(ob, blk, 16u * bb[j]);
    }
    /* exception positions, ascending within each frame */
    for (size_t j = 0; j < nb; ++j) {
        load_frame(z, n, j, f);
        for (unsigned i = 0; i < 128; ++i)
            if (exceeds(f[i], bb[j])) ob_u8(ob, (uint8_t)i);
    }
    /* exception high parts at B-b bits, in position order */
    for (size_t j = 0; j < nb; ++j) {
        if (!nn[j]) continue;
        unsigned hw = BB[j] - bb[j];
        uint8_t hi[512];
        memset(hi, 0, sizeof hi);
        load_frame(z, n, j, f);
        unsigned e = 0;
        for (unsigned i = 0; i < 128; ++i)
            if (exceeds(f[i], bb[j])) put_bits(hi, (uint64_t)e++ * hw, f[i] >> bb[j], hw);
        ob_put(ob, hi, (nn[j] * hw + 7) / 8);
    }
    free(bb);
    free(nn);
    free(BB);
}

size_t orc_pfor_encode(const uint32_t* z, uint32_t n, uint8_t* out, size_t cap) {
    obuf ob = {0};
    pfor_emit(&ob, z, n);
    size_t len = ob.oom ? 0 : ob.n;
    if (out && len <= cap) memcpy(out, ob.p, len);
    free(ob.p);
    return len;
}

/* Parses one residual section; z receives n_expect values.  *used gets the
 * section's byte length before the final pad to 4. */
int orc_pfor_decode(const uint8_t* in, size_t len, unsigned bits, uint32_t n_expect, uint32_t* z,
                    size_t* used) {
    if (len < 4) return ORC_E_CORRUPT;
    uint32_t n = rd_u32(in);
    if (n != n_expect) return ORC_E_CORRUPT;
    size_t nb = (n + 127) / 128;
    size_t hdr = 4 + 3 * nb;
    size_t hdr4 = (hdr + 3) & ~(size_t)3;
    if (hdr4 > len) return ORC_E_CORRUPT;
    const uint8_t* bb = in + 4;
    const uint8_t* nn = bb + nb;
    const uint8_t* BB = nn + nb;
    size_t pay = 0, pos = 0, high = 0;
    for (size_t j = 0; j < nb; ++j) {
        unsigned b = bb[j], e = nn[j], B = BB[j];
        if (B > bits || b > B || e > 128) return ORC_E_CORRUPT;
        if (e && b == B) return ORC_E_CORRUPT;
        pay += 16u * b;
        pos += e;
        high += (e * (B - b) + 7) / 8;
    }
    size_t total = hdr4 + pay + pos + high;
    if (total > len) return ORC_E_CORRUPT;
    const uint8_t* p_pay = in + hdr4;
    const uint8_t* p_pos = p_pay + pay;
    const uint8_t* p_high = p_pos + pos;
    for (size_t j = 0; j < nb; ++j) {
        unsigned b = bb[j], e = nn[j], B = BB[j];
        size_t real = n - 128 * j < 128 ? n - 128 * j : 128;
        uint32_t f[128];
        for (unsigned i = 0; i < 128; ++i) f[i] = get_bits(p_pay, (uint64_t)i * b, b);
        int last = -1;
        for (unsigned k = 0; k < e; ++k) {
            int i = p_pos[k];
            if (i <= last || (size_t)i >= real) return ORC_E_CORRUPT;
            last = i;
            f[i] |= get_bits(p_high, (uint64_t)k * (B - b), B - b) << b;
        }
        for (size_t i = 0; i < real; ++i) z[128 * j + i] = f[i];
        p_pay += 16u * b;
        p_pos += e;
        p_high += (e * (B - b) + 7) / 8;
    }
    if (used) *used = total;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. III-C: the zero bitmask is packed into bytes and compressed with     */
/* Zstd.  The frame written here is a valid Zstandard frame (RFC 8878)      */
/* restricted to Raw and RLE blocks: runs of >= 8 equal bytes become RLE     */
/* blocks, the stretches between them Raw blocks, every block at most 128 KiB.*/
/* ------------------------------------------------------------------------ */
#define ZSTD_MAGIC 0xFD2FB528u
#define ZBLOCK_MAX 131072u
#define RLE_MIN_RUN 8u

typedef struct {
    int rle;
    size_t start, size;
} zblock;

static size_t frame_blocks(const uint8_t* in, size_t n, zblock* out) {
    size_t cnt = 0, raw_start = 0, i = 0;
#define EMIT(is_rle, st, sz)                                                  \
    do {                                                                      \
        size_t s_ = (st), left_ = (sz);                                       \
        while (left_) {                                                       \
            size_t piece_ = left_ > ZBLOCK_MAX ? ZBLOCK_MAX : left_;          \
            if (out) { out[cnt].rle = (is_rle); out[cnt].start = s_; out[cnt].size = piece_; } \
            cnt++;                                                            \
            s_ += piece_;                                                     \
            left_ -= piece_;                                                  \
        }                                                                     \
    } while (0)
    while (i < n) {
        size_t j = i;
        while (j < n && in[j] == in[i]) j++;
        if (j - i >= RLE_MIN_RUN) {
            EMIT(0, raw_start, i - raw_start);
            EMIT(1, i, j - i);
            raw_start = j;
        }
        i = j;
    }
    EMIT(0, raw_start, n - raw_start);
#undef EMIT
    return cnt;
}

size_t orc_frame(const uint8_t* in, size_t n, uint8_t* out, size_t cap) {
    obuf ob = {0};
    ob_u32(&ob, ZSTD_MAGIC);
    /* Frame_Header_Descriptor: single segment, no checksum, no dictionary;
     * the content size field takes the smallest of its 1/2/4-byte forms */
    if (n <= 255) {
        ob_u8(&ob, 0x20);
        ob_u8(&ob, (uint8_t)n);
    } else if (n <= 65791) {
        ob_u8(&ob, 0x60);
        ob_u16(&ob, (uint16_t)(n - 256));
    } else {
        ob_u8(&ob, 0xA0);
        ob_u32(&ob, (uint32_t)n);
    }
    size_t nblk = frame_blocks(in, n, NULL);
    zblock* blk = (zblock*)malloc((nblk ? nblk : 1) * sizeof(zblock));
    if (!blk) { free(ob.p); return 0; }
    frame_blocks(in, n, blk);
    if (nblk == 0) { /* empty content: one empty last Raw block */
        ob_u8(&ob, 1); ob_u8(&ob, 0); ob_u8(&ob, 0);
    }
    for (size_t k = 0; k < nblk; ++k) {
        uint32_t last = (k + 1 == nblk) ? 1u : 0u;
        uint32_t h = last | ((blk[k].rle ? 1u : 0u) << 1) | ((uint32_t)blk[k].size << 3);
        ob_u8(&ob, (uint8_t)h);
        ob_u8(&ob, (uint8_t)(h >> 8));
        ob_u8(&ob, (uint8_t)(h >> 16));
        if (blk[k].rle) ob_u8(&ob, in[blk[k].start]);
        else ob_put(&ob, in + blk[k].start, blk[k].size);
    }
    free(blk);
    size_t len = ob.oom ? 0 : ob.n;
    if (out && len <= cap) memcpy(out, ob.p, len);
    free(ob.p);
    return len;
}

/* Reads a frame of the accepted form (single segment, no dictionary, no
 * checksum, Raw/RLE blocks only) whose content is exactly n_expect bytes
 * and which ends exactly at len. */
int orc_unframe(const uint8_t* in, size_t len, uint8_t* out, size_t n_expect) {
    if (len < 5 || rd_u32(in) != ZSTD_MAGIC) return ORC_E_CORRUPT;
    uint8_t fhd = in[4];
    unsigned fcs_flag = fhd >> 6, single = (fhd >> 5) & 1, reserved = (fhd >> 3) & 1;
    unsigned checksum = (fhd >> 2) & 1, dict = fhd & 3;
    if (!single || reserved || checksum || dict) return ORC_E_CORRUPT;
    size_t p = 5;
    uint64_t fcs;
    size_t fcs_len = fcs_flag == 0 ? 1 : fcs_flag == 1 ? 2 : fcs_flag == 2 ? 4 : 8;
    if (p + fcs_len > len) return ORC_E_CORRUPT;
    if (fcs_len == 1) fcs = in[p];
    else if (fcs_len == 2) fcs = (uint64_t)rd_u16(in + p) + 256;
    else if (fcs_len == 4) fcs = rd_u32(in + p);
    else fcs = (uint64_t)rd_u32(in + p) | ((uint64_t)rd_u32(in + p + 4) << 32);
    p += fcs_len;
    if (fcs != n_expect) return ORC_E_CORRUPT;
    size_t got = 0;
    for (;;) {
        if (p + 3 > len) return ORC_E_CORRUPT;
        uint32_t h = (uint32_t)in[p] | ((uint32_t)in[p + 1] << 8) | ((uint32_t)in[p + 2] << 16);
        p += 3;
        unsigned last = h & 1, type = (h >> 1) & 3;
        size_t size = h >> 3;
        if (size > ZBLOCK_MAX || got + size > n_expect) return ORC_E_CORRUPT;
        if (type == 0) {
            if (p + size > len) return ORC_E_CORRUPT;
            memcpy(out + got, in + p, size);
            p += size;
        } else if (type == 1) {
            if (p + 1 > len) return ORC_E_CORRUPT;
            memset(out + got, in[p], size);
            p += 1;
        } else {
            return ORC_E_CORRUPT;
        }
        got += size;
        if (last) break;
    }
    if (got != n_expect || p != len) return ORC_E_CORRUPT;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. III-E / IV-E: trial compression on a few scanlines (4 by default),   */
/* spread evenly over the scan: the band centres floor((2j+1)H/(2K)).       */
/* ------------------------------------------------------------------------ */
unsigned orc_trial_rows(uint32_t height, uint32_t k, uint32_t* rows) {
    unsigned cnt = 0;
    for (uint32_t j = 0; j < k; ++j) {
        uint32_t r = (uint32_t)(((uint64_t)(2 * j + 1) * height) / (2ull * k));
        if (cnt == 0 || rows[cnt - 1] != r) rows[cnt++] = r; /* ascending: drop repeats */
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* whole codec                                                               */
/* ------------------------------------------------------------------------ */
static uint64_t read_sample(const void* plane, unsigned wb, size_t i) {
    if (wb == 1) return ((const uint8_t*)plane)[i];
    if (wb == 2) return ((const uint16_t*)plane)[i];
    return ((const uint32_t*)plane)[i];
}
static void write_sample(void* plane, unsigned wb, size_t i, uint64_t v) {
    if (wb == 1) ((uint8_t*)plane)[i] = (uint8_t)v;
    else if (wb == 2) ((uint16_t*)plane)[i] = (uint16_t)v;
    else ((uint32_t*)plane)[i] = (uint32_t)v;
}

static int layout_ok(const orc_layout* L) {
    if (!L || L->n_attrs < 1 || L->n_attrs > ORC_MAX_ATTRS) return 0;
    if (L->height == 0 || L->width == 0) return 0;
    for (unsigned a = 0; a < L->n_attrs; ++a) {
        unsigned wb = L->width_bytes[a];
        if (wb != 1 && wb != 2 && wb != 4) return 0;
        if (L->precision[a] == 0) return 0;
    }
    return 1;
}

static size_t frame_bound(size_t n) { return 16 + n + 4 * (n / ZBLOCK_MAX + 1); }

size_t orc_encode_bound(const orc_layout* L, uint32_t n_scans) {
    if (!layout_ok(L)) return 0;
    size_t npx = (size_t)L->height * L->width;
    size_t mbytes = (npx + 7) / 8, nb = (npx + 127) / 128;
    size_t total = 20 + 8 * (size_t)L->n_attrs + 4 * (size_t)n_scans * L->n_attrs;
    for (unsigned a = 0; a < L->n_attrs; ++a) {
        size_t bits = 8u * L->width_bytes[a];
        size_t rec = 12 + frame_bound(mbytes) + 3 + 4 + 3 * nb + 3 + nb * 16 * bits + 3;
        total += rec * n_scans;
    }
    return total;
}

/* Sec. III-E: P is chosen when the trial residuals against the previous scan
 * pack smaller than the intra-scan ones; the mask is not part of the trial. */
static int trial_choose_p(const uint64_t* Q, const uint64_t* Qp, const orc_layout* L, unsigned bits,
                          uint32_t k) {
    uint32_t H = L->height, W = L->width;
    uint32_t* rows = (uint32_t*)malloc(sizeof(uint32_t) * (k ? k : 1));
    unsigned nr = orc_trial_rows(H, k, rows);
    size_t cap = (size_t)nr * W;
    uint32_t* zi = (uint32_t*)malloc(sizeof(uint32_t) * (cap ? cap : 1));
    uint32_t* zp = (uint32_t*)malloc(sizeof(uint32_t) * (cap ? cap : 1));
    uint64_t m = low_mask(bits);
    size_t cnt = 0;
    uint64_t prev_i = 0, prev_p = 0;
    for (unsigned r = 0; r < nr; ++r) {
        for (uint32_t c = 0; c < W; ++c) {
            size_t i = (size_t)rows[r] * W + c;
            if (Q[i] == 0) continue;
            uint64_t u = Q[i];                 /* intra value */
            uint64_t v = (Q[i] - Qp[i]) & m;   /* temporal difference */
            zi[cnt] = orc_zigzag((uint32_t)((u - prev_i) & m), bits);
            zp[cnt] = orc_zigzag((uint32_t)((v - prev_p) & m), bits);
            prev_i = u;
            prev_p = v;
            cnt++;
        }
    }
    int choose_p = orc_pfor_cost(zp, cnt) < orc_pfor_cost(zi, cnt);
    free(rows);
    free(zi);
    free(zp);
    return choose_p;
}

static size_t mask_bytes(size_t npx) { return (npx + 7) / 8; }

/* One record: the scan of attribute a, coded as an I- or P-scan. */
static void encode_record(obuf* ob, unsigned a, const uint64_t* Q, const uint64_t* Qp,
                          const uint8_t* mb, const uint8_t* mb_prev, int pmode, size_t npx,
                          unsigned bits) {
    size_t rec_start = ob->n;
    size_t nm = mask_bytes(npx);
    uint64_t m = low_mask(bits);

    /* Sec. III-D: a P-scan stores its mask XORed with the previous mask */
    uint8_t* mc = (uint8_t*)malloc(nm ? nm : 1);
    for (size_t i = 0; i < nm; ++i) mc[i] = pmode ? (uint8_t)(mb[i] ^ mb_prev[i]) : mb[i];
    size_t flen = orc_frame(mc, nm, NULL, 0);
    uint8_t* fr = (uint8_t*)malloc(flen ? flen : 1);
    orc_frame(mc, nm, fr, flen);

    ob_u32(ob, 0); /* record length, patched below */
    ob_u8(ob, (uint8_t)(pmode ? 1 : 0));
    ob_u8(ob, (uint8_t)a);
    ob_u16(ob, 0);
    ob_u32(ob, (uint32_t)flen);
    ob_put(ob, fr, flen);
    ob_pad4(ob);

    /* Sec. III-C: remove the zeros, flattening the scan to one vector;
     * Sec. III-D: a P-scan takes the difference to the previous scan at the
     * current in-range positions; then the horizontal delta and ZigZag */
    uint32_t n = 0;
    for (size_t i = 0; i < npx; ++i) n += Q[i] != 0;
    uint32_t* z = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint64_t prev = 0;
    uint32_t k = 0;
    for (size_t i = 0; i < npx; ++i) {
        if (Q[i] == 0) continue;
        uint64_t s = pmode ? ((Q[i] - Qp[i]) & m) : Q[i];
        z[k++] = orc_zigzag((uint32_t)((s - prev) & m), bits);
        prev = s;
    }
    pfor_emit(ob, z, n);
    ob_pad4(ob);

    if (!ob->oom) {
        uint32_t len = (uint32_t)(ob->n - rec_start);
        ob->p[rec_start + 0] = (uint8_t)len;
        ob->p[rec_start + 1] = (uint8_t)(len >> 8);
        ob->p[rec_start + 2] = (uint8_t)(len >> 16);
        ob->p[rec_start + 3] = (uint8_t)(len >> 24);
    }
    free(z);
    free(fr);
    free(mc);
}

/* Sec. III-E, the brute-force alternative to the trial: the scan is coded
 * both ways, mask included, and the smaller record is kept (equal sizes:
 * the I-scan). */
static int brute_choose_p(unsigned a, const uint64_t* Q, const uint64_t* Qp, const uint8_t* mb,
                          const uint8_t* mb_prev, size_t npx, unsigned bits) {
    obuf bi = {0}, bp = {0};
    encode_record(&bi, a, Q, Qp, mb, mb_prev, 0, npx, bits);
    encode_record(&bp, a, Q, Qp, mb, mb_prev, 1, npx, bits);
    int choose_p = bp.n < bi.n;
    free(bi.p);
    free(bp.p);
    return choose_p;
}

int orc_encode(const orc_layout* L, const orc_options* opt, uint32_t T, const void* const* planes,
               const void* const* prev_planes, uint8_t* out, size_t cap, size_t* out_len,
               uint8_t* modes) {
    if (!layout_ok(L) || !planes || !out_len) return ORC_E_INVALID;
    uint32_t mode = opt ? opt->mode : 0;
    uint32_t k = (opt && opt->trial_rows) ? opt->trial_rows : 4;
    if (mode > 3) return ORC_E_INVALID;
    unsigned A = L->n_attrs;
    size_t npx = (size_t)L->height * L->width, nm = mask_bytes(npx);

    obuf ob = {0};
    /* stream header: magic, version, attribute count, shape, scan count */
    ob_put(&ob, "JFY1", 4);
    ob_u16(&ob, 1);
    ob_u16(&ob, (uint16_t)A);
    ob_u32(&ob, L->height);
    ob_u32(&ob, L->width);
    ob_u32(&ob, T);
    /* Sec. III-A: the precision is stored in the stream */
    for (unsigned a = 0; a < A; ++a) {
        ob_u8(&ob, L->width_bytes[a]);
        ob_u8(&ob, 0); ob_u8(&ob, 0); ob_u8(&ob, 0);
        ob_u32(&ob, L->precision[a]);
    }
    size_t table = ob.n; /* record length table, patched below */
    for (size_t r = 0; r < (size_t)T * A; ++r) ob_u32(&ob, 0);

    /* scans in time order; the attributes of one scan follow each other */
    uint64_t** Qs = (uint64_t**)calloc(A, sizeof(uint64_t*));
    uint64_t** Qps = (uint64_t**)calloc(A, sizeof(uint64_t*));
    uint8_t** mbs = (uint8_t**)calloc(A, sizeof(uint8_t*));
    uint8_t** mbps = (uint8_t**)calloc(A, sizeof(uint8_t*));
    int* have_prev = (int*)calloc(A, sizeof(int));
    for (unsigned a = 0; a < A; ++a) {
        Qs[a] = (uint64_t*)malloc(sizeof(uint64_t) * npx);
        Qps[a] = (uint64_t*)malloc(sizeof(uint64_t) * npx);
        mbs[a] = (uint8_t*)malloc(nm);
        mbps[a] = (uint8_t*)malloc(nm);
        if (prev_planes && prev_planes[a]) {
            unsigned wb = L->width_bytes[a];
            memset(mbps[a], 0, nm);
            for (size_t i = 0; i < npx; ++i) {
                Qps[a][i] = orc_quantize(read_sample(prev_planes[a], wb, i), L->precision[a]);
                if (Qps[a][i] == 0) mbps[a][i >> 3] |= (uint8_t)(1u << (i & 7));
            }
            have_prev[a] = 1;
        }
    }
    for (uint32_t t = 0; t < T; ++t) {
        for (unsigned a = 0; a < A; ++a) {
            unsigned wb = L->width_bytes[a], bits = 8 * wb;
            uint32_t P = L->precision[a];
            const void* plane = (const uint8_t*)planes[a] + (size_t)t * npx * wb;
            uint64_t* Q = Qs[a];
            uint8_t* mb = mbs[a];
            /* Sec. III-B quantize; Sec. III-C mask: 1 marks an out-of-range
             * (zero) sample, packed LSB-first over the flattened scan */
            memset(mb, 0, nm);
            for (size_t i = 0; i < npx; ++i) {
                Q[i] = orc_quantize(read_sample(plane, wb, i), P);
                if (Q[i] == 0) mb[i >> 3] |= (uint8_t)(1u << (i & 7));
            }
            /* Sec. III-E: the I/P choice */
            int pmode = 0;
            if (have_prev[a]) {
                if (mode == 1) pmode = 0;
                else if (mode == 2) pmode = 1;
                else if (mode == 3) pmode = brute_choose_p(a, Q, Qps[a], mb, mbps[a], npx, bits);
                else pmode = trial_choose_p(Q, Qps[a], L, bits, k);
            }
            if (modes) modes[(size_t)t * A + a] = (uint8_t)pmode;
            size_t before = ob.n;
            encode_record(&ob, a, Q, Qps[a], mb, mbps[a], pmode, npx, bits);
            if (!ob.oom) {
                uint32_t len = (uint32_t)(ob.n - before);
                size_t at = table + 4 * ((size_t)t * A + a);
                ob.p[at + 0] = (uint8_t)len;
                ob.p[at + 1] = (uint8_t)(len >> 8);
                ob.p[at + 2] = (uint8_t)(len >> 16);
                ob.p[at + 3] = (uint8_t)(len >> 24);
            }
            /* the current scan becomes the previous one */
            uint64_t* tq = Qps[a]; Qps[a] = Qs[a]; Qs[a] = tq;
            uint8_t* tm = mbps[a]; mbps[a] = mbs[a]; mbs[a] = tm;
            have_prev[a] = 1;
        }
    }
    for (unsigned a = 0; a < A; ++a) { free(Qs[a]); free(Qps[a]); free(mbs[a]); free(mbps[a]); }
    free(Qs); free(Qps); free(mbs); free(mbps); free(have_prev);

    if (ob.oom) { free(ob.p); return ORC_E_INVALID; }
    *out_len = ob.n;
    int rc = ORC_OK;
    if (ob.n > cap || !out) rc = ORC_E_CAPACITY;
    else memcpy(out, ob.p, ob.n);
    free(ob.p);
    return rc;
}

/* Header parse.  T = 0 in the header means "records until the end of the
 * buffer" (no length table); then the scan count is found by walking the
 * records' own length fields. */
static int parse_header(const uint8_t* in, size_t len, orc_layout* L, uint32_t* T_hdr, size_t* hdr_len) {
    if (!in || len < 20 || memcmp(in, "JFY1", 4) != 0) return ORC_E_CORRUPT;
    if (rd_u16(in + 4) != 1) return ORC_E_CORRUPT;
    unsigned A = rd_u16(in + 6);
    if (A < 1 || A > ORC_MAX_ATTRS) return ORC_E_CORRUPT;
    memset(L, 0, sizeof *L);
    L->n_attrs = A;
    L->height = rd_u32(in + 8);
    L->width = rd_u32(in + 12);
    *T_hdr = rd_u32(in + 16);
    size_t p = 20;
    if (len < p + 8 * (size_t)A) return ORC_E_CORRUPT;
    for (unsigned a = 0; a < A; ++a) {
        L->width_bytes[a] = in[p];
        if (in[p + 1] || in[p + 2] || in[p + 3]) return ORC_E_CORRUPT;
        L->precision[a] = rd_u32(in + p + 4);
        p += 8;
    }
    if (!layout_ok(L)) return ORC_E_CORRUPT;
    *hdr_len = p;
    return ORC_OK;
}

int orc_peek(const uint8_t* in, size_t len, orc_layout* L, uint32_t* n_scans) {
    uint32_t T;
    size_t p;
    int rc = parse_header(in, len, L, &T, &p);
    if (rc) return rc;
    if (T) {
        size_t nrec = (size_t)T * L->n_attrs;
        if (len < p + 4 * nrec) return ORC_E_CORRUPT;
        size_t total = p + 4 * nrec;
        for (size_t r = 0; r < nrec; ++r) total += rd_u32(in + p + 4 * r);
        if (total != len) return ORC_E_CORRUPT;
    } else {
        size_t q = p, nrec = 0;
        while (q < len) {
            if (q + 4 > len) return ORC_E_CORRUPT;
            uint32_t rl = rd_u32(in + q);
            if (rl < 12 || rl % 4 || rl > len - q) return ORC_E_CORRUPT;
            q += rl;
            nrec++;
        }
        if (nrec % L->n_attrs) return ORC_E_CORRUPT;
        T = (uint32_t)(nrec / L->n_attrs);
    }
    if (n_scans) *n_scans = T;
    return ORC_OK;
}

int orc_decode(const uint8_t* in, size_t len, void* const* planes_out) {
    orc_layout L;
    uint32_t T_hdr, T;
    size_t p;
    int rc = parse_header(in, len, &L, &T_hdr, &p);
    if (rc) return rc;
    rc = orc_peek(in, len, &L, &T);
    if (rc) return rc;
    const size_t hdr_end = p;
    if (T_hdr) p += 4 * (size_t)T_hdr * L.n_attrs; /* the length table, checked record by record below */
    unsigned A = L.n_attrs;
    size_t npx = (size_t)L.height * L.width, nm = mask_bytes(npx);
    uint64_t** Qp = (uint64_t**)calloc(A, sizeof(uint64_t*));
    uint8_t** mbp = (uint8_t**)calloc(A, sizeof(uint8_t*));
    uint8_t* mb = (uint8_t*)malloc(nm);
    uint32_t* z = (uint32_t*)malloc(sizeof(uint32_t) * npx);
    for (unsigned a = 0; a < A; ++a) {
        Qp[a] = (uint64_t*)calloc(npx, sizeof(uint64_t));
        mbp[a] = (uint8_t*)calloc(nm, 1);
    }
    rc = ORC_OK;
    for (uint32_t t = 0; t < T && rc == ORC_OK; ++t) {
        for (unsigned a = 0; a < A && rc == ORC_OK; ++a) {
            unsigned wb = L.width_bytes[a], bits = 8 * wb;
            uint64_t m = low_mask(bits);
            const uint8_t* r = in + p;
            size_t avail = len - p;
            if (avail < 12) { rc = ORC_E_CORRUPT; break; }
            uint32_t rl = rd_u32(r);
            if (rl < 12 || rl % 4 || rl > avail) { rc = ORC_E_CORRUPT; break; }
            /* the length table repeats every record's own length */
            if (T_hdr && rd_u32(in + hdr_end + 4 * ((size_t)t * A + a)) != rl) { rc = ORC_E_CORRUPT; break; }
            unsigned pmode = r[4], attr = r[5];
            if (pmode > 1 || attr != a || rd_u16(r + 6) != 0) { rc = ORC_E_CORRUPT; break; }
            if (pmode && t == 0) { rc = ORC_E_CORRUPT; break; } /* nothing to predict from */
            uint32_t flen = rd_u32(r + 8);
            if (flen > rl - 12) { rc = ORC_E_CORRUPT; break; }
            if (orc_unframe(r + 12, flen, mb, nm) != ORC_OK) { rc = ORC_E_CORRUPT; break; }
            if (pmode) for (size_t i = 0; i < nm; ++i) mb[i] ^= mbp[a][i];
            if (npx % 8 && (mb[nm - 1] >> (npx % 8))) { rc = ORC_E_CORRUPT; break; }
            uint32_t n = 0;
            for (size_t i = 0; i < npx; ++i) n += !((mb[i >> 3] >> (i & 7)) & 1u);
            size_t sec = (12 + (size_t)flen + 3) & ~(size_t)3;
            if (sec > rl) { rc = ORC_E_CORRUPT; break; }
            size_t used = 0;
            if (orc_pfor_decode(r + sec, rl - sec, bits, n, z, &used) != ORC_OK) { rc = ORC_E_CORRUPT; break; }
            if (sec + ((used + 3) & ~(size_t)3) != rl) { rc = ORC_E_CORRUPT; break; }
            /* reverse: ZigZag, delta (running sum), temporal difference,
             * zero removal (scatter), quantization */
            uint64_t s = 0;
            uint32_t k = 0;
            void* plane = (uint8_t*)planes_out[a] + (size_t)t * npx * wb;
            for (size_t i = 0; i < npx; ++i) {
                uint64_t q = 0;
                if (!((mb[i >> 3] >> (i & 7)) & 1u)) {
                    s = (s + orc_unzigzag(z[k++], bits)) & m;
                    q = pmode ? ((s + Qp[a][i]) & m) : s;
                }
                Qp[a][i] = q;
                write_sample(plane, wb, i, orc_dequantize(q, L.precision[a], bits));
            }
            memcpy(mbp[a], mb, nm);
            p += rl;
        }
    }
    for (unsigned a = 0; a < A; ++a) { free(Qp[a]); free(mbp[a]); }
    free(Qp); free(mbp); free(mb); free(z);
    return rc;
}
