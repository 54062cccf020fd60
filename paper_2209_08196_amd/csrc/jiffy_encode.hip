// Jiffy encoder kernels for gfx950.
//
// One call encodes every (scan, attribute) record of a batch at once: the
// records of a scan sequence are independent once the previous scan is an
// input, so each kernel runs over all records together.
//
//   k_enc_trial    I/P choice by trial compression of a few scanlines (Sec. III-E)
//   k_enc_tiles    quantize (Sec. III-B), zero bitmask (Sec. III-C), running
//                  count of in-range samples (decoupled look-back over the
//                  record's tiles), zero removal, temporal difference
//                  (Sec. III-D), delta, ZigZag (Eq. 1), frame width choice and
//                  bit packing (Sec. II)
//   (k_enc_mframe's last workgroups: the same for frames that cross tile boundaries)
//   k_enc_mframe   mask (XOR previous for a P-scan, Sec. III-D) as a Raw/RLE
//                  Zstandard frame (Sec. III-C)
//   k_enc_sizes    per-record section layout (prefix sums of frame sizes)
//   k_enc_offsets  record offsets in the output (prefix sum over records)
//   k_enc_assemble copies everything to its place in the stream
#define JIFFY_KERNEL_TU 1
#include "jiffy_device.h"

namespace jiffy {

// The record of global tile t and the tile's index inside it: by division
// when every record has `per` tiles, else from the maps.
__device__ __forceinline__ uint32_t tile_owner(const JG uint32_t* item_of, const JG uint32_t* first_of, uint32_t per,
                                               uint32_t t, uint32_t& lt) {
    if (per) {
        const uint32_t r = t / per;
        lt = t - r * per;
        return r;
    }
    const uint32_t r = item_of[t];
    lt = t - first_of[r];
    return r;
}

// ---------------------------------------------------------------------------
// Frame coding, four lanes per frame (Sec. II).  Lane q of the quad owns
// values 32q .. 32q+31 of the frame, so its low-b-bit parts fill exactly
// b words of the packed frame (words qb .. qb+b-1) and no lane waits for
// another.  Delta (to the preceding value) and ZigZag (Eq. 1) run in
// registers; the bit widths are counted in LDS; each lane then evaluates
// cost(b) for eight of the 32 widths and the quad takes the minimum.  The
// frame is built in an LDS row and copied to its slot with 16-byte stores.
// ---------------------------------------------------------------------------

// The quad's frame: z holds lane q's 32 values (in) and their ZigZag codes
// (out); real = number of real values (the rest count as 0); pred = the
// value before the first.  The width histogram goes to `hist` (36 LDS words,
// cleared here; words 0..31 count widths 1..32, word 32 + q width 0), and
// with kStash the codes also go back to vrow.  Returns the width key
// cost << 14 | (63 - b) << 8 | n(b) of the cheapest b (ties: larger b) and
// the frame's maximum width in B.  All four lanes call it together.
// kXf selects what is coded: 2 the ZigZag code of the difference to the
// preceding value (the codec), 1 that difference modulo 2^bits, 0 the values
// themselves (pred unused); 0 and 1 serve the ablated codecs only.
template <bool kStash, int kXf = 2>
__device__ __forceinline__ uint32_t quad_frame_key(uint32_t z[32], uint32_t* vrow, uint32_t* hist, uint32_t real,
                                                   uint32_t pred, uint32_t bits, uint32_t q, uint32_t& Bout) {
    uint4* h4 = (uint4*)hist;
    h4[2 * q] = make_uint4(0u, 0u, 0u, 0u);
    h4[2 * q + 1] = make_uint4(0u, 0u, 0u, 0u);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    uint32_t prev = dpp_mov<0x111>(z[31]);  // the previous lane's last value
    if (q == 0) prev = pred;
    const uint32_t i0 = 32u * q, zslot = 32u + q;
    uint32_t orv = 0;  // the widest code is the width of their OR
    // a code of width w >= 1 counts in word w - 1 = 31 - clz, a zero in the lane's own word
    auto code = [&](int i, bool real_i) {
        const uint32_t x = z[i];
        uint32_t r = 0u;  // zigzag keeps the low `bits` bits only
        if (real_i) r = kXf == 2 ? zigzag(x - prev, bits) : kXf == 1 ? (x - prev) & low_mask32(bits) : x;
        prev = x;
        z[i] = r;
        orv |= r;
        __hip_atomic_fetch_add(hist + (r ? 31u - (uint32_t)__builtin_clz(r) : zslot), 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WAVEFRONT);
    };
    if (i0 + 32u <= real) {  // every value of the lane is real (all but a record's last frame)
#pragma unroll
        for (int i = 0; i < 32; ++i) code(i, true);
    } else {
#pragma unroll
        for (int i = 0; i < 32; ++i) code(i, i0 + i < real);
    }
    uint32_t B = orv ? 32u - (uint32_t)__builtin_clz(orv) : 0u;
    B = max(B, dpp_mov<kQuadXor1>(B));
    B = max(B, dpp_mov<kQuadXor2>(B));
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // n(b) = values wider than b bits; lane q evaluates b = 8q .. 8q+7
    const uint4 ha = h4[2 * q], hb = h4[2 * q + 1];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if (kStash) {  // the codes replace the values (and the histogram, when it lives there)
        uint4* v4 = (uint4*)(vrow + 36 * q);
#pragma unroll
        for (int c = 0; c < 8; ++c) v4[c] = make_uint4(z[4 * c], z[4 * c + 1], z[4 * c + 2], z[4 * c + 3]);
    }
    const uint32_t h[8] = {ha.x, ha.y, ha.z, ha.w, hb.x, hb.y, hb.z, hb.w};  // widths 8q+1 .. 8q+8
    uint32_t loc = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) loc += h[k];
    const uint32_t c1 = quad_bcast<1>(loc), c2 = quad_bcast<2>(loc), c3 = quad_bcast<3>(loc);
    uint32_t n = (q < 1 ? c1 : 0u) + (q < 2 ? c2 : 0u) + (q < 3 ? c3 : 0u);
    // b = B costs 16 B with no exceptions
    uint32_t key = ((16u * B) << 14) | ((63u - B) << 8);
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        n += h[k];
        const uint32_t b = 8u * q + k;
        if (b < B) {
            const uint32_t cost = 16u * b + n + (n * (B - b) + 7u) / 8u;
            key = min(key, (cost << 14) | ((63u - b) << 8) | n);
        }
    }
    key = min(key, dpp_mov<kQuadXor1>(key));
    key = min(key, dpp_mov<kQuadXor2>(key));
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    Bout = B;
    return key;
}

__device__ __forceinline__ void load_quad_values(const uint32_t* vrow, uint32_t q, uint32_t z[32]) {
    const uint4* v4 = (const uint4*)(vrow + 36 * q);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint4 t = v4[c];
        z[4 * c] = t.x; z[4 * c + 1] = t.y; z[4 * c + 2] = t.z; z[4 * c + 3] = t.w;
    }
}

// packed size of the quad's frame (vrow: its values in row layout, which
// the histogram then overwrites)
__device__ __forceinline__ uint32_t frame_cost_quad(uint32_t* vrow, uint32_t real, uint32_t pred, uint32_t bits,
                                                    uint32_t q) {
    uint32_t z[32], B;
    load_quad_values(vrow, q, z);
    return quad_frame_key<false>(z, vrow, vrow, real, pred, bits, q, B) >> 14;
}

// Position of the k-th (from 0) set bit of a (k < popcount(a)).
__device__ __forceinline__ uint32_t select64(uint64_t a, uint32_t k) {
    uint32_t p = 0;
#pragma unroll
    for (uint32_t w = 32; w >= 1; w >>= 1) {
        const uint32_t c = __popcll(a & ((1ull << w) - 1ull));
        if (k >= c) {
            k -= c;
            a >>= w;
            p += w;
        }
    }
    return p;
}

// Bit offset, inside a frame's exception bytes, of item j: the n positions
// (8 bits each) come first, then the n high parts (hw bits each).
__device__ __forceinline__ uint32_t exc_bit(uint32_t j, uint32_t n, uint32_t hw) {
    return j < n ? 8u * j : 8u * n + (j - n) * hw;
}

// The low B bits of a lane's 32 codes as its B words of the packed frame
// (value i at bits [iB, (i+1)B)), built with shifts known at compile time
// and stored unconditionally.
template <int B>
__device__ __forceinline__ void pack32(const uint32_t z[32], JG uint32_t* dst) {
    constexpr uint32_t kMask = B == 32 ? 0xFFFFFFFFu : ((1u << B) - 1u);
    uint32_t w[B];
#pragma unroll
    for (int k = 0; k < B; ++k) w[k] = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const int bit = i * B, lo = bit >> 5, sh = bit & 31;
        const uint32_t v = z[i] & kMask;
        w[lo] |= v << sh;
        if (sh + B > 32) w[lo + 1] |= v >> (32 - sh);
    }
#pragma unroll
    for (int k = 0; k < B; ++k) dst[k] = w[k];
}
#define JIFFY_PACK_CASE(B) \
    case B: pack32<B>(z, dst); break;
__device__ __forceinline__ void pack_lane(const uint32_t z[32], uint32_t b, JG uint32_t* dst) {
    switch (b) {
        JIFFY_PACK_CASE(1) JIFFY_PACK_CASE(2) JIFFY_PACK_CASE(3) JIFFY_PACK_CASE(4)
        JIFFY_PACK_CASE(5) JIFFY_PACK_CASE(6) JIFFY_PACK_CASE(7) JIFFY_PACK_CASE(8)
        JIFFY_PACK_CASE(9) JIFFY_PACK_CASE(10) JIFFY_PACK_CASE(11) JIFFY_PACK_CASE(12)
        JIFFY_PACK_CASE(13) JIFFY_PACK_CASE(14) JIFFY_PACK_CASE(15) JIFFY_PACK_CASE(16)
        JIFFY_PACK_CASE(17) JIFFY_PACK_CASE(18) JIFFY_PACK_CASE(19) JIFFY_PACK_CASE(20)
        JIFFY_PACK_CASE(21) JIFFY_PACK_CASE(22) JIFFY_PACK_CASE(23) JIFFY_PACK_CASE(24)
        JIFFY_PACK_CASE(25) JIFFY_PACK_CASE(26) JIFFY_PACK_CASE(27) JIFFY_PACK_CASE(28)
        JIFFY_PACK_CASE(29) JIFFY_PACK_CASE(30) JIFFY_PACK_CASE(31) JIFFY_PACK_CASE(32)
        default: break;  // b = 0: no payload
    }
}
#undef JIFFY_PACK_CASE

// vrow: the frame's values (row layout); the width histogram, then the
// codes replace them.  The packed frame goes straight to its slot: lane q
// stores its b words of low bits (words qb .. qb+b-1).  The exception bytes
// from byte 16b -- the positions, then the high parts, one little-endian
// bit stream of 8n + n(B - b) bits -- are split between the lanes by whole
// words: lane q writes the words from the one that holds item q*2n/4 up to
// the one that holds item (q+1)*2n/4 (exclusive), so no word has two
// writers; each lane walks the exceptions from its first item on, reading
// their codes back from vrow four at a time.  b | n << 8 | B << 16 goes to
// *info.
__device__ __forceinline__ void code_frame_quad(uint32_t* vrow, uint32_t real, uint32_t pred, uint32_t bits,
                                                uint32_t q, JG uint8_t* slot, JG uint32_t* info) {
    uint32_t z[32], B;
    load_quad_values(vrow, q, z);
    const uint32_t key = quad_frame_key<true>(z, vrow, vrow, real, pred, bits, q, B);
    const uint32_t b = 63u - ((key >> 8) & 63u), nexc = key & 255u;
    const uint32_t hw = B - b, lm = low_mask32(b);
    JG uint32_t* sw = (JG uint32_t*)slot;
    pack_lane(z, b, sw + q * b);  // low b bits of each value
    uint32_t ex = 0;  // this lane's exceptions
#pragma unroll
    for (int i = 0; i < 32; ++i) ex |= (z[i] > lm ? 1u : 0u) << i;
    const uint64_t elo = (uint64_t)quad_bcast<0>(ex) | ((uint64_t)quad_bcast<1>(ex) << 32);
    const uint64_t ehi = (uint64_t)quad_bcast<2>(ex) | ((uint64_t)quad_bcast<3>(ex) << 32);
    if (q == 0) *info = b | (nexc << 8) | (B << 16);
    if (nexc == 0) return;
    const uint32_t n2 = 2u * nexc, T = exc_bit(n2, nexc, hw);
    const uint32_t w0 = exc_bit((q * n2) >> 2, nexc, hw) >> 5;
    const uint32_t w1 = q == 3 ? (T + 31u) >> 5 : exc_bit(((q + 1u) * n2) >> 2, nexc, hw) >> 5;
    if (w0 >= w1) return;
    const uint32_t bb = 32u * w0, be = min(32u * w1, T);
    // the item holding bit bb, and the exception it belongs to
    uint32_t j = bb < 8u * nexc ? bb / 8u : nexc + (bb - 8u * nexc) / hw;
    uint64_t ca, cb;  // exceptions from the cursor on: the current half, then the high half (if not in it)
    uint32_t cbase;
    {
        const uint32_t k = j < nexc ? j : j - nexc, c0 = __popcll(elo);
        if (k < c0) {
            ca = elo & (~0ull << select64(elo, k));
            cb = ehi;
            cbase = 0;
        } else {
            ca = ehi & (~0ull << select64(ehi, k - c0));
            cb = 0;
            cbase = 64;
        }
    }
    JG uint32_t* sec = sw + 4u * b;
    uint64_t acc = 0;
    uint32_t nacc = 0, wi = w0, s = exc_bit(j, nexc, hw);
    while (s < be) {
        uint32_t pos[4], code[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (j + t == nexc) {  // the positions are done: the high parts start again from exception 0
                ca = elo;
                cb = ehi;
                cbase = 0;
            }
            if (!ca) {
                ca = cb;
                cb = 0;
                cbase = 64;
            }
            pos[t] = ca ? cbase + (uint32_t)__builtin_ctzll(ca) : 0u;
            ca &= ca - 1ull;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) code[t] = vrow[row_off(pos[t])];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (s < be) {
                const bool is_pos = j < nexc;
                uint32_t v = is_pos ? pos[t] : code[t] >> b;
                uint32_t wd = is_pos ? 8u : hw;
                const uint32_t s_next = s + wd;
                if (s < bb) {  // the item began in the previous lane's last word
                    v >>= bb - s;
                    wd -= bb - s;
                }
                acc |= (uint64_t)v << nacc;
                nacc += wd;
                if (nacc >= 32) {
                    if (wi < w1) sec[wi] = (uint32_t)acc;
                    ++wi;
                    acc >>= 32;
                    nacc -= 32;
                }
                ++j;
                s = s_next;
            }
        }
    }
    if (nacc && wi < w1) sec[wi] = (uint32_t)acc;
}

// ---------------------------------------------------------------------------
// Trial compression (Sec. III-E): the nonzero samples of the band-centre
// rows floor((2j+1)H/(2K)) (all rows when K >= H), row by row, coded as
// the I residuals (the samples) and as the P residuals (differences to the
// previous scan); P iff its packed size is strictly smaller.  The mask is
// not part of the trial.  One workgroup per record: chunks of 8192 trial
// pixels are compacted into LDS frame rows (a frame left incomplete carries
// to the next chunk) and each whole frame is costed by a quad, the I
// residuals first, then the P residuals in the same rows.
// ---------------------------------------------------------------------------
struct TrialLds {
    uint32_t rows[kTileFrames * kRow];
    uint32_t carry[2][kFrame];  // the incomplete frame of each residual kind
    uint32_t scratch[8];
    unsigned long long cost[2];
};

// Half h (16 pixels) of a thread's 32 trial pixels from trial pixel tp0 on:
// v gets the I residuals (the quantized samples) or, with pkind, the P
// residuals (differences to the previous scan); returns their keep bits.
// Holding one kind of 16 values at a time keeps the registers low (each
// kind re-reads the few trial rows, which the cache still holds).
template <int WB>
__device__ __forceinline__ uint32_t trial_half(const EncItem& it, uint32_t tp0, uint32_t NT, bool whole, uint32_t h,
                                               bool pkind, uint32_t v[16]) {
    const uint32_t H = it.height, W = it.width, K = it.trial_rows, m = low_mask32(it.bits);
    const uint32_t t0 = tp0 + 16 * h;
    uint32_t keep = 0;
    if (whole) {  // the thread's pixels lie in one row, 16-sample aligned: vector loads
        uint32_t xs[16], xp[16];
        if (t0 < NT) {
            const uint32_t ri = t0 / W, c = t0 - ri * W;
            const uint32_t row = K >= H ? ri : (uint32_t)(((uint64_t)(2 * ri + 1) * H) / (2ull * K));
            const uint32_t p = row * W + c;
            load16<WB>(it.x, p, it.npx, true, xs);
            if (pkind) load16<WB>(it.xprev, p, it.npx, true, xp);
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) xs[i] = xp[i] = 0;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t qv = quantize(xs[i], it.div);
            keep |= (qv != 0 ? 1u : 0u) << i;
            if (pkind) {
                const uint32_t qp = it.prev_quantized ? xp[i] : quantize(xp[i], it.div);
                v[i] = (qv - qp) & m;
            } else {
                v[i] = qv;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t tp = t0 + i;
            uint32_t u = 0;
            if (tp < NT) {
                const uint32_t ri = tp / W, c = tp - ri * W;
                const uint32_t row = K >= H ? ri : (uint32_t)(((uint64_t)(2 * ri + 1) * H) / (2ull * K));
                const uint32_t p = row * W + c;
                const uint32_t qv = quantize(load1<WB>(it.x, p), it.div);
                keep |= (qv != 0 ? 1u : 0u) << i;
                u = qv;
                if (pkind) {
                    uint32_t qp = load1<WB>(it.xprev, p);
                    if (!it.prev_quantized) qp = quantize(qp, it.div);
                    u = (qv - qp) & m;
                }
            }
            v[i] = u;
        }
    }
    return keep;
}

// The same decision with one residual kind of 16 values in registers at a
// time (each kind re-reads the trial rows): far fewer registers, for the
// fused launch, whose register count is that of its largest phase.
template <int WB>
__device__ __forceinline__ void enc_trial_body_lowreg(const EncItem& it, TrialLds& L, JG EncRes* res) {
    const uint32_t tid = threadIdx.x, g = tid >> 2, q = tid & 3u;
    const uint32_t H = it.height, W = it.width, K = it.trial_rows;
    const uint32_t nr = K >= H ? H : K;  // distinct trial rows
    const uint32_t NT = nr * W;          // trial pixels
    if (tid < 2) L.cost[tid] = 0;
    // rows of a multiple of 32 samples: a thread's 32 trial pixels lie in one row
    const bool whole = it.aligned16 && W % 32 == 0;
    uint32_t carry = 0, pred[2] = {0u, 0u};  // values in the incomplete frame; value before it
    for (uint32_t cs = 0; cs < NT; cs += kFTile) {
        const uint32_t tp0 = cs + tid * 32;
        uint32_t v[16];
        const uint32_t keep = trial_half<WB>(it, tp0, NT, whole, 0, false, v) |
                              (trial_half<WB>(it, tp0, NT, whole, 1, false, v) << 16);
        uint32_t nv;
        const uint32_t off = block_excl_scan<256>(__popc(keep), L.scratch, &nv);
        const uint32_t total = carry + nv, nfull = total >> 7, rem = total & 127u;
        const bool last = cs + kFTile >= NT;
        const uint32_t ncost = nfull + (last && rem ? 1u : 0u);  // frames costed now
        for (int kind = 0; kind < 2; ++kind) {
            // the carried frame start, then this chunk's kept values
            if (tid < carry) L.rows[row_off(tid)] = L.carry[kind][tid];
            uint32_t k = carry + off;
            for (uint32_t h = 0; h < 2; ++h) {
                trial_half<WB>(it, tp0, NT, whole, h, kind == 1, v);
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (keep & (1u << (16 * h + i))) {
                        L.rows[tile_word(k, 0)] = v[i];
                        ++k;
                    }
            }
            __syncthreads();
            // predecessors, and the new incomplete frame, before any row turns into a histogram
            // (quad g costs frames g and g + 64: a chunk can hold 65)
            uint32_t pv[2];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const uint32_t f = g + 64 * hh;
                pv[hh] = (f < ncost && f > 0) ? L.rows[tile_word(128 * f - 1, 0)] : pred[kind];
            }
            const uint32_t npred = nfull ? L.rows[tile_word(128 * nfull - 1, 0)] : pred[kind];
            if (!last && tid < rem) L.carry[kind][tid] = L.rows[tile_word(128 * nfull + tid, 0)];
            __syncthreads();
            for (int hh = 0; hh < 2; ++hh) {  // one frame's 32 values per lane in registers at a time
                const uint32_t f = g + 64 * hh;
                if (f < ncost) {
                    const uint32_t real = f < nfull ? kFrame : rem;
                    const uint32_t c = frame_cost_quad(L.rows + f * kRow, real, hh ? pv[1] : pv[0], it.bits, q);
                    if (q == 0) atomicAdd(&L.cost[kind], (unsigned long long)c);
                }
            }
            pred[kind] = npred;
            __syncthreads();
        }
        carry = rem;
    }
    if (tid == 0) res->mode = L.cost[1] < L.cost[0] ? 1u : 0u;
}

template <int WB>
__device__ __forceinline__ void enc_trial_body(const EncItem& it, TrialLds& L, JG EncRes* res) {
    const uint32_t tid = threadIdx.x, g = tid >> 2, q = tid & 3u;
    const uint32_t m = low_mask32(it.bits);
    const uint32_t H = it.height, W = it.width, K = it.trial_rows;
    const uint32_t nr = K >= H ? H : K;  // distinct trial rows
    const uint32_t NT = nr * W;          // trial pixels
    if (tid < 2) L.cost[tid] = 0;
    // rows of a multiple of 32 samples: a thread's 32 trial pixels lie in one row
    const bool whole = it.aligned16 && W % 32 == 0;
    uint32_t carry = 0, pred[2] = {0u, 0u};  // values in the incomplete frame; value before it
    for (uint32_t cs = 0; cs < NT; cs += kFTile) {
        // this thread's 32 trial pixels
        uint32_t val[2][32];
        uint32_t keep = 0;
        const uint32_t tp0 = cs + tid * 32;
        if (whole) {  // one row, 16-sample aligned: vector loads
            uint32_t xs[32], xp[32];
            if (tp0 < NT) {
                const uint32_t ri = tp0 / W, c = tp0 - ri * W;
                const uint32_t row = K >= H ? ri : (uint32_t)(((uint64_t)(2 * ri + 1) * H) / (2ull * K));
                const uint32_t p = row * W + c;
                load16<WB>(it.x, p, it.npx, true, xs);
                load16<WB>(it.x, p + 16, it.npx, true, xs + 16);
                load16<WB>(it.xprev, p, it.npx, true, xp);
                load16<WB>(it.xprev, p + 16, it.npx, true, xp + 16);
            } else {
#pragma unroll
                for (int i = 0; i < 32; ++i) xs[i] = xp[i] = 0;
            }
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const uint32_t qv = quantize(xs[i], it.div);
                const uint32_t qp = it.prev_quantized ? xp[i] : quantize(xp[i], it.div);
                keep |= (qv != 0 ? 1u : 0u) << i;
                val[0][i] = qv;
                val[1][i] = (qv - qp) & m;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const uint32_t tp = tp0 + i;
                uint32_t u = 0, v = 0;
                if (tp < NT) {
                    const uint32_t ri = tp / W, c = tp - ri * W;
                    const uint32_t row = K >= H ? ri : (uint32_t)(((uint64_t)(2 * ri + 1) * H) / (2ull * K));
                    const uint32_t p = row * W + c;
                    const uint32_t qv = quantize(load1<WB>(it.x, p), it.div);
                    uint32_t qp = load1<WB>(it.xprev, p);
                    if (!it.prev_quantized) qp = quantize(qp, it.div);
                    keep |= (qv != 0 ? 1u : 0u) << i;
                    u = qv;
                    v = (qv - qp) & m;
                }
                val[0][i] = u;
                val[1][i] = v;
            }
        }
        uint32_t nv;
        const uint32_t off = block_excl_scan<256>(__popc(keep), L.scratch, &nv);
        const uint32_t total = carry + nv, nfull = total >> 7, rem = total & 127u;
        const bool last = cs + kFTile >= NT;
        const uint32_t ncost = nfull + (last && rem ? 1u : 0u);  // frames costed now
#pragma unroll
        for (int kind = 0; kind < 2; ++kind) {
            // the carried frame start, then this chunk's kept values
            if (tid < carry) L.rows[row_off(tid)] = L.carry[kind][tid];
            uint32_t k = carry + off;
#pragma unroll
            for (int i = 0; i < 32; ++i)
                if (keep & (1u << i)) {
                    L.rows[tile_word(k, 0)] = val[kind][i];
                    ++k;
                }
            __syncthreads();
            // predecessors, and the new incomplete frame, before any row turns into a histogram
            // (quad g costs frames g and g + 64: a chunk can hold 65)
            uint32_t pv[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t f = g + 64 * h;
                pv[h] = (f < ncost && f > 0) ? L.rows[tile_word(128 * f - 1, 0)] : pred[kind];
            }
            const uint32_t npred = nfull ? L.rows[tile_word(128 * nfull - 1, 0)] : pred[kind];
            if (!last && tid < rem) L.carry[kind][tid] = L.rows[tile_word(128 * nfull + tid, 0)];
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t f = g + 64 * h;
                if (f < ncost) {
                    const uint32_t real = f < nfull ? kFrame : rem;
                    const uint32_t c = frame_cost_quad(L.rows + f * kRow, real, pv[h], it.bits, q);
                    if (q == 0) atomicAdd(&L.cost[kind], (unsigned long long)c);
                }
            }
            pred[kind] = npred;
            __syncthreads();
        }
        carry = rem;
    }
    if (tid == 0) res->mode = L.cost[1] < L.cost[0] ? 1u : 0u;
}

// Record r's I/P decision; also clears its tile tickets and look-back states.
template <bool kLowReg = false>
__device__ __forceinline__ void enc_trial_item(const EncPlan& plan, uint32_t r, TrialLds& lds) {
    const EncItem it = plan.items[r];
    for (uint32_t i = threadIdx.x; i < it.ntiles; i += 256) it.tstat[i] = 0;
    if (threadIdx.x == 0) *it.tctr = 0u;
    if (!it.has_prev || it.mode_req != 0) {
        if (threadIdx.x == 0) plan.res[r].mode = (it.has_prev && it.mode_req == 2) ? 1u : 0u;
        return;
    }
    if (kLowReg) {
        switch (it.wb) {
            case 4: enc_trial_body_lowreg<4>(it, lds, plan.res + r); break;
            case 2: enc_trial_body_lowreg<2>(it, lds, plan.res + r); break;
            default: enc_trial_body_lowreg<1>(it, lds, plan.res + r); break;
        }
        return;
    }
    switch (it.wb) {
        case 4: enc_trial_body<4>(it, lds, plan.res + r); break;
        case 2: enc_trial_body<2>(it, lds, plan.res + r); break;
        default: enc_trial_body<1>(it, lds, plan.res + r); break;
    }
}

// Held to three waves per SIMD: left alone the compiler gives the trial 209
// registers, two waves per SIMD, for a kernel bound by its loads' latency;
// at three (168 registers, nothing spilled) it takes 27% less time.
__global__ __launch_bounds__(256, 3) void k_enc_trial(EncPlan plan) {
    // the call's error word starts at zero (a plan reused without an upload
    // keeps the previous call's); no kernel before k_enc_tiles touches it
    if (blockIdx.x == 0 && threadIdx.x == 0) *plan.err = 0u;
    __shared__ TrialLds lds;
    enc_trial_item(plan, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Residuals and frame packing per kFTile-pixel tile.  Each thread reads 32
// consecutive samples (and the previous scan's for a P-scan); the in-range
// residuals -- the sample (I) or its difference to the previous scan
// (P, Sec. III-D) -- are compacted in LDS (zero removal, Sec. III-C), each
// frame in its own row.  Then one quad of lanes codes each frame that lies
// wholly inside the tile (at most 64).  A frame that crosses a tile
// boundary is staged in its slot by each tile it touches (its values, and
// the value before it by the tile where it starts) and coded by
// k_enc_mframe's fixup workgroups.
// ---------------------------------------------------------------------------
template <int WB>
__device__ __forceinline__ uint32_t residual_at(const EncItem& it, uint32_t mode, uint32_t p, uint32_t m) {
    const uint32_t q = quantize(load1<WB>(it.x, p), it.div);
    if (!mode) return q;
    uint32_t qp = load1<WB>(it.xprev, p);
    if (!it.prev_quantized) qp = quantize(qp, it.div);
    return (q - qp) & m;
}


struct TileLds {
    uint32_t rows[kTileFrames * kRow];  // frame rows
    uint32_t sink[256];                 // where the compaction's unkept values go
    uint32_t scratch[8], scratch2[8];
    uint32_t pred, kb, tp, ticket;
};

// Look-back state of an encoder tile: bit 63 its own count and last pixel
// are published, bit 62 its running ones are; the in-range count in bits
// 0..30 and the last in-range pixel plus 1 (0: none) in bits 31..61.
constexpr uint64_t kEsAgg = 1ull << 63, kEsIncl = 1ull << 62;
constexpr uint32_t kEncSpinMax = 1u << 16;  // polls before giving up
__device__ __forceinline__ uint32_t es_cnt(uint64_t s) { return (uint32_t)s & 0x7FFFFFFFu; }
__device__ __forceinline__ uint32_t es_lp(uint64_t s) { return (uint32_t)(s >> 31) & 0x7FFFFFFFu; }

// One wave: publishes the tile's count and last pixel, then adds up the
// counts (and takes the largest last pixel) of the tiles before it, from the
// nearest one whose running values are known, 64 tiles per round.  Returns
// the running count before the tile in cnt_before and the last in-range
// pixel plus 1 before it in lp_before.
// Lane l: the state of tile end - 1 - l (before the first tile: nothing).
__device__ __forceinline__ uint64_t enc_lookback_poll(const JG uint64_t* st, uint32_t end) {
    const int idx = (int)end - 1 - (int)lane_id();
    return idx >= 0 ? __hip_atomic_load(st + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kEsIncl;
}

// first: the first round's states when polled earlier (a state only moves
// from empty to aggregate to inclusive, so an early read is as valid as a
// late one), has_first whether it was
__device__ void enc_lookback(JG uint64_t* st, uint32_t lt, uint32_t cnt, uint32_t lp, JG uint32_t* err,
                             uint32_t& cnt_before, uint32_t& lp_before, uint64_t first, bool has_first) {
    const uint32_t l = lane_id();
    if (l == 0)
        __hip_atomic_store(st + lt, (lt ? kEsAgg : kEsIncl) | cnt | ((uint64_t)lp << 31), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    uint32_t ec = 0, el = 0, end = lt, spins = 0;  // tiles [0, end) not combined yet
    while (end > 0) {
        const uint64_t s = has_first ? first : enc_lookback_poll(st, end);
        has_first = false;
        const uint64_t f = s & (kEsAgg | kEsIncl);
        const uint64_t incl = ballot(f == kEsIncl), empty = ballot(f == 0);
        const uint32_t fi = incl ? (uint32_t)__builtin_ctzll(incl) : 64u;
        const uint32_t fe = empty ? (uint32_t)__builtin_ctzll(empty) : 64u;
        if (fe < fi) {  // a nearer tile has not published: take the ones before it, poll again
            if (fe) {
                ec += wave_sum(l < fe ? es_cnt(s) : 0u);
                el = max(el, wave_max(l < fe ? es_lp(s) : 0u));
                end -= fe;
            }
            if (++spins > kEncSpinMax) {  // never expected: a tile before this one did not publish
                if (l == 0) atomicOr(err, kErrStall);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        ec += wave_sum(l <= fi ? es_cnt(s) : 0u);
        el = max(el, wave_max(l <= fi ? es_lp(s) : 0u));
        if (fi < 64) break;
        end -= 64;
    }
    if (l == 0 && lt)
        __hip_atomic_store(st + lt, kEsIncl | (ec + cnt) | ((uint64_t)max(el, lp) << 31), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    cnt_before = ec;
    lp_before = el;
}

// A thread's 32 samples of tile lt.
template <int WB>
__device__ __forceinline__ void enc_tile_load(const EncItem& it, uint32_t lt, uint32_t s[32]) {
    const uint32_t p0 = lt * kFTile + threadIdx.x * 32;
    if (p0 < it.npx) {
        load16<WB>(it.x, p0, it.npx, it.aligned16, s);
        load16<WB>(it.x, p0 + 16, it.npx, it.aligned16, s + 16);
    }
}

// s: the thread's samples, as enc_tile_load gives them
// first_poll: wave 0's first look-back round when has_poll (see enc_lookback)
template <int WB>
__device__ __forceinline__ void enc_tile_body(const EncPlan& plan, const EncItem& it, uint32_t r, uint32_t lt,
                                              uint32_t mode, TileLds& L, uint32_t s[32], uint64_t first_poll = 0,
                                              bool has_poll = false) {
    const uint32_t m = low_mask32(it.bits);
    const uint32_t tid = threadIdx.x;
    const uint32_t p0 = lt * kFTile + tid * 32;
    uint32_t keep = 0;
    if (p0 < it.npx) {
        uint32_t xp[32];
        if (mode) {
            load16<WB>(it.xprev, p0, it.npx, it.aligned16, xp);
            load16<WB>(it.xprev, p0 + 16, it.npx, it.aligned16, xp + 16);
        }
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            s[i] = quantize(s[i], it.div);
            keep |= (s[i] != 0 ? 1u : 0u) << i;
        }
        if (it.qout) {  // the quantized scan, kept for the next scan's prediction
            store16<WB>(it.qout, p0, it.npx, it.aligned16, s);
            if (p0 + 16 < it.npx) store16<WB>(it.qout, p0 + 16, it.npx, it.aligned16, s + 16);
        }
        if (mode) {
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const uint32_t qp = it.prev_quantized ? xp[i] : quantize(xp[i], it.div);
                s[i] = (s[i] - qp) & m;
            }
        }
    }
    {  // the zero bitmask: one 64-pixel word per pair of threads
        const uint64_t w = (uint64_t)keep | ((uint64_t)__shfl_down(keep, 1, kWave) << 32);
        if (!(tid & 1u) && p0 < it.npx) it.vw[p0 >> 6] = w;
    }
    uint32_t nv, lp_tile;
    const uint32_t off = block_excl_scan<256>(__popc(keep), L.scratch, &nv);
    (void)block_excl_max<256>(keep ? p0 + 32u - (uint32_t)__clz(keep) : 0u, L.scratch2, &lp_tile);
    // in-range samples and the last in-range pixel before this tile, from the tiles before it
    if (tid < kWave) {
        uint32_t kb_w, tp_w;
        enc_lookback(it.tstat, lt, nv, lp_tile, plan.err, kb_w, tp_w, first_poll, has_poll);
        if (tid == 0) {
            L.kb = kb_w;
            L.tp = tp_w;  // the pixel after the last in-range one before the tile (0: none)
            if (lt + 1 == it.ntiles) {  // the record's last tile knows its count
                plan.res[r].N = kb_w + nv;
                plan.res[r].nb = div_up(kb_w + nv, kFrame);
            }
        }
    }
    __syncthreads();
    const uint32_t kb = L.kb;
    // the residual before the tile's first value, needed only when that value
    // starts a frame (else the frame's predecessor is a value of this tile, or
    // the frame crosses into the tile and its start stages the predecessor);
    // its load overlaps the compaction
    const uint32_t tp = L.tp;
    const uint32_t pred_v = (tid == 0 && tp && !(kb & 127u)) ? residual_at<WB>(it, mode, tp - 1, m) : 0u;
    // the record's size is known in its last tile only: elsewhere a frame that
    // runs past the tile's values is taken to continue in a later tile (if it
    // is the record's last, the fixup workgroups code it)
    const uint32_t N = lt + 1 == it.ntiles ? kb + nv : 0xFFFFFFFFu;
    const uint32_t jf = kb >> 7;
    {
        // kept values go to their row; the others to this thread's sink word
        uint32_t k = kb + off;  // index of the next kept value
        uint32_t* const dummy = L.sink + tid;
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            const bool kp = (keep >> i) & 1u;
            *(kp ? L.rows + tile_word(k, jf) : dummy) = s[i];
            k += kp ? 1u : 0u;
        }
    }
    if (tid == 0) L.pred = pred_v;
    __syncthreads();
    if (nv == 0) {
        if (tid == 0) it.tfix[lt] = kNoFix;
        return;
    }
    const uint32_t ke = kb + nv;  // end of the tile's values
    const uint32_t jl = (ke - 1) >> 7;
    const uint32_t kl0 = jl << 7, kl1 = min(kl0 + kFrame, N);
    const bool head_part = (kb & 127u) != 0;               // frame jf began in an earlier tile
    const bool tail_part = kl1 > ke && !(jl == jf && head_part);  // frame jl starts here, ends later
    if (tid == 0) it.tfix[lt] = tail_part ? jl : kNoFix;
    auto value_at = [&](uint32_t k) { return L.rows[tile_word(k, jf)]; };
    // stage the crossing frames: thread t < 128 value t of frame jf, t >= 128 value t - 128 of frame jl
    if (tid < kFrame) {
        const uint32_t k = (jf << 7) + tid;
        if (head_part && k >= kb && k < ke) ((JG uint32_t*)(it.slots + (size_t)jf * kSlotBytes))[tid] = value_at(k);
    } else {
        const uint32_t i = tid - kFrame, k = kl0 + i;
        JG uint32_t* sw = (JG uint32_t*)(it.slots + (size_t)jl * kSlotBytes);
        if (tail_part && k < ke) sw[i] = value_at(k);
        if (tail_part && i == 0) sw[kFrame] = kl0 > kb ? value_at(kl0 - 1) : L.pred;
    }
    // the whole frames: quad g codes frame jc0 + g
    const uint32_t g = tid >> 2, q = tid & 3u;
    const uint32_t j = ((kb + 127u) >> 7) + g;
    const uint32_t k0 = j << 7, kend = min(k0 + kFrame, N);
    const bool whole = k0 < ke && kend <= ke;
    uint32_t pred = 0;
    if (whole) pred = k0 > kb ? value_at(k0 - 1) : L.pred;
    __syncthreads();  // every row is read before its quad overwrites it
    if (!whole) return;
    code_frame_quad(L.rows + (j - jf) * kRow, kend - k0, pred, it.bits, q,
                    it.slots + (size_t)j * kSlotBytes, it.blkinfo + j);
}

template <int WB>
__device__ __forceinline__ void enc_tile_run(const EncPlan& plan, const EncItem& it, uint32_t r, uint32_t lt,
                                             uint32_t mode, TileLds& lds) {
    uint32_t s[32];
    enc_tile_load<WB>(it, lt, s);
    enc_tile_body<WB>(plan, it, r, lt, mode, lds, s);
}

// mode: the record's trial result (0 = I, 1 = P)
__device__ __forceinline__ void enc_tile_item(const EncPlan& plan, const EncItem& it, uint32_t r, uint32_t lt,
                                              uint32_t mode, TileLds& lds) {
    switch (it.wb) {
        case 4: enc_tile_run<4>(plan, it, r, lt, mode, lds); break;
        case 2: enc_tile_run<2>(plan, it, r, lt, mode, lds); break;
        default: enc_tile_run<1>(plan, it, r, lt, mode, lds); break;
    }
}

// The record is fixed by the workgroup index; the tile within it is taken
// in arrival order (a ticket), so every tile a workgroup waits for has
// started.  With records of one size the workgroups are laid out tile-major
// (workgroup i serves record i mod n), so a record's tiles arrive far apart
// and, as workgroups usually arrive in index order, in order: the samples
// of the tile the index names are requested while the ticket is on its way,
// and requested again only when the ticket names another tile.
template <int WB>
__device__ __forceinline__ void enc_tile_ticketed(const EncPlan& plan, const EncItem& it, uint32_t r,
                                                  uint32_t lt_guess, uint32_t mode, TileLds& lds) {
    uint32_t s[32];
    if (lt_guess < it.ntiles) enc_tile_load<WB>(it, lt_guess, s);
    __syncthreads();
    const uint32_t lt = lds.ticket;
    if (lt >= it.ntiles) {  // never expected: the record's ticket counter was not cleared
        if (threadIdx.x == 0) atomicOr(plan.err, kErrStall);
        return;
    }
    if (lt != lt_guess) enc_tile_load<WB>(it, lt, s);
    // the tiles before this one were dispatched long before (tile-major), so
    // one early read of their states usually settles the look-back
    uint64_t poll = 0;
    if (threadIdx.x < kWave) poll = enc_lookback_poll(it.tstat, lt);
    enc_tile_body<WB>(plan, it, r, lt, mode, lds, s, poll, true);
}

__global__ __launch_bounds__(256) void k_enc_tiles(EncPlan plan) {
    uint32_t lt_guess, r;
    if (plan.ftpi) {
        r = blockIdx.x % plan.n_items;
        lt_guess = blockIdx.x / plan.n_items;
    } else {
        r = tile_owner(plan.ftile_item, plan.ftile_first, plan.ftpi, blockIdx.x, lt_guess);
    }
    const EncItem it = plan.items[r];
    __shared__ TileLds lds;
    if (threadIdx.x == 0) lds.ticket = atomicAdd(it.tctr, 1u);
    const uint32_t mode = plan.res[r].mode;  // requested with the ticket
    switch (it.wb) {
        case 4: enc_tile_ticketed<4>(plan, it, r, lt_guess, mode, lds); break;
        case 2: enc_tile_ticketed<2>(plan, it, r, lt_guess, mode, lds); break;
        default: enc_tile_ticketed<1>(plan, it, r, lt_guess, mode, lds); break;
    }
}

// The frames that cross tile boundaries: one quad per tile entry, the tile
// entries [t0, t0 + kFixQuads) per workgroup; the staged values go to the
// quad's LDS row first.  Runs in workgroups of k_enc_mframe (see there).
constexpr uint32_t kFixQuads = kFixGroup;
__device__ __forceinline__ void enc_fixup_quads(const EncPlan& plan, uint32_t t0, uint32_t* rows) {
    const uint32_t g = threadIdx.x >> 2, q = threadIdx.x & 3u;
    const uint32_t t = t0 + g;
    if (g >= kFixQuads || t >= plan.n_ftiles) return;  // no barrier follows
    uint32_t lt;
    const uint32_t r = tile_owner(plan.ftile_item, plan.ftile_first, plan.ftpi, t, lt);
    const EncItem& it = plan.items[r];
    const uint32_t j = it.tfix[lt];
    if (j == kNoFix || j >= it.maxnb) return;
    const uint32_t N = plan.res[r].N;
    const uint32_t real = min(kFrame, N - j * kFrame);
    JG uint8_t* slot = it.slots + (size_t)j * kSlotBytes;
    const JG uint4* s4 = (const JG uint4*)slot;
    uint4* v4 = (uint4*)(rows + g * kRow + 36 * q);
#pragma unroll
    for (int c = 0; c < 8; ++c) v4[c] = s4[8 * q + c];
    const uint32_t pred = ((const JG uint32_t*)slot)[kFrame];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    code_frame_quad(rows + g * kRow, real, pred, it.bits, q, slot, it.blkinfo + j);
}

// ---------------------------------------------------------------------------
// Mask frame (Sec. III-C/D): content byte i holds mask bits 8i..8i+7 (bit = 1:
// zero sample), XORed with the previous mask for a P-scan.  Runs of >= 8
// equal bytes become RLE blocks, the stretches between them Raw blocks,
// each split at 128 KiB (RFC 8878 frame, single segment, no checksum).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t content_word(const EncItem& it, uint32_t mode, uint32_t w) {
    const uint64_t tm = tail_mask(w, it.nwords, it.npx);
    uint64_t mk = ~it.vw[w] & tm;
    if (mode) mk ^= ~it.vwprev[w] & tm;
    return mk;
}
__device__ __forceinline__ uint32_t content_byte(const EncItem& it, uint32_t mode, uint32_t i) {
    return (uint32_t)(content_word(it, mode, i >> 3) >> (8 * (i & 7))) & 0xFFu;
}

// Run classification of content bytes [b0, b0 + 32): bit k of `lng` is set
// when byte b0 + k lies in a run of >= kRleMinRun equal bytes; bit k of
// `start` when a segment (an RLE run or a raw stretch) begins there.
// Works on a 64-byte window [b0 - 16, b0 + 48) held in eight words.
struct RunBits {
    uint32_t lng, start;
    uint64_t win[8];
};
__device__ __forceinline__ void classify32(const EncItem& it, uint32_t mode, uint32_t nm, uint32_t b0, RunBits& R) {
    const int w0 = (int)(b0 >> 3) - 2;  // b0 is a multiple of 32
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int w = w0 + k;
        R.win[k] = (w >= 0 && (uint32_t)w < it.nwords && 8u * (uint32_t)w < nm) ? content_word(it, mode, w) : 0ull;
    }
    // eq bit k: byte (b0 - 16 + k) equals the byte before it (both inside the
    // content).  Four bytes at a time: XOR each byte with its predecessor,
    // flag the zero bytes exactly (no carries between bytes: the low seven
    // bits are added separately), gather the four flags with a multiply.
    uint64_t eq = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t w = (uint32_t)(R.win[j >> 1] >> (32 * (j & 1)));
        const uint32_t pw = j ? (uint32_t)(R.win[(j - 1) >> 1] >> (32 * ((j - 1) & 1))) : 0u;
        const uint32_t y = w ^ __builtin_amdgcn_alignbyte(w, pw, 3);  // byte t XOR byte t - 1
        const uint32_t z = ~(((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y | 0x7F7F7F7Fu);  // bit 8t + 7: byte t of y is 0
        eq |= (uint64_t)((((z >> 7) & 0x01010101u) * 0x10204081u) >> 28) << (4 * j);
    }
    {  // pairs inside the content only: byte k - 1 at or after its start, byte k before its end
        const int lo = b0 == 0 ? 16 : 0;  // b0 is a multiple of 32
        const int hi = min(64, (int)nm + 16 - (int)b0);
        uint64_t vm = 0;
        if (hi > lo + 1) vm = (hi >= 64 ? ~0ull : ((1ull << hi) - 1ull)) & ~((1ull << (lo + 1)) - 1ull);
        eq &= vm;
    }
    // e8 bit k: bytes k .. k+7 all equal; lng bit k: some such window covers k
    uint64_t e8 = ~0ull;
    for (int d = 1; d < (int)kRleMinRun; ++d) e8 &= eq >> d;
    e8 &= ~0ull >> (kRleMinRun - 1);  // windows that leave the 64-byte view are unknown: not long
    uint64_t lng = 0;
    for (int d = 0; d < (int)kRleMinRun; ++d) lng |= e8 << d;
    // bytes b0-1 .. b0+31 are window bits 15 .. 47
    const uint64_t cur = lng >> 16, prv = lng >> 15, neq = ~(eq >> 16);
    uint64_t st = ((cur ^ prv) | (cur & neq)) & 0xFFFFFFFFull;
    if (b0 == 0) st |= 1ull;
    uint32_t valid = nm > b0 ? (nm - b0 >= 32 ? 0xFFFFFFFFu : ((1u << (nm - b0)) - 1u)) : 0u;
    R.lng = (uint32_t)cur & valid;
    R.start = (uint32_t)st & valid;
}

// Content byte b0 + k (k < 32) of a classified window: selects among its four
// middle words, so that the window stays in registers (an index computed at
// run time would move it to scratch memory).
__device__ __forceinline__ uint32_t win_byte(const RunBits& R, uint32_t k) {
    const uint32_t q = k >> 3;
    uint64_t w = 0;
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) w |= R.win[2 + c] & (q == c ? ~0ull : 0ull);
    return (uint32_t)(w >> (8 * (k & 7))) & 0xFFu;
}

constexpr uint32_t kMfThreads = 512;   // the mask-frame kernel: one workgroup per record covers 16 KiB per round
constexpr uint32_t kMfKeep = 4;        // rounds whose classification stays in registers between passes
constexpr uint32_t kMfSegLds = 6144;   // segments its LDS table holds (more: the workspace table)

template <int NT, int SEGS>
struct alignas(16) MfLds {
    uint32_t segs[SEGS];    // segment start | RLE << 31
    uint32_t segoff[SEGS];  // its offset in the frame
    uint8_t segb[SEGS];     // an RLE segment's byte
    uint32_t scratch[NT / 64 + 1];
};

// Pass 1 of one round: the round's segment starts, numbered from nseg, go
// to the LDS table (those that fit) or to the workspace table.
template <int NT, int SEGS>
__device__ __forceinline__ void mframe_starts(const EncItem& it, const RunBits& R, uint32_t b0, bool to_ws,
                                              MfLds<NT, SEGS>& M, uint32_t& nseg) {
    uint32_t total;
    uint32_t sid = block_excl_scan<NT>(__popc(R.start), M.scratch, &total) + nseg;
    for (uint32_t m = R.start; m; m &= m - 1) {
        const uint32_t k = __ffs(m) - 1;
        const uint32_t e = (b0 + k) | (((R.lng >> k) & 1u) << 31);
        if (to_ws) it.segs[sid] = e;
        else if (sid < (uint32_t)SEGS) {
            M.segs[sid] = e;
            M.segb[sid] = (uint8_t)win_byte(R, k);
        }
        ++sid;
    }
    nseg += total;
}

// Passes 2 and 3 over the segment table (in LDS, or in the workspace).
template <bool kLds, int NT, int SEGS>
__device__ __forceinline__ void mframe_write(const EncPlan& plan, uint32_t r, const EncItem& it, uint32_t mode,
                                             uint32_t nm, uint32_t nseg, uint32_t hdr, MfLds<NT, SEGS>& M,
                                             RunBits (&Rk)[kMfKeep]) {
    constexpr uint32_t kStep = NT * 32;
    const uint32_t tid = threadIdx.x;
    auto seg = [&](uint32_t i) -> uint32_t { return kLds ? M.segs[i] : it.segs[i]; };
    auto segoff = [&](uint32_t i) -> uint32_t { return kLds ? M.segoff[i] : it.segoff[i]; };
    // pass 2: encoded sizes and offsets of the segments
    uint32_t off_carry = hdr;
    for (uint32_t s0 = 0; s0 < nseg; s0 += NT) {
        const uint32_t sg = s0 + tid;
        uint32_t size = 0;
        if (sg < nseg) {
            const uint32_t a = seg(sg);
            const uint32_t start = a & 0x7FFFFFFFu;
            const uint32_t end = (sg + 1 < nseg) ? (seg(sg + 1) & 0x7FFFFFFFu) : nm;
            const uint32_t len = end - start;
            const uint32_t nblk = div_up(len, kZstdBlockMax);
            size = (a >> 31) ? 4u * nblk : 3u * nblk + len;
        }
        uint32_t total;
        const uint32_t off = block_excl_scan<NT>(size, M.scratch, &total) + off_carry;
        if (sg < nseg) {
            if (kLds) M.segoff[sg] = off;
            else it.segoff[sg] = off;
        }
        off_carry += total;
    }
    __syncthreads();
    // pass 3: write the frame
    uint8_t* f = it.frame;
    if (tid == 0) {
        f[0] = 0x28; f[1] = 0xB5; f[2] = 0x2F; f[3] = 0xFD;
        if (nm <= 255) { f[4] = 0x20; f[5] = (uint8_t)nm; }
        else if (nm <= 65791) { f[4] = 0x60; f[5] = (uint8_t)(nm - 256); f[6] = (uint8_t)((nm - 256) >> 8); }
        else { f[4] = 0xA0; f[5] = (uint8_t)nm; f[6] = (uint8_t)(nm >> 8); f[7] = (uint8_t)(nm >> 16); f[8] = (uint8_t)(nm >> 24); }
        plan.res[r].flen = off_carry;
        plan.res[r].nseg = nseg;
    }
    // block headers (and the byte of each RLE block)
    for (uint32_t sg = tid; sg < nseg; sg += NT) {
        const uint32_t a = seg(sg);
        const uint32_t start = a & 0x7FFFFFFFu;
        const uint32_t end = (sg + 1 < nseg) ? (seg(sg + 1) & 0x7FFFFFFFu) : nm;
        const uint32_t len = end - start;
        const uint32_t nblk = div_up(len, kZstdBlockMax);
        const uint32_t is_rle = a >> 31;
        const uint32_t rb = is_rle ? (kLds ? (uint32_t)M.segb[sg] : content_byte(it, mode, start)) : 0u;
        uint32_t o = segoff(sg);
        for (uint32_t q = 0; q < nblk; ++q) {
            const uint32_t blen = min(kZstdBlockMax, len - q * kZstdBlockMax);
            const uint32_t last = (sg + 1 == nseg && q + 1 == nblk) ? 1u : 0u;
            const uint32_t h = last | (is_rle << 1) | (blen << 3);
            f[o] = (uint8_t)h; f[o + 1] = (uint8_t)(h >> 8); f[o + 2] = (uint8_t)(h >> 16);
            if (is_rle) {
                f[o + 3] = (uint8_t)rb;
                o += 4;
            } else {
                o += 3 + blen;
            }
        }
    }
    // raw bytes: the segment of every byte from the same classification
    uint32_t seg_carry = 0;
    auto raw_round = [&](const RunBits& R, uint32_t b0) {
        uint32_t total;
        uint32_t sid = block_excl_scan<NT>(__popc(R.start), M.scratch, &total) + seg_carry;
        const uint32_t nvalid = nm > b0 ? min(32u, nm - b0) : 0u;
        uint32_t sg = sid ? sid - 1 : 0, sstart = 0, soff = 0;
        if (sid) { sstart = seg(sg) & 0x7FFFFFFFu; soff = segoff(sg); }
        // unrolled, so that each byte's place in the window is fixed (the
        // words named one by one: an array indexed in the loop would go to
        // scratch memory before the unrolling)
        const uint64_t w0 = R.win[2], w1 = R.win[3], w2 = R.win[4], w3 = R.win[5];
#pragma unroll
        for (uint32_t k = 0; k < 32; ++k) {
            if (k >= nvalid) break;
            if ((R.start >> k) & 1u) {
                sg = sid++;
                sstart = b0 + k;
                soff = segoff(sg);
            }
            if ((R.lng >> k) & 1u) continue;
            const uint32_t i = b0 + k;
            const uint32_t q = (i - sstart) / kZstdBlockMax;
            const uint64_t wk = k < 8 ? w0 : k < 16 ? w1 : k < 24 ? w2 : w3;
            f[soff + 3u * (q + 1u) + (i - sstart)] = (uint8_t)(wk >> (8 * (k & 7)));
        }
        seg_carry += total;
    };
#pragma unroll
    for (uint32_t c = 0; c < kMfKeep; ++c)
        if (c * kStep < nm) raw_round(Rk[c], c * kStep + 32 * tid);
    for (uint32_t c0 = kMfKeep * kStep; c0 < nm; c0 += kStep) {
        RunBits R;
        classify32(it, mode, nm, c0 + 32 * tid, R);
        raw_round(R, c0 + 32 * tid);
    }
}

// The mask frame of record r, by a workgroup of NT threads.  Pass 1 finds
// the segment starts (the first kMfKeep rounds' classification is kept in
// registers for the raw bytes); the segment table lives in LDS when it
// fits, else in the workspace.
template <int NT, int SEGS>
__device__ __forceinline__ void enc_mframe_item(const EncPlan& plan, uint32_t r, MfLds<NT, SEGS>& M) {
    constexpr uint32_t kStep = NT * 32;
    const EncItem it = plan.items[r];
    const uint32_t mode = plan.res[r].mode;
    const uint32_t nm = div_up(it.npx, 8);
    const uint32_t hdr = nm <= 255 ? 6u : nm <= 65791 ? 7u : 9u;
    const uint32_t tid = threadIdx.x;
    RunBits Rk[kMfKeep];
    uint32_t nseg = 0;
    // the kept rounds classified first (no barrier between them, so their
    // loads are in flight together), then their segment starts numbered
#pragma unroll
    for (uint32_t c = 0; c < kMfKeep; ++c)
        if (c * kStep < nm) classify32(it, mode, nm, c * kStep + 32 * tid, Rk[c]);
#pragma unroll
    for (uint32_t c = 0; c < kMfKeep; ++c)
        if (c * kStep < nm) mframe_starts(it, Rk[c], c * kStep + 32 * tid, false, M, nseg);
    for (uint32_t c0 = kMfKeep * kStep; c0 < nm; c0 += kStep) {
        RunBits R;
        classify32(it, mode, nm, c0 + 32 * tid, R);
        mframe_starts(it, R, c0 + 32 * tid, false, M, nseg);
    }
    __syncthreads();
    if (nseg <= (uint32_t)SEGS) {
        mframe_write<true>(plan, r, it, mode, nm, nseg, hdr, M, Rk);
        return;
    }
    // too many segments for LDS: the starts again, into the workspace table
    nseg = 0;
#pragma unroll
    for (uint32_t c = 0; c < kMfKeep; ++c)
        if (c * kStep < nm) mframe_starts(it, Rk[c], c * kStep + 32 * tid, true, M, nseg);
    for (uint32_t c0 = kMfKeep * kStep; c0 < nm; c0 += kStep) {
        RunBits R;
        classify32(it, mode, nm, c0 + 32 * tid, R);
        mframe_starts(it, R, c0 + 32 * tid, true, M, nseg);
    }
    __syncthreads();
    mframe_write<false>(plan, r, it, mode, nm, nseg, hdr, M, Rk);
}

// One workgroup per record (the workgroups after them code the tile-crossing
// frames, enc_fixup_quads, in the same LDS).
union MfKernelLds {
    MfLds<kMfThreads, kMfSegLds> mf;
    uint32_t fix[kFixQuads * kRow];
};
__global__ __launch_bounds__(kMfThreads) void k_enc_mframe(EncPlan plan) {
    __shared__ MfKernelLds M;
    if (blockIdx.x >= plan.n_items) {  // the tile-crossing frames: independent of the masks, same launch
        enc_fixup_quads(plan, (blockIdx.x - plan.n_items) * kFixQuads, M.fix);
        return;
    }
    enc_mframe_item(plan, blockIdx.x, M.mf);
}

// ---------------------------------------------------------------------------
// Section layout of each record: prefix sums of payload, position and high
// part sizes over its frames (the three in one pass of 1024 frames); the
// record length.
// ---------------------------------------------------------------------------
constexpr int kSizeThreads = 1024;

template <int NT>
__device__ __forceinline__ void enc_sizes_item(const EncPlan& plan, uint32_t r, uint32_t* scratch /* 3 * (NT/64 + 1) */) {
    const EncItem& it = plan.items[r];
    const uint32_t nb = min(plan.res[r].nb, it.maxnb);  // (never more; kept in bounds whatever a stall left)
    uint32_t cp = 0, cn = 0, ch = 0;
    // the widths of kAhead passes are requested together, then scanned pass by pass
    constexpr uint32_t kAhead = 4;
    for (uint32_t ja = 0; ja < nb; ja += NT * kAhead) {
        uint32_t infos[kAhead];
#pragma unroll
        for (uint32_t u = 0; u < kAhead; ++u) {
            const uint32_t j = ja + NT * u + threadIdx.x;
            infos[u] = j < nb ? it.blkinfo[j] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < kAhead; ++u) {
            if (ja + NT * u >= nb) break;
            const uint32_t j = ja + NT * u + threadIdx.x;
            uint32_t v[3] = {0u, 0u, 0u};  // payload, position and high part bytes of frame j
            if (j < nb) {
                const uint32_t info = infos[u];
                const uint32_t b = info & 0xFF, n = (info >> 8) & 0xFF, B = (info >> 16) & 0xFF;
                v[0] = 16 * b;
                v[1] = n;
                v[2] = (n * (B - b) + 7) / 8;
            }
            uint32_t tot[3];
            block_excl_scan3<NT>(v, scratch, tot);
            if (j < nb) {
                it.blkoffs[3 * j] = cp + v[0];
                it.blkoffs[3 * j + 1] = cn + v[1];
                it.blkoffs[3 * j + 2] = ch + v[2];
            }
            cp += tot[0]; cn += tot[1]; ch += tot[2];
        }
    }
    if (threadIdx.x == 0) {
        EncRes& rs = plan.res[r];
        rs.pay = cp;
        rs.pos = cn;
        rs.high = ch;
        rs.rec_len = align4(12 + rs.flen) + align4(4 + 3 * nb) + align4(cp + cn + ch);
    }
}

__global__ __launch_bounds__(kSizeThreads) void k_enc_sizes(EncPlan plan) {
    __shared__ uint32_t scratch[3 * (kSizeThreads / kWave + 1)];
    enc_sizes_item<kSizeThreads>(plan, blockIdx.x, scratch);
}

// ---------------------------------------------------------------------------
// Record offsets: one prefix sum over all records, rebased per output.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_enc_offsets(EncPlan plan) {
    __shared__ uint64_t scratch[20];
    // record lengths of kAhead rounds are requested together, then scanned round by round
    constexpr uint32_t kAhead = 8;
    uint64_t carry = 0;
    for (uint32_t ra = 0; ra < plan.n_items; ra += 1024 * kAhead) {
        uint32_t lens[kAhead];
#pragma unroll
        for (uint32_t u = 0; u < kAhead; ++u) {
            const uint32_t r = ra + 1024 * u + threadIdx.x;
            lens[u] = r < plan.n_items ? plan.res[r].rec_len : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < kAhead; ++u) {
            if (ra + 1024 * u >= plan.n_items) break;
            const uint32_t r = ra + 1024 * u + threadIdx.x;
            uint64_t total;
            const uint64_t pre = block_excl_scan64<1024>((uint64_t)lens[u], scratch, &total) + carry;
            if (r < plan.n_items) plan.res[r].rec_off = pre;
            carry += total;
        }
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < plan.n_outs; k += 1024) {
        EncOut& o = plan.outs[k];
        uint64_t body = 0, base = 0;
        if (o.n_items) {
            const uint32_t last = o.first_item + o.n_items - 1;
            base = plan.res[o.first_item].rec_off;
            body = plan.res[last].rec_off + plan.res[last].rec_len - base;
        }
        o.gbase = base;
        o.len = o.hdr_len + body;
        o.ok = o.len <= o.cap ? 1u : 0u;
        if (!o.ok) atomicOr(plan.err, kErrCapacity);
        if (plan.host_res) {
            JG uint32_t* h = (JG uint32_t*)plan.host_res + 4 * k;
            store_system(h, (uint32_t)o.len);
            store_system(h + 1, (uint32_t)(o.len >> 32));
            store_system(h + 2, o.ok);
        }
    }
    __syncthreads();
    // every record rebased to its output (the reads of kAhead rounds requested together)
    for (uint32_t ra = 0; ra < plan.n_items; ra += 1024 * kAhead) {
        uint32_t oid[kAhead], md[kAhead], ln[kAhead];
        uint64_t off[kAhead];
#pragma unroll
        for (uint32_t u = 0; u < kAhead; ++u) {
            const uint32_t r = min(ra + 1024 * u + threadIdx.x, plan.n_items - 1);  // past the end: the last (unused)
            oid[u] = plan.items[r].out_id;
            off[u] = plan.res[r].rec_off;
            md[u] = plan.res[r].mode;
            ln[u] = plan.res[r].rec_len;
        }
#pragma unroll
        for (uint32_t u = 0; u < kAhead; ++u) {
            const uint32_t r = ra + 1024 * u + threadIdx.x;
            if (r >= plan.n_items) break;
            const EncOut& o = plan.outs[oid[u]];
            plan.res[r].rec_off = off[u] - o.gbase + o.hdr_len;
            if (plan.host_res) {  // the record's mode, and after the error word its length
                JG uint32_t* h = (JG uint32_t*)(plan.host_res + 16ull * plan.n_outs);
                store_system(h + r, md[u]);
                store_system(h + plan.n_items + 1 + r, ln[u]);
            }
        }
    }
    if (plan.host_res && threadIdx.x == 0)
        store_system((JG uint32_t*)(plan.host_res + 16ull * plan.n_outs) + plan.n_items, *plan.err);
}

// ---------------------------------------------------------------------------
// Assembly.  Part 0 of record r: its header, mask frame, section header and
// padding (and the stream header and table for an output's first record);
// part p >= 1: the packed frames of group p - 1.  The kernel runs one
// workgroup per (part, record).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void enc_assemble_item(const EncPlan& plan, uint32_t r, uint32_t part) {
    // the record's results are requested with its item, so that a part past
    // the record's frames (most of the grid for a sparse record) leaves after
    // one round trip
    const EncRes rs = plan.res[r];
    const EncItem it = plan.items[r];
    if (part > 0 && (part - 1) * kAsmFrames >= rs.nb) return;
    const EncOut& o = plan.outs[it.out_id];
    if (!o.ok) return;
    // the record lies inside the output and has at most maxnb frames (always, unless a bounded wait ran out)
    if (rs.rec_off + rs.rec_len > o.cap || rs.nb > it.maxnb) return;
    uint8_t* rec = o.base + rs.rec_off;
    const uint32_t sec = align4(12 + rs.flen);
    const uint32_t hdr4 = align4(4 + 3 * rs.nb);
    const uint32_t pay0 = sec + hdr4, pos0 = pay0 + rs.pay, high0 = pos0 + rs.pos, end = high0 + rs.high;
    const uint32_t tid = threadIdx.x;
    if (part == 0) {
        if (tid == 0) {
            uint32_t* h = (uint32_t*)rec;
            h[0] = rs.rec_len;
            h[1] = rs.mode | (it.attr << 8);
            h[2] = rs.flen;
            *(uint32_t*)(rec + sec) = rs.N;
        }
        {  // the mask frame, eight words per thread per round (loads first)
            const uint32_t nw = rs.flen / 4;
            const uint32_t* fw = (const uint32_t*)it.frame;  // staging and record are word aligned
            uint32_t* dw = (uint32_t*)(rec + 12);
            for (uint32_t k0 = 0; k0 < nw; k0 += 8 * 256) {
                uint32_t v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const uint32_t k = k0 + u * 256 + tid;
                    v[u] = k < nw ? fw[k] : 0u;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const uint32_t k = k0 + u * 256 + tid;
                    if (k < nw) dw[k] = v[u];
                }
            }
            for (uint32_t k = 4 * nw + tid; k < rs.flen; k += 256) rec[12 + k] = it.frame[k];
        }
        for (uint32_t k = 12 + rs.flen + tid; k < sec; k += 256) rec[k] = 0;
        for (uint32_t j0 = 0; j0 < rs.nb; j0 += 8 * 256) {  // widths, counts and maximum widths
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t j = j0 + u * 256 + tid;
                v[u] = j < rs.nb ? it.blkinfo[j] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t j = j0 + u * 256 + tid;
                if (j < rs.nb) {
                    rec[sec + 4 + j] = (uint8_t)(v[u] & 0xFF);
                    rec[sec + 4 + rs.nb + j] = (uint8_t)((v[u] >> 8) & 0xFF);
                    rec[sec + 4 + 2 * rs.nb + j] = (uint8_t)((v[u] >> 16) & 0xFF);
                }
            }
        }
        for (uint32_t k = sec + 4 + 3 * rs.nb + tid; k < pay0; k += 256) rec[k] = 0;
        for (uint32_t k = end + tid; k < rs.rec_len; k += 256) rec[k] = 0;
        if (r == o.first_item && o.hdr_len) {
            uint8_t* s = o.base;
            if (tid == 0) {
                s[0] = 'J'; s[1] = 'F'; s[2] = 'Y'; s[3] = '1';
                *(uint16_t*)(s + 4) = 1;
                *(uint16_t*)(s + 6) = (uint16_t)o.n_attrs;
                *(uint32_t*)(s + 8) = o.height;
                *(uint32_t*)(s + 12) = o.width;
                *(uint32_t*)(s + 16) = o.n_scans;
            }
            if (tid < o.n_attrs) {
                uint32_t* a = (uint32_t*)(s + 20 + 8 * tid);
                a[0] = o.attr_wb[tid];
                a[1] = o.attr_p[tid];
            }
            uint32_t* table = (uint32_t*)(s + 20 + 8 * o.n_attrs);
            for (uint32_t k = tid; k < o.n_items; k += 256) table[k] = plan.res[o.first_item + k].rec_len;
        }
        return;
    }
    // 64 frames per workgroup: 16 lanes per frame, each group of 16 lanes
    // takes four frames.  A frame's slot holds its payload words, then its
    // exception bytes (positions, high parts), at most 512 bytes in all (the
    // width choice never costs more than a frame at full width): the four
    // frames' metadata is loaded in one round, then every word of the four
    // coded frames in another (words past a frame's end read its first word
    // again: no extra traffic), then the stores.  Payload words go to the
    // payload section whole; exception bytes to the position and high-part
    // sections one by one.
    constexpr int kPer = kAsmFrames / 16;
    constexpr uint32_t kCodedMax = 16 * 32;  // bytes of a frame coded at full width
    constexpr int kSlotRounds = kCodedMax / 4 / 16;
    static_assert(kCodedMax <= kSlotBytes, "a coded frame fits its slot");
    const uint32_t jg = (part - 1) * kAsmFrames + (tid >> 4) * kPer;
    if (jg >= rs.nb) return;
    const uint32_t l = tid & 15u;
    uint32_t info[kPer], op[kPer], on[kPer], oh[kPer];
#pragma unroll
    for (int f = 0; f < kPer; ++f) {
        const uint32_t j = min(jg + f, rs.nb - 1);  // past the record's frames: its last again (unused)
        info[f] = it.blkinfo[j];
        op[f] = it.blkoffs[3 * j];
        on[f] = it.blkoffs[3 * j + 1];
        oh[f] = it.blkoffs[3 * j + 2];
    }
    uint32_t v[kPer][kSlotRounds], nwf[kPer];
#pragma unroll
    for (int f = 0; f < kPer; ++f) {
        const uint32_t b = info[f] & 0xFFu, n = (info[f] >> 8) & 0xFFu, B = (info[f] >> 16) & 0xFFu;
        nwf[f] = jg + f < rs.nb ? (16u * b + n + (n * (B - b) + 7u) / 8u + 3u) / 4u : 0u;
        const uint32_t* sw = (const uint32_t*)(it.slots + (size_t)min(jg + f, rs.nb - 1) * kSlotBytes);
#pragma unroll
        for (int u = 0; u < kSlotRounds; ++u) {
            const uint32_t i = l + 16u * u;
            v[f][u] = sw[i < nwf[f] ? i : 0u];
        }
    }
#pragma unroll
    for (int f = 0; f < kPer; ++f) {
        const uint32_t b = info[f] & 0xFFu, n = (info[f] >> 8) & 0xFFu, B = (info[f] >> 16) & 0xFFu;
        const uint32_t ne = n + (n * (B - b) + 7u) / 8u;  // exception bytes
        uint32_t* dw = (uint32_t*)(rec + pay0 + op[f]);  // payloads are whole words
        uint8_t* dpos = rec + pos0 + on[f];
        uint8_t* dhigh = rec + high0 + oh[f];
#pragma unroll
        for (int u = 0; u < kSlotRounds; ++u) {
            const uint32_t i = l + 16u * u;
            if (i >= nwf[f]) continue;
            if (i < 4u * b) {
                dw[i] = v[f][u];
                continue;
            }
            const uint32_t e0 = 4u * (i - 4u * b);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t e = e0 + k;
                const uint8_t byte = (uint8_t)(v[f][u] >> (8 * k));
                if (e < n) dpos[e] = byte;
                else if (e < ne) dhigh[e - n] = byte;
            }
        }
    }
}

// Held to six waves per SIMD (80 registers instead of 86, nothing spilled):
// its workgroups are short chains of loads and stores, so more of them in
// flight pay (3% less time; at eight waves the spills cost 56% more).
__global__ __launch_bounds__(256, 6) void k_enc_assemble(EncPlan plan) { enc_assemble_item(plan, blockIdx.y, blockIdx.x); }

// ---------------------------------------------------------------------------
// Plan upload: 16 bytes per thread from host-mapped memory.
// ---------------------------------------------------------------------------
// Kernel parameters are plain pointers: an address-space qualifier in the
// signature would change the device symbol's name but not the host's.
__global__ __launch_bounds__(256) void k_copy_in(const uint4* src, uint4* dst, uint32_t n16) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n16) ((JG uint4*)dst)[i] = load_system16((const JG uint4*)src + i);
}

// Record copies of a brute-force encode: job j (host-mapped, read with
// system-scope loads) moves len bytes (a multiple of 4) from src to dst,
// both device memory, word by word with every load of a round issued first.
__global__ __launch_bounds__(256) void k_copy_records(const CopyJob* jobs, uint32_t n) {
    const uint32_t j = blockIdx.x;
    if (j >= n) return;
    const uint4 a = load_system16((const JG uint4*)(jobs + j));
    const uint4 b = load_system16((const JG uint4*)(jobs + j) + 1);
    const JG uint32_t* src = (const JG uint32_t*)((uint64_t)a.x | ((uint64_t)a.y << 32));
    JG uint32_t* dst = (JG uint32_t*)((uint64_t)a.z | ((uint64_t)a.w << 32));
    const uint32_t nw = b.x / 4;
    for (uint32_t k0 = 0; k0 < nw; k0 += 8 * 256) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t k = k0 + u * 256 + threadIdx.x;
            v[u] = k < nw ? src[k] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t k = k0 + u * 256 + threadIdx.x;
            if (k < nw) dst[k] = v[u];
        }
    }
}

hipError_t launch_copy_records(const CopyJob* host_jobs, uint32_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    JIFFY_LAUNCH("k_copy_records", k_copy_records, dim3(n), dim3(256), stream, host_jobs, n);
    return hipGetLastError();
}

hipError_t launch_copy_in(const void* host, void* dev, size_t bytes, hipStream_t stream) {
    const uint32_t n16 = (uint32_t)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    JIFFY_LAUNCH("k_copy_in", k_copy_in, dim3(div_up(n16, 256)), dim3(256), stream, (const uint4*)host, (uint4*)dev,
                 n16);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused persistent encoder: every phase of an encode in one launch.  A grid
// of workgroups (at most what the device holds at once) takes work items
// from one queue in order:
//   trial(r) | tile(t) | mask frame(r) | fixup group(g) | sizes(r) | assembly(r, part)
// An item waits (bounded polls, then agent-scope acquire) only for items
// earlier in the queue, each of which a running workgroup has taken, so
// the lowest unfinished item can always proceed: phases of different
// records overlap and no grid-wide barrier is needed.  Completion is
// published with an agent-scope release before the counter update.
// The record offsets are a decoupled look-back over the sizes items.
// ---------------------------------------------------------------------------
constexpr uint32_t kFusedThreads = 256;
constexpr uint32_t kFusedSegs = 4096;               // mask-frame segments kept in LDS
constexpr uint32_t kFusedSpinMax = 1u << 22;        // polls of a dependency before giving up

union FusedLds {
    TrialLds trial;
    TileLds tile;
    MfLds<kFusedThreads, kFusedSegs> mf;
    uint32_t fix[kFixQuads * kRow];
    uint32_t sizes[3 * (kFusedThreads / kWave + 1)];
};
// The fused kernel's LDS, at file scope for its phase functions (only
// k_enc_fused reaches them).
__shared__ FusedLds fused_lds;

__device__ __forceinline__ void fused_trial(const EncPlan& plan, uint32_t r) {
    enc_trial_item<true>(plan, r, fused_lds.trial);
}
__device__ __forceinline__ void fused_tile(const EncPlan& plan, uint32_t r, uint32_t lt) {
    const EncItem it = plan.items[r];
    enc_tile_item(plan, it, r, lt, plan.res[r].mode, fused_lds.tile);
}
__device__ __forceinline__ void fused_mframe(const EncPlan& plan, uint32_t r) { enc_mframe_item(plan, r, fused_lds.mf); }
__device__ __forceinline__ void fused_fixup(const EncPlan& plan, uint32_t t0) { enc_fixup_quads(plan, t0, fused_lds.fix); }
__device__ __forceinline__ void fused_sizes(const EncPlan& plan, uint32_t r) {
    enc_sizes_item<kFusedThreads>(plan, r, fused_lds.sizes);
}
__device__ __forceinline__ void fused_assemble(const EncPlan& plan, uint32_t r, uint32_t part) {
    enc_assemble_item(plan, r, part);
}

// Waits until *w >= target (thread 0 polls), then makes what the producers
// released visible to the workgroup.
__device__ __forceinline__ void fused_wait(const JG uint32_t* w, uint32_t target, JG uint32_t* err) {
    if (threadIdx.x == 0) {
        uint32_t spins = 0;
        while (__hip_atomic_load((uint32_t*)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kFusedSpinMax) {  // never expected: an earlier item did not finish
                atomicOr(err, kErrStall);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Publishes the item's writes (every thread's) and adds v to *w.
__device__ __forceinline__ void fused_signal(JG uint32_t* w, uint32_t v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add((uint32_t*)w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Record look-back state: bit 63 its length is published, bit 62 its
// inclusive offset is; the value in bits 0..61.
constexpr uint64_t kRsAgg = 1ull << 63, kRsIncl = 1ull << 62, kRsVal = kRsIncl - 1;

// One wave: publishes record r's length, then adds up the lengths of the
// records before it in its output (from record `first` on) from the nearest
// one whose inclusive offset is known.  Returns the bytes of the output's
// records before r.
__device__ uint64_t rec_lookback(JG uint64_t* st, uint32_t r, uint32_t first, uint64_t len, JG uint32_t* err) {
    const uint32_t l = lane_id();
    if (l == 0)
        __hip_atomic_store((uint64_t*)st + r, (r > first ? kRsAgg : kRsIncl) | len, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    uint32_t end = r, spins = 0;  // records [first, end) not added yet
    while (end > first) {
        const int idx = (int)end - 1 - (int)l;
        uint64_t v = kRsIncl;  // before the output's first record: nothing
        if (idx >= (int)first) v = __hip_atomic_load((uint64_t*)st + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t f = v & (kRsAgg | kRsIncl);
        const uint64_t incl = ballot(f == kRsIncl), empty = ballot(f == 0);
        const uint32_t fi = incl ? (uint32_t)__builtin_ctzll(incl) : 64u;
        const uint32_t fe = empty ? (uint32_t)__builtin_ctzll(empty) : 64u;
        auto add = [&](uint32_t upto) {  // the values of lanes [0, upto)
            uint64_t x = l < upto ? (v & kRsVal) : 0ull;
            for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
            excl += x;
        };
        if (fe < fi) {  // a nearer record has not published: take the ones before it, poll again
            if (fe) {
                add(fe);
                end -= fe;
            }
            if (++spins > kFusedSpinMax) {
                if (l == 0) atomicOr(err, kErrStall);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        add(min(fi + 1, 64u));
        if (fi < 64) break;
        end -= 64;
    }
    if (l == 0 && r > first)
        __hip_atomic_store((uint64_t*)st + r, kRsIncl | (excl + len), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// The record of assembly item a (asm_first: first item of every record, and the total).
__device__ __forceinline__ uint32_t asm_owner(const JG uint32_t* first, uint32_t n, uint32_t a) {
    uint32_t lo = 0, hi = n;  // the last r with first[r] <= a
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (first[mid] <= a) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kFusedThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_enc_fused(EncPlan plan) {
    __shared__ uint32_t s_item;
    const uint32_t R = plan.n_items, F = plan.n_ftiles, G = plan.n_fix;
    const uint32_t q_tile = R, q_mf = q_tile + F, q_fix = q_mf + R, q_size = q_fix + G, q_asm = q_size + R;
    const uint32_t total = q_asm + plan.n_asm;
    JG uint32_t* dep = plan.fdep;  // per record: trial done, tiles done, mask frame done, -
    for (;;) {
        if (threadIdx.x == 0) s_item = __hip_atomic_fetch_add((uint32_t*)plan.fctl, 1u, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t q = s_item;
        __syncthreads();  // every thread has the item before thread 0 takes the next
        if (q >= total) break;
        if (q < q_tile) {  // trial
            fused_trial(plan, q);
            fused_signal(dep + 4 * q, 1u);
        } else if (q < q_mf) {  // tile, after its record's decision
            uint32_t lt;
            const uint32_t r = tile_owner(plan.ftile_item, plan.ftile_first, plan.ftpi, q - q_tile, lt);
            fused_wait(dep + 4 * r, 1u, plan.err);
            fused_tile(plan, r, lt);
            __syncthreads();
            fused_signal(dep + 4 * r + 1, 1u);
        } else if (q < q_fix) {  // mask frame, after the record's (and its predecessor's) zero bitmask
            const uint32_t r = q - q_mf;
            const EncItem& it = plan.items[r];
            fused_wait(dep + 4 * r + 1, it.ntiles, plan.err);
            if (it.prev_item != kNoFix) fused_wait(dep + 4 * it.prev_item + 1, plan.items[it.prev_item].ntiles, plan.err);
            fused_mframe(plan, r);
            fused_signal(dep + 4 * r + 2, 1u);
        } else if (q < q_size) {  // tile-crossing frames of 64 tiles, after those records' tiles
            const uint32_t g = q - q_fix, t0 = g * kFixQuads, t1 = min(t0 + kFixQuads, F) - 1;
            uint32_t lt;
            const uint32_t r0 = tile_owner(plan.ftile_item, plan.ftile_first, plan.ftpi, t0, lt);
            const uint32_t r1 = tile_owner(plan.ftile_item, plan.ftile_first, plan.ftpi, t1, lt);
            for (uint32_t r = r0; r <= r1; ++r) fused_wait(dep + 4 * r + 1, plan.items[r].ntiles, plan.err);
            fused_fixup(plan, t0);
            __syncthreads();
            fused_signal(plan.ffix + g, 1u);
        } else if (q < q_asm) {  // sizes and the record's offset in its output
            const uint32_t r = q - q_size;
            const EncItem& it = plan.items[r];
            const uint32_t t0 = plan.ftpi ? r * plan.ftpi : plan.ftile_first[r];
            fused_wait(dep + 4 * r + 1, it.ntiles, plan.err);
            fused_wait(dep + 4 * r + 2, 1u, plan.err);
            for (uint32_t g = t0 / kFixQuads; g <= (t0 + it.ntiles - 1) / kFixQuads; ++g)
                fused_wait(plan.ffix + g, 1u, plan.err);
            fused_sizes(plan, r);
            __syncthreads();
            EncOut& o = plan.outs[it.out_id];
            const bool last = r + 1 == o.first_item + o.n_items;
            if (threadIdx.x < kWave) {
                EncRes& rs = plan.res[r];
                const uint64_t before = rec_lookback(plan.fstat, r, o.first_item, rs.rec_len, plan.err);
                if (threadIdx.x == 0) {
                    rs.rec_off = before + o.hdr_len;
                    if (plan.host_res) {
                        JG uint32_t* h = (JG uint32_t*)(plan.host_res + 16ull * plan.n_outs);
                        store_system(h + r, rs.mode);
                        store_system(h + plan.n_items + 1 + r, rs.rec_len);
                    }
                    if (last) {  // the output's length and whether it fits
                        o.len = o.hdr_len + before + rs.rec_len;
                        o.ok = o.len <= o.cap ? 1u : 0u;
                        if (!o.ok) atomicOr(plan.err, kErrCapacity);
                        if (plan.host_res) {
                            JG uint32_t* h = (JG uint32_t*)plan.host_res + 4 * it.out_id;
                            store_system(h, (uint32_t)o.len);
                            store_system(h + 1, (uint32_t)(o.len >> 32));
                            store_system(h + 2, o.ok);
                        }
                    }
                }
            }
            fused_signal(dep + 4 * r + 3, 1u);
            if (last) fused_signal(plan.fout + it.out_id, 1u);
        } else {  // assembly, once the record's offset and its output's length are known
            const uint32_t a = q - q_asm;
            const uint32_t r = plan.fasm ? asm_owner(plan.fasm, R, a) : a / (plan.max_asm + 1);
            const uint32_t part = a - (plan.fasm ? plan.fasm[r] : r * (plan.max_asm + 1));
            const EncItem& it = plan.items[r];
            const EncOut& o = plan.outs[it.out_id];
            fused_wait(plan.fout + it.out_id, 1u, plan.err);
            fused_wait(dep + 4 * r + 3, 1u, plan.err);
            if (part == 0 && r == o.first_item && o.hdr_len)  // the stream's table holds every record's length
                for (uint32_t k = r; k < r + o.n_items; ++k) fused_wait(dep + 4 * k + 3, 1u, plan.err);
            fused_assemble(plan, r, part);
        }
        __syncthreads();  // the LDS is free for the next item
    }
    // the last workgroup out reports the error word
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (threadIdx.x == 0) {
        const uint32_t d = __hip_atomic_fetch_add((uint32_t*)plan.fctl + 1, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (d + 1 == gridDim.x && plan.host_res) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            store_system((JG uint32_t*)(plan.host_res + 16ull * plan.n_outs) + plan.n_items,
                         __hip_atomic_load((uint32_t*)plan.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        }
    }
}

hipError_t launch_encode_fused(const EncPlan& plan, uint32_t grid, hipStream_t stream) {
    if (plan.n_items == 0) return hipSuccess;
    JIFFY_LAUNCH("k_enc_fused", k_enc_fused, dim3(grid), dim3(kFusedThreads), stream, plan);
    return hipGetLastError();
}

hipError_t fused_occupancy(int* per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_enc_fused, kFusedThreads, 0);
}

hipError_t launch_encode(const EncPlan& plan, hipStream_t stream) {
    if (plan.n_items == 0) return hipSuccess;
    JIFFY_LAUNCH("k_enc_trial", k_enc_trial, dim3(plan.n_items), dim3(256), stream, plan);
    JIFFY_LAUNCH("k_enc_tiles", k_enc_tiles, dim3(plan.n_ftiles), dim3(256), stream, plan);
    JIFFY_LAUNCH("k_enc_mframe", k_enc_mframe, dim3(plan.n_items + div_up(plan.n_ftiles, kFixQuads)),
                 dim3(kMfThreads), stream, plan);
    JIFFY_LAUNCH("k_enc_sizes", k_enc_sizes, dim3(plan.n_items), dim3(kSizeThreads), stream, plan);
    JIFFY_LAUNCH("k_enc_offsets", k_enc_offsets, dim3(1), dim3(1024), stream, plan);
    JIFFY_LAUNCH("k_enc_assemble", k_enc_assemble, dim3(plan.max_asm + 1, plan.n_items), dim3(256), stream, plan);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ablated codecs (Sec. IV-H, Table IV) and the run-length mask codec.  These
// measure record sizes only; no stream is written.
//
// k_abl_levels: levels 1-3 code every pixel of a record, zeros included.
// Each quad takes one frame of 128 pixels, loads and quantizes its lanes'
// 32 values once and costs the frame three times with the coder's width
// choice: the values, their differences to the preceding pixel (modulo
// 2^bits) and the ZigZag codes of those differences.
//
// k_abl_runs: the record's zero bitmask (XOR the previous scan's for the
// P-mask) as alternating runs, the first of in-range pixels and possibly
// empty.  A run starts wherever a pixel's bit differs from its
// predecessor's (the bit before pixel 0 counts as 0), so the run starts are
// the set bits of m ^ (m << 1): one workgroup per record lists them in
// order (a workgroup scan of their counts per 64-pixel word, the words
// built by ballots over 64 consecutive pixels) and then costs the frames of
// run lengths (the first as is, the others minus one), a quad per frame.
// ---------------------------------------------------------------------------
constexpr uint32_t kAblQuads = 64;          // frames per workgroup of k_abl_levels
constexpr uint32_t kAblRunThreads = 1024;   // one workgroup per record of k_abl_runs

template <int WB>
__device__ __forceinline__ void abl_levels_frame(const AblArgs& g, const AblAttr& at, uint32_t t, uint32_t f,
                                                 uint32_t q, uint32_t* hist, uint32_t cost[3]) {
    const uint8_t* base = (const uint8_t*)at.x + (uint64_t)t * g.npx * WB;
    const bool aligned = ((uintptr_t)base & 15u) == 0;
    uint32_t v[32];
    load16<WB>(base, 128u * f + 32u * q, g.npx, aligned, v);
    load16<WB>(base, 128u * f + 32u * q + 16u, g.npx, aligned, v + 16);
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = quantize(v[i], at.div);
    const uint32_t pred = (q == 0 && f > 0) ? quantize(load1<WB>(base, 128u * f - 1u), at.div) : 0u;
    const uint32_t real = min(kFrame, g.npx - 128u * f);
    uint32_t z[32], B;
#pragma unroll
    for (int i = 0; i < 32; ++i) z[i] = v[i];
    cost[0] = quad_frame_key<false, 0>(z, nullptr, hist, real, pred, at.bits, q, B) >> 14;
#pragma unroll
    for (int i = 0; i < 32; ++i) z[i] = v[i];
    cost[1] = quad_frame_key<false, 1>(z, nullptr, hist, real, pred, at.bits, q, B) >> 14;
#pragma unroll
    for (int i = 0; i < 32; ++i) z[i] = v[i];
    cost[2] = quad_frame_key<false, 2>(z, nullptr, hist, real, pred, at.bits, q, B) >> 14;
}

__global__ __launch_bounds__(256) void k_abl_levels(AblArgs g) {
    __shared__ uint32_t hist[kAblQuads * 36];
    __shared__ uint32_t wsum[3];
    const uint32_t r = blockIdx.x / g.chunks, c = blockIdx.x - r * g.chunks;
    const uint32_t t = r / g.A, a = r - t * g.A;
    const uint32_t quad = threadIdx.x >> 2, q = threadIdx.x & 3u;
    const uint32_t f = c * kAblQuads + quad;
    if (threadIdx.x < 3) wsum[threadIdx.x] = 0;
    __syncthreads();
    const AblAttr at = g.attr[a];
    if (f < g.nb) {
        uint32_t cost[3];
        uint32_t* h = hist + 36 * quad;
        if (at.wb == 1) abl_levels_frame<1>(g, at, t, f, q, h, cost);
        else if (at.wb == 2) abl_levels_frame<2>(g, at, t, f, q, h, cost);
        else abl_levels_frame<4>(g, at, t, f, q, h, cost);
        if (q == 0)
            for (int k = 0; k < 3; ++k) atomicAdd(&wsum[k], cost[k]);
    }
    __syncthreads();
    if (threadIdx.x < 3 && wsum[threadIdx.x])
        atomicAdd((unsigned long long*)(g.acc + 8ull * r + threadIdx.x), (unsigned long long)wsum[threadIdx.x]);
}

// bit p of the mask being coded (pixels from npx on read as 0)
template <int WB>
__device__ __forceinline__ bool abl_mask_bit(const uint8_t* base, const uint8_t* prev, uint32_t p, uint32_t npx) {
    if (p >= npx) return false;
    bool b = load1<WB>(base, p) == 0u;
    if (prev) b = b != (load1<WB>(prev, p) == 0u);
    return b;
}

template <int WB>
__device__ void abl_runs_record(const AblArgs& g, const AblAttr& at, uint32_t r, uint32_t t, uint32_t kind,
                                uint32_t* runs, uint32_t* hist, uint32_t* scan, uint64_t* lsum) {
    const uint32_t npx = g.npx, l = lane_id(), wv = threadIdx.x / kWave;
    const uint8_t* base = (const uint8_t*)at.x + (uint64_t)t * npx * WB;
    const uint8_t* prev = kind ? base - (uint64_t)npx * WB : nullptr;
    const uint32_t nwords = div_up(npx, 64u);
    uint32_t K = 0;  // run starts listed so far (pixel 0 counts only when its bit is 1)
    for (uint32_t w0 = 0; w0 < nwords; w0 += kAblRunThreads) {
        const uint32_t wbase = w0 + 64u * wv;
        uint64_t my = 0;  // lane k: mask word wbase + k
        for (uint32_t k = 0; k < 64u && wbase + k < nwords; ++k) {
            const uint64_t m = ballot(abl_mask_bit<WB>(base, prev, 64u * (wbase + k) + l, npx));
            if (l == k) my = m;
        }
        const uint32_t wi = wbase + l;
        uint64_t st = 0;  // run starts in word wi
        if (wi < nwords) {
            const uint64_t carry = wi ? (uint64_t)abl_mask_bit<WB>(base, prev, 64u * wi - 1u, npx) : 0ull;
            st = my ^ ((my << 1) | carry);
            const uint32_t left = npx - 64u * wi;
            if (left < 64u) st &= (1ull << left) - 1ull;
        }
        uint32_t total;
        const uint32_t before = block_excl_scan<kAblRunThreads>((uint32_t)__popcll(st), scan, &total);
        uint32_t* dst = runs + K + before;
        while (st) {
            *dst++ = 64u * wi + (uint32_t)__builtin_ctzll(st);
            st &= st - 1ull;
        }
        K += total;
    }
    __syncthreads();  // every run start stored
    // values: run j spans [E(j), E(j+1)) with E(0) = 0, E(j) = runs[j-1], E(K+1) = npx
    const uint32_t nv = K + 1, nbr = div_up(nv, kFrame);
    const uint32_t quad = threadIdx.x >> 2, q = threadIdx.x & 3u;
    uint64_t sum = 0;
    for (uint32_t fr = quad; fr < nbr; fr += kAblRunThreads / 4) {
        uint32_t z[32], B;
        const uint32_t i0 = 128u * fr + 32u * q;
#pragma unroll
        for (int e = 0; e < 32; ++e) {
            const uint32_t i = i0 + e;
            uint32_t v = 0;
            if (i < nv) {
                const uint32_t lo = i ? runs[i - 1] : 0u;
                const uint32_t hi = i < K ? runs[i] : npx;
                v = hi - lo - (i ? 1u : 0u);
            }
            z[e] = v;
        }
        const uint32_t real = min(kFrame, nv - 128u * fr);
        sum += quad_frame_key<false, 0>(z, nullptr, hist + 36 * quad, real, 0u, 32u, q, B) >> 14;
    }
    if (q == 0 && sum) atomicAdd((unsigned long long*)lsum, (unsigned long long)sum);
    __syncthreads();
    if (threadIdx.x == 0) {
        g.acc[8ull * r + 3 + 2 * kind] = *lsum;
        g.acc[8ull * r + 4 + 2 * kind] = nv;
        *lsum = 0;
    }
    __syncthreads();  // runs and lsum are free for the next record
}

__global__ __launch_bounds__(kAblRunThreads) void k_abl_runs(AblArgs g) {
    __shared__ uint32_t hist[(kAblRunThreads / 4) * 36];
    __shared__ uint32_t scan[kAblRunThreads / kWave + 1];
    __shared__ uint64_t lsum;
    if (threadIdx.x == 0) lsum = 0;
    __syncthreads();
    uint32_t* runs = g.runs + (uint64_t)blockIdx.x * g.npx;
    const uint32_t n = g.T * g.A;
    for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
        const uint32_t t = r / g.A, a = r - t * g.A;
        const AblAttr at = g.attr[a];
        for (uint32_t kind = 0; kind < (t ? 2u : 1u); ++kind) {
            if (at.wb == 1) abl_runs_record<1>(g, at, r, t, kind, runs, hist, scan, &lsum);
            else if (at.wb == 2) abl_runs_record<2>(g, at, r, t, kind, runs, hist, scan, &lsum);
            else abl_runs_record<4>(g, at, r, t, kind, runs, hist, scan, &lsum);
        }
    }
}

hipError_t launch_ablate(const AblArgs& a, uint32_t run_groups, hipStream_t stream) {
    const uint32_t n = a.T * a.A;
    if (n == 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(a.acc, 0, 8ull * n * sizeof(uint64_t), stream);
    if (e != hipSuccess) return e;
    JIFFY_LAUNCH("k_abl_levels", k_abl_levels, dim3(n * a.chunks), dim3(256), stream, a);
    JIFFY_LAUNCH("k_abl_runs", k_abl_runs, dim3(run_groups), dim3(kAblRunThreads), stream, a);
    return hipGetLastError();
}

}  // namespace jiffy
