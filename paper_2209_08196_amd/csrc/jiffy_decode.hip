// Jiffy decoder kernels for gfx950.  Decoding reverses each encoding step
// (Sec. III-C: "a straightforward reversal"):
//
//   k_dec_parse    record header, mask frame (Raw/RLE Zstandard blocks) to mask
//                  bytes, residual-section header and its frame offsets
//   k_dec_mask     mask chain over time: a P-scan's mask is its content XOR
//                  the previous mask (Sec. III-D); valid-sample words
//   k_dec_scan     running count of valid samples; where each frame ends
//   k_dec_fsum     bit unpacking, exception patching (Sec. II), inverse
//                  ZigZag (Eq. 1); the sum of each frame's deltas
//   k_dec_bscan    running sum over frames (undoes the delta, Sec. III-C)
//   k_dec_group    unpacks a group of frames again, running sums inside
//                  them, values back to their pixels, zeros elsewhere
//   k_dec_temporal adds the previous scan for P-scans (Sec. III-D) and
//                  restores the original representation, q * P (Sec. III-A)
//
// Every offset read from the stream is checked before it is used; a
// malformed stream raises kErrCorrupt and later kernels do nothing.
#define JIFFY_KERNEL_TU 1
#include "jiffy_device.h"

namespace jiffy {

constexpr uint32_t kWin = 16384;            // frame positions per parsing window
constexpr uint32_t kChunk = 256;            // bytes per chunk of the chain stitching
constexpr uint32_t kWinChunks = kWin / kChunk;
constexpr uint32_t kJInvalid = 0xFFFFFFFFu; // no valid block chain continues here
constexpr uint32_t kJLast = 0xFFFFFFFEu;    // a last block that ends the frame exactly

__device__ __forceinline__ uint32_t rd32(const uint8_t* p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dec_parse(DecPlan plan) {
    const uint32_t r = blockIdx.x;
    const DecItem it = plan.items[r];
    const uint8_t* rec = it.rec;
    const uint32_t L = it.rec_len;
    const uint32_t nm = div_up(it.npx, 8);
    const uint32_t tid = threadIdx.x;
    __shared__ uint32_t s_err, s_pos, s_done, s_flen, s_mode;
    __shared__ uint32_t scratch[8];

    if (tid == 0) {
        uint32_t err = 0;
        const uint32_t mode = rec[4], attr = rec[5];
        const uint32_t resv = rec[6] | (rec[7] << 8);
        const uint32_t flen = rd32(rec + 8);
        if (mode > 1 || attr != it.attr || resv != 0 || flen > L - 12) err = 1;
        if (mode == 1 && it.t == 0) err = 1;  // nothing to predict from
        uint32_t pos = 0;
        if (!err) {
            const uint8_t* f = rec + 12;
            if (flen < 6 || rd32(f) != 0xFD2FB528u) err = 1;
            else {
                const uint32_t fhd = f[4];
                const uint32_t fcs_flag = fhd >> 6, single = (fhd >> 5) & 1;
                const uint32_t reserved = (fhd >> 3) & 1, checksum = (fhd >> 2) & 1, dict = fhd & 3;
                if (!single || reserved || checksum || dict) err = 1;
                const uint32_t fcs_len = fcs_flag == 0 ? 1 : fcs_flag == 1 ? 2 : fcs_flag == 2 ? 4 : 8;
                pos = 5;
                if (!err && pos + fcs_len > flen) err = 1;
                if (!err) {
                    uint64_t fcs;
                    if (fcs_len == 1) fcs = f[pos];
                    else if (fcs_len == 2) fcs = (uint64_t)(f[pos] | (f[pos + 1] << 8)) + 256;
                    else if (fcs_len == 4) fcs = rd32(f + pos);
                    else fcs = (uint64_t)rd32(f + pos) | ((uint64_t)rd32(f + pos + 4) << 32);
                    if (fcs != nm) err = 1;
                    pos += fcs_len;
                }
            }
        }
        s_err = err;
        s_pos = pos;
        s_done = 0;
        s_flen = flen;
        s_mode = mode;
    }
    __syncthreads();
    const uint32_t flen = s_flen;
    uint8_t* cwb = (uint8_t*)it.cw;
    // The block headers form a chain (each one gives the next one's
    // position).  The frame is taken in windows of kWin positions: every
    // position gets the position of the block that would follow a header
    // there; pointer jumping inside kChunk-byte chunks turns that into each
    // position's exit from its chunk; one lane then follows the true chain
    // from chunk to chunk (at most kWin / kChunk steps); lanes walk the
    // chunks in parallel to build the block table; all lanes expand it.
    __shared__ uint32_t J[kWin];
    __shared__ uint32_t c_entry[kWinChunks], c_cnt[kWinChunks], c_size[kWinChunks];
    __shared__ uint32_t c_boff[kWinChunks + 1], c_coff[kWinChunks + 1];
    __shared__ uint32_t s_changed;
    const uint8_t* f = rec + 12;
    auto header_next = [&](uint32_t i, uint32_t* size_out, uint32_t* rle_out) -> uint32_t {
        if (i + 3 > flen) return kJInvalid;
        const uint32_t h = (uint32_t)f[i] | ((uint32_t)f[i + 1] << 8) | ((uint32_t)f[i + 2] << 16);
        const uint32_t last = h & 1, type = (h >> 1) & 3, size = h >> 3;
        if (type > 1 || size > kZstdBlockMax) return kJInvalid;
        const uint32_t n = i + 3 + (type ? 1u : size);
        if (size_out) *size_out = size;
        if (rle_out) *rle_out = type;
        if (last) return n == flen ? kJLast : kJInvalid;
        return n < flen ? n : kJInvalid;
    };
    uint32_t wentry = s_pos, content = 0;
    bool fin = false;
    while (!s_err && !fin) {
        const uint32_t ws = wentry, we = min(ws + kWin, flen);
        if (ws >= flen) {  // a header must start here: the chain ran off the frame
            __syncthreads();
            if (tid == 0) s_err = 1;
            __syncthreads();
            break;
        }
        for (uint32_t i = ws + tid; i < we; i += 256) J[i - ws] = header_next(i, nullptr, nullptr);
        __syncthreads();
        // pointer jumping until every position holds its chunk exit
        for (int round = 0; round < 16; ++round) {
            if (tid == 0) s_changed = 0;
            __syncthreads();
            uint32_t ch = 0;
            for (uint32_t i = ws + tid; i < we; i += 256) {
                const uint32_t j = J[i - ws];
                if (j < we && (j - ws) / kChunk == (i - ws) / kChunk) {
                    J[i - ws] = J[j - ws];
                    ch = 1;
                }
            }
            if (ch) s_changed = 1;
            __syncthreads();
            if (!s_changed) break;
        }
        // follow the true chain over the chunks
        for (uint32_t c = tid; c < kWinChunks; c += 256) c_entry[c] = kJInvalid;
        __syncthreads();
        if (tid == 0) {
            uint32_t e = ws, err = 0;
            while (e < we) {
                c_entry[(e - ws) / kChunk] = e;
                e = J[e - ws];
            }
            if (e == kJInvalid) err = 1;
            else if (e == kJLast) s_done = 1;
            else wentry = e;  // first header of the next window
            s_err = err;
            s_pos = e;
        }
        __syncthreads();
        if (s_err) break;
        wentry = s_pos;
        fin = s_done;
        // per-chunk block counts and content sizes
        for (uint32_t c = tid; c < kWinChunks; c += 256) {
            uint32_t cnt = 0, csz = 0;
            const uint32_t cend = ws + (c + 1) * kChunk;
            for (uint32_t pos = c_entry[c]; pos != kJInvalid && pos < cend && pos < we;) {
                uint32_t size = 0, rle = 0;
                const uint32_t n = header_next(pos, &size, &rle);
                cnt++;
                csz += size;
                if (n >= kJLast) break;
                pos = n;
            }
            c_cnt[c] = cnt;
            c_size[c] = csz;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t b = 0, co = content;
            for (uint32_t c = 0; c < kWinChunks; ++c) {
                c_boff[c] = b;
                c_coff[c] = co;
                b += c_cnt[c];
                co += c_size[c];
            }
            c_boff[kWinChunks] = b;
            c_coff[kWinChunks] = co;
            if (co > nm) s_err = 1;
        }
        __syncthreads();
        if (s_err) break;
        // block table (reuses J): tdst[k] content offset, tsrc[k] frame offset | RLE << 31
        uint32_t* tdst = J;
        uint32_t* tsrc = J + kWin / 2;
        const uint32_t nblk = c_boff[kWinChunks];
        for (uint32_t c = tid; c < kWinChunks; c += 256) {
            uint32_t k = c_boff[c], d = c_coff[c];
            const uint32_t cend = ws + (c + 1) * kChunk;
            for (uint32_t pos = c_entry[c]; pos != kJInvalid && pos < cend && pos < we;) {
                uint32_t size = 0, rle = 0;
                const uint32_t n = header_next(pos, &size, &rle);
                tdst[k] = d;
                tsrc[k] = (pos + 3) | (rle << 31);
                k++;
                d += size;
                if (n >= kJLast) break;
                pos = n;
            }
        }
        if (tid == 0) tdst[nblk] = c_coff[kWinChunks];
        __syncthreads();
        if (nblk) {
            const uint32_t d0 = tdst[0], d1 = tdst[nblk];
            for (uint32_t q = (d0 & ~3u) + 4 * tid; q < d1; q += 4 * 256) {
                // block holding byte max(q, d0): largest k with tdst[k] <= it
                const uint32_t first = q < d0 ? d0 : q;
                uint32_t lo = 0, hi = nblk - 1;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (tdst[mid] <= first) lo = mid; else hi = mid - 1;
                }
                uint32_t k = lo, word = 0, full = 1;
                for (uint32_t b = 0; b < 4; ++b) {
                    const uint32_t d = q + b;
                    if (d < d0 || d >= d1) { full = 0; continue; }
                    while (d >= tdst[k + 1]) k++;
                    const uint32_t src = tsrc[k] & 0x7FFFFFFFu;
                    const uint32_t v = (tsrc[k] >> 31) ? f[src] : f[src + (d - tdst[k])];
                    word |= v << (8 * b);
                }
                if (full) *(uint32_t*)(cwb + q) = word;
                else
                    for (uint32_t b = 0; b < 4; ++b)
                        if (q + b >= d0 && q + b < d1) cwb[q + b] = (uint8_t)(word >> (8 * b));
            }
        }
        content = c_coff[kWinChunks];
        __syncthreads();
    }
    if (tid == 0 && !s_err && content != nm) s_err = 1;
    __syncthreads();
    // bytes past the mask content in its last word
    for (uint32_t i = nm + tid; i < it.nwords * 8u; i += 256) cwb[i] = 0;

    // residual section header
    __shared__ uint32_t s_N, s_nb, s_sec;
    if (tid == 0 && !s_err) {
        const uint32_t sec = align4(12 + flen);
        uint32_t err = 0, N = 0, nb = 0;
        if (sec + 4 > L) err = 1;
        else {
            N = rd32(rec + sec);
            if (N > it.npx) err = 1;
            nb = div_up(N, kFrame);
            if (!err && sec + align4(4 + 3 * nb) > L) err = 1;
        }
        s_err = err; s_N = N; s_nb = nb; s_sec = sec;
    }
    __syncthreads();
    if (s_err) {
        if (tid == 0) { plan.res[r].err = 1; atomicOr(plan.err, kErrCorrupt); }
        return;
    }
    const uint32_t sec = s_sec, N = s_N, nb = s_nb;
    const uint8_t* hb = rec + sec + 4;
    uint32_t cp = 0, cn = 0, ch = 0, bad = 0;
    for (uint32_t j0 = 0; j0 < nb; j0 += 256) {
        const uint32_t j = j0 + tid;
        uint32_t pay = 0, pos = 0, high = 0;
        if (j < nb) {
            const uint32_t b = hb[j], n = hb[nb + j], B = hb[2 * nb + j];
            if (B > it.bits || b > B || n > 128 || (n && b == B)) bad = 1;
            pay = 16 * b;
            pos = n;
            high = (n * (B - b) + 7) / 8;
            it.blkinfo[j] = b | (n << 8) | (B << 16);
        }
        uint32_t tp, tn, th;
        const uint32_t op = block_excl_scan<256>(pay, scratch, &tp);
        const uint32_t on = block_excl_scan<256>(pos, scratch, &tn);
        const uint32_t oh = block_excl_scan<256>(high, scratch, &th);
        if (j < nb) {
            it.blkoffs[3 * j] = cp + op;
            it.blkoffs[3 * j + 1] = cn + on;
            it.blkoffs[3 * j + 2] = ch + oh;
        }
        cp += tp; cn += tn; ch += th;
    }
    if (bad) atomicOr(&s_err, 1u);
    __syncthreads();
    if (tid == 0) {
        const uint32_t pay0 = sec + align4(4 + 3 * nb);
        // the record must end exactly after the padded sections
        uint32_t err = s_err;
        if ((uint64_t)pay0 + align4(cp + cn + ch) != L) err = 1;
        DecRes& rs = plan.res[r];
        rs.mode = s_mode;
        rs.flen = flen;
        rs.N = N;
        rs.nb = nb;
        rs.sec = sec;
        rs.pay_off = pay0;
        rs.pos_off = pay0 + cp;
        rs.high_off = pay0 + cp + cn;
        rs.high_end = pay0 + cp + cn + ch;
        rs.err = err;
        plan.modes[r] = (uint8_t)s_mode;
        if (err) atomicOr(plan.err, kErrCorrupt);
    }
}

// ---------------------------------------------------------------------------
// Mask chain over time, one thread per mask word of one attribute; scans are
// taken eight at a time so that their loads overlap.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t* item_words(const DecPlan& plan, uint32_t r, uint32_t off) {
    return (uint64_t*)(plan.ws + plan.item_stride * r + off);
}

__global__ __launch_bounds__(64) void k_dec_mask(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t a = blockIdx.y;
    const uint32_t w = blockIdx.x * 64 + threadIdx.x;
    if (w >= plan.nwords) return;
    const uint64_t tm = tail_mask(w, plan.nwords, plan.npx);
    const uint32_t A = plan.n_attrs, T = plan.n_scans;
    uint64_t mprev = 0;
    bool bad = false;
    for (uint32_t t0 = 0; t0 < T; t0 += 8) {
        uint64_t c[8];
        uint32_t md[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t t = t0 + k;
            c[k] = 0;
            md[k] = 0;
            if (t < T) {
                const uint32_t r = t * A + a;
                c[k] = item_words(plan, r, plan.off_cw)[w];
                md[k] = plan.modes[r];
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t t = t0 + k;
            if (t < T) {
                const uint64_t m = md[k] ? (c[k] ^ mprev) : c[k];
                bad |= (m & ~tm) != 0;  // mask bits past the scan
                item_words(plan, t * A + a, plan.off_vw)[w] = ~m & tm;
                mprev = m;
            }
        }
    }
    if (bad) atomicOr(plan.err, kErrCorrupt);
}

// ---------------------------------------------------------------------------
// Running count of valid samples: N must match the section header; the
// pixel of every frame's last value (where each frame group ends).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_dec_scan(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t r = blockIdx.x;
    const DecItem it = plan.items[r];
    __shared__ uint32_t scratch[20];
    uint32_t carry = 0;
    for (uint32_t w0 = 0; w0 < it.nwords; w0 += 1024) {
        const uint32_t w = w0 + threadIdx.x;
        const uint64_t v = w < it.nwords ? it.vw[w] : 0ull;
        const uint32_t pc = __popcll(v);
        uint32_t total;
        const uint32_t pre = block_excl_scan<1024>(pc, scratch, &total) + carry;
        if (pc) {
            const uint32_t k = pre + ((127u - pre) & 127u);  // first frame end at or after pre
            if (k < pre + pc && (k >> 7) < it.maxnb) it.blklast[k >> 7] = 64u * w + select_bit(v, k - pre);
        }
        carry += total;
    }
    if (threadIdx.x == 0 && carry != plan.res[r].N) atomicOr(plan.err, kErrCorrupt);
}

// ---------------------------------------------------------------------------
// Frame unpacking (Sec. II).  A workgroup stages the packed bytes of a group
// of frames in LDS first: the group's payloads, exception positions and
// exception high parts are three contiguous byte ranges of the record, read
// with coalesced word loads.  One wave then unpacks one frame: the 128
// slots, the exception high parts patched in, inverse ZigZag (Eq. 1).
// Lane l gets the deltas of slots l and l + 64 (0 past the real values).
// ---------------------------------------------------------------------------
constexpr uint32_t kStageWords = 512;  // valid-sample words staged per group (more are read from memory)

struct GroupStage {
    uint32_t info[kGroupFrames];
    uint32_t offs[kGroupFrames + 1][3];  // relative to the group's first frame
    uint32_t base[3];                    // word-aligned start of each staged range in the record
    uint32_t fbase[kGroupFrames];        // running sum before each frame (k_dec_group)
    uint32_t prange[2];                  // first and last pixel of the group (k_dec_group)
    uint64_t vw[kStageWords];            // valid words of the pixel range (k_dec_group)
    uint32_t pay[kGroupFrames * 128 + 2];
    uint32_t pos[kGroupFrames * 32 + 2];
    uint32_t high[kGroupFrames * 128 + 2];
    uint32_t zf[4][128];
};

__device__ __forceinline__ uint32_t bits_at(const uint32_t* w, uint32_t bp, uint32_t width) {
    if (width == 0) return 0;
    const uint64_t v = (uint64_t)w[bp >> 5] | ((uint64_t)w[(bp >> 5) + 1] << 32);
    return (uint32_t)(v >> (bp & 31)) & low_mask32(width);
}

// all threads: metadata of frames [j0, j1) and their packed bytes into S;
// with `scatter` also the frames' running-sum bases, the group's pixel
// range and its valid words.  Independent loads are issued together.
__device__ __forceinline__ void stage_group(const DecItem& it, const DecRes& rs, uint32_t j0, uint32_t j1,
                                            GroupStage& S, bool scatter) {
    const uint32_t tid = threadIdx.x, cnt = j1 - j0;
    if (scatter) {
        if (tid < cnt) S.fbase[tid] = it.bsum[j0 + tid];
        if (tid == 64) S.prange[0] = j0 == 0 ? 0u : it.blklast[j0 - 1] + 1;
        if (tid == 65) S.prange[1] = (j1 >= rs.nb) ? it.npx - 1 : it.blklast[j1 - 1];
    }
    if (tid <= cnt && cnt) {
        const uint32_t j = j0 + tid;
        uint32_t o0, o1, o2;
        if (j < rs.nb) {
            o0 = it.blkoffs[3 * j];
            o1 = it.blkoffs[3 * j + 1];
            o2 = it.blkoffs[3 * j + 2];
        } else {  // end of the sections
            o0 = rs.pos_off - rs.pay_off;
            o1 = rs.high_off - rs.pos_off;
            o2 = rs.high_end - rs.high_off;
        }
        S.offs[tid][0] = o0;
        S.offs[tid][1] = o1;
        S.offs[tid][2] = o2;
        if (tid < cnt) S.info[tid] = it.blkinfo[j];
    }
    __syncthreads();
    if (scatter) {
        const uint32_t v0 = S.prange[0] >> 6, v1 = min((S.prange[1] >> 6) + 1, v0 + kStageWords);
        for (uint32_t w = v0 + tid; w < v1; w += 256) S.vw[w - v0] = it.vw[w];
    }
    if (cnt) {
        const uint32_t starts[3] = {rs.pay_off + S.offs[0][0], rs.pos_off + S.offs[0][1],
                                    rs.high_off + S.offs[0][2]};
        const uint32_t ends[3] = {rs.pay_off + S.offs[cnt][0], rs.pos_off + S.offs[cnt][1],
                                  rs.high_off + S.offs[cnt][2]};
        uint32_t* dst[3] = {S.pay, S.pos, S.high};
        const uint32_t cap[3] = {kGroupFrames * 128 + 2, kGroupFrames * 32 + 2, kGroupFrames * 128 + 2};
        const uint32_t* recw = (const uint32_t*)it.rec;  // records are 4-byte aligned
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const uint32_t w0 = starts[q] >> 2, w1 = (ends[q] + 3) >> 2;
            for (uint32_t w = w0 + tid; w < w1 && w - w0 < cap[q]; w += 256) dst[q][w - w0] = recw[w];
            if (tid == 0) S.base[q] = w0 * 4;
        }
    }
    __syncthreads();
}

// one wave: frame k of the staged group
__device__ __forceinline__ void unpack_staged(const DecPlan& plan, const DecItem& it, const DecRes& rs,
                                              GroupStage& S, uint32_t j0, uint32_t k, uint32_t wave, uint32_t& d0,
                                              uint32_t& d1) {
    const uint32_t l = lane_id();
    const uint32_t j = j0 + k;
    const uint32_t info = S.info[k];
    const uint32_t b = info & 0xFF, n = (info >> 8) & 0xFF, B = (info >> 16) & 0xFF;
    const uint32_t hwid = B - b;
    const uint32_t real = min(kFrame, rs.N - j * kFrame);
    const uint32_t pw0 = (rs.pay_off + S.offs[k][0] - S.base[0]) >> 2;  // payloads are word aligned
    const uint8_t* posb = (const uint8_t*)S.pos + (rs.pos_off + S.offs[k][1] - S.base[1]);
    const uint32_t hbit0 = 8 * (rs.high_off + S.offs[k][2] - S.base[2]);
    uint32_t* zf = S.zf[wave];
    zf[l] = bits_at(S.pay + pw0, l * b, b);
    zf[l + 64] = bits_at(S.pay + pw0, (l + 64) * b, b);
    __builtin_amdgcn_wave_barrier();
    for (uint32_t e = l; e < n; e += 64) {
        const uint32_t p = posb[e];
        const bool ok = p < real && (e == 0 || posb[e - 1] < p);
        if (!ok) { atomicOr(plan.err, kErrCorrupt); continue; }
        zf[p] |= bits_at(S.high, hbit0 + e * hwid, hwid) << b;
    }
    __builtin_amdgcn_wave_barrier();
    d0 = l < real ? unzigzag(zf[l], it.bits) : 0u;
    d1 = l + 64 < real ? unzigzag(zf[l + 64], it.bits) : 0u;
    __builtin_amdgcn_wave_barrier();
}

// per-frame sums of the deltas (mod 2^w)
__global__ __launch_bounds__(256) void k_dec_fsum(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t r = blockIdx.y;
    const DecItem it = plan.items[r];
    const DecRes rs = plan.res[r];
    const uint32_t j0 = blockIdx.x * kGroupFrames;
    if (j0 >= rs.nb) return;
    const uint32_t j1 = min(j0 + kGroupFrames, rs.nb);
    __shared__ GroupStage S;
    stage_group(it, rs, j0, j1, S, false);
    const uint32_t wave = threadIdx.x / kWave;
    for (uint32_t k = wave; k < j1 - j0; k += 4) {
        uint32_t d0, d1;
        unpack_staged(plan, it, rs, S, j0, k, wave, d0, d1);
        const uint32_t s = wave_sum(d0 + d1);
        if (lane_id() == 0) it.bsum[j0 + k] = s & low_mask32(it.bits);
    }
}

// exclusive running sum over the frames (mod 2^w): each frame's base value
__global__ __launch_bounds__(1024) void k_dec_bscan(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t r = blockIdx.x;
    const DecItem it = plan.items[r];
    const uint32_t nb = plan.res[r].nb;
    const uint32_t m = low_mask32(it.bits);
    __shared__ uint32_t scratch[20];
    uint32_t carry = 0;
    for (uint32_t j0 = 0; j0 < nb; j0 += 1024) {
        const uint32_t j = j0 + threadIdx.x;
        const uint32_t v = j < nb ? it.bsum[j] : 0u;
        uint32_t total;
        const uint32_t pre = block_excl_scan<1024>(v, scratch, &total) + carry;
        if (j < nb) it.bsum[j] = pre & m;
        carry += total;
    }
}

// ---------------------------------------------------------------------------
// One workgroup per group of kGroupFrames frames: the frames' running sums
// (undoing the delta, Sec. III-C) go to LDS, then the group's pixel range is
// written: the k-th valid pixel gets value k, the others zero.  The ranges
// of consecutive groups tile the scan.  For a P-scan the value is the
// difference to the previous scan (added by k_dec_temporal); for P > 1 the
// quantized value (restored there too).
// ---------------------------------------------------------------------------
template <int WB>
__device__ __forceinline__ void dec_group_scatter(const DecItem& it, const GroupStage& S, const uint32_t* sv,
                                                  uint32_t* scratch) {
    using T = typename SampleT<WB>::T;
    T* out = (T*)it.out;
    const uint32_t p_lo = S.prange[0], p_hi = S.prange[1];
    const uint32_t v0 = p_lo >> 6;
    uint32_t cnt = 0;
    for (uint32_t c0 = p_lo & ~15u; c0 <= p_hi; c0 += 256 * 16) {
        const uint32_t p0 = c0 + threadIdx.x * 16;
        uint32_t bits16 = 0, inr = 0;
        if (p0 <= p_hi && p0 + 15 >= p_lo && p0 < it.npx) {
            const uint32_t w = p0 >> 6;
            const uint64_t v = (w - v0 < kStageWords) ? S.vw[w - v0] : it.vw[w];
            bits16 = (uint32_t)(v >> (16 * ((p0 >> 4) & 3))) & 0xFFFFu;
            const uint32_t lo = p0 < p_lo ? p_lo - p0 : 0u;
            const uint32_t hi = p_hi - p0 >= 15 ? 15u : p_hi - p0;
            inr = ((0xFFFFu >> (15 - hi)) >> lo) << lo;  // pixels p0+lo .. p0+hi
            bits16 &= inr;
        }
        uint32_t total;
        uint32_t k = block_excl_scan<256>(__popc(bits16), scratch, &total) + cnt;
        uint32_t vals[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            uint32_t val = 0;
            if (bits16 & (1u << i)) val = sv[k++];
            vals[i] = val;
        }
        if (inr == 0xFFFFu && it.aligned16) {
            store16<WB>(it.out, p0, it.npx, true, vals);
        } else if (inr) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (inr & (1u << i)) out[p0 + i] = (T)vals[i];
        }
        cnt += total;
    }
}

__global__ __launch_bounds__(256) void k_dec_group(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t r = blockIdx.y;
    const DecItem it = plan.items[r];
    const DecRes rs = plan.res[r];
    const uint32_t g = blockIdx.x;
    const uint32_t j0 = g * kGroupFrames;
    if (j0 >= rs.nb && !(g == 0 && rs.nb == 0)) return;
    const uint32_t j1 = min(j0 + kGroupFrames, rs.nb);
    __shared__ GroupStage S;
    __shared__ uint32_t sv[kGroupFrames * kFrame];
    __shared__ uint32_t scratch[8];
    const uint32_t wave = threadIdx.x / kWave, l = lane_id();
    const uint32_t m = low_mask32(it.bits);
    stage_group(it, rs, j0, j1, S, true);
    for (uint32_t k = wave; k < j1 - j0; k += 4) {
        uint32_t d0, d1;
        unpack_staged(plan, it, rs, S, j0, k, wave, d0, d1);
        const uint32_t a0 = wave_incl_scan(d0) + S.fbase[k];
        const uint32_t t0 = (uint32_t)__shfl((int)a0, 63, kWave);
        const uint32_t a1 = wave_incl_scan(d1) + t0;
        uint32_t* dst = sv + k * kFrame;
        dst[l] = a0 & m;
        dst[l + 64] = a1 & m;
    }
    __syncthreads();
    switch (it.wb) {
        case 4: dec_group_scatter<4>(it, S, sv, scratch); break;
        case 2: dec_group_scatter<2>(it, S, sv, scratch); break;
        default: dec_group_scatter<1>(it, S, sv, scratch); break;
    }
}

// ---------------------------------------------------------------------------
// Over time, per pixel: a P-scan adds the previous decoded scan at its valid
// pixels (Sec. III-D); then q * P, saturated to the sample width.  The
// attribute's modes are staged in LDS; a scan is read only when it is a
// P-scan, precedes one, or has P > 1.
// ---------------------------------------------------------------------------
constexpr uint32_t kModeLds = 8192;

template <int WB>
__device__ __forceinline__ void dec_temporal_body(const DecPlan& plan, uint32_t a, uint32_t p0, const uint8_t* md) {
    uint32_t qprev[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) qprev[i] = 0;
    const uint32_t A = plan.n_attrs, T = plan.n_scans;
    const uint32_t P = plan.attr_P[a], bits = 8 * WB, m = low_mask32(bits);
    const uint64_t stride = (uint64_t)plan.npx * WB;
    const bool al = ((uintptr_t)plan.out_base[a] % 16 == 0) && (stride % 16 == 0);
    auto mode_of = [&](uint32_t t) -> uint32_t { return t < kModeLds ? md[t] : plan.modes[t * A + a]; };
    for (uint32_t t = 0; t < T; ++t) {
        const uint32_t mode = mode_of(t);
        const bool next_p = (t + 1 < T) && mode_of(t + 1) == 1;
        if (mode == 0 && P == 1 && !next_p) continue;
        void* out = (uint8_t*)plan.out_base[a] + stride * t;
        uint32_t v[16];
        load16<WB>(out, p0, plan.npx, al, v);
        if (mode == 1) {
            const uint64_t vw = item_words(plan, t * A + a, plan.off_vw)[p0 >> 6];
            const uint32_t bits16 = (uint32_t)(vw >> (16 * ((p0 >> 4) & 3))) & 0xFFFFu;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t q = (bits16 & (1u << i)) ? ((v[i] + qprev[i]) & m) : 0u;
                qprev[i] = q;
                v[i] = dequantize(q, P, bits);
            }
            store16<WB>(out, p0, plan.npx, al, v);
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                qprev[i] = v[i];
                v[i] = dequantize(v[i], P, bits);
            }
            if (P > 1) store16<WB>(out, p0, plan.npx, al, v);
        }
    }
}

__global__ __launch_bounds__(256) void k_dec_temporal(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t a = blockIdx.y;
    __shared__ uint8_t md[kModeLds];
    const uint32_t A = plan.n_attrs;
    for (uint32_t t = threadIdx.x; t < plan.n_scans && t < kModeLds; t += 256) md[t] = plan.modes[t * A + a];
    __syncthreads();
    const uint32_t p0 = (blockIdx.x * 256 + threadIdx.x) * 16;
    if (p0 >= plan.npx) return;
    switch (plan.attr_wb[a]) {
        case 4: dec_temporal_body<4>(plan, a, p0, md); break;
        case 2: dec_temporal_body<2>(plan, a, p0, md); break;
        default: dec_temporal_body<1>(plan, a, p0, md); break;
    }
}

hipError_t launch_decode(const DecPlan& plan, hipStream_t stream) {
    if (plan.n_items == 0) return hipSuccess;
    JIFFY_LAUNCH("k_dec_parse", k_dec_parse, dim3(plan.n_items), dim3(256), stream, plan);
    JIFFY_LAUNCH("k_dec_mask", k_dec_mask, dim3(div_up(plan.nwords, 64), plan.n_attrs), dim3(64), stream, plan);
    JIFFY_LAUNCH("k_dec_scan", k_dec_scan, dim3(plan.n_items), dim3(1024), stream, plan);
    JIFFY_LAUNCH("k_dec_fsum", k_dec_fsum, dim3(plan.max_groups, plan.n_items), dim3(256), stream, plan);
    JIFFY_LAUNCH("k_dec_bscan", k_dec_bscan, dim3(plan.n_items), dim3(1024), stream, plan);
    JIFFY_LAUNCH("k_dec_group", k_dec_group, dim3(plan.max_groups, plan.n_items), dim3(256), stream, plan);
    if (plan.need_temporal)
        JIFFY_LAUNCH("k_dec_temporal", k_dec_temporal, dim3(div_up(plan.npx, 256 * 16), plan.n_attrs), dim3(256),
                     stream, plan);
    return hipGetLastError();
}

}  // namespace jiffy
