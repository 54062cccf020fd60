// Jiffy decoder kernels for gfx950.  Decoding reverses each encoding step
// (Sec. III-C: "a straightforward reversal"):
//
//   k_dec_parse    record header, mask frame (Raw/RLE Zstandard blocks) to mask
//                  bytes, residual-section header and its frame offsets
//   k_dec_mask     mask chain over time: a P-scan's mask is its content XOR
//                  the previous mask (Sec. III-D); valid-sample words
//   k_dec_scan     running count of valid samples (where each value lands)
//   k_dec_frames   bit unpacking, exception patching (Sec. II), inverse
//                  ZigZag (Eq. 1), running sum inside each frame
//   k_dec_bscan    running sum over frames (undoes the delta, Sec. III-C)
//   k_dec_scatter  values back to their pixels, zeros elsewhere
//   k_dec_temporal adds the previous scan for P-scans (Sec. III-D) and
//                  restores the original representation, q * P (Sec. III-A)
//
// Every offset read from the stream is checked before it is used; a
// malformed stream raises kErrCorrupt and later kernels do nothing.
#include "jiffy_device.h"

namespace jiffy {

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
    __shared__ uint32_t s_err, s_pos, s_got, s_done, s_nblk, s_flen, s_mode;
    __shared__ uint32_t bsrc[256], bdst[256], bsz[256];
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
        s_got = 0;
        s_done = 0;
        s_flen = flen;
        s_mode = mode;
    }
    __syncthreads();
    const uint32_t flen = s_flen;
    uint8_t* cwb = (uint8_t*)it.cw;
    // block walk (one lane) and expansion (all lanes), 256 blocks per round
    while (!s_err && !s_done) {
        if (tid == 0) {
            const uint8_t* f = rec + 12;
            uint32_t pos = s_pos, got = s_got, nblk = 0, err = 0, done = 0;
            while (nblk < 256) {
                if (pos + 3 > flen) { err = 1; break; }
                const uint32_t h = f[pos] | (f[pos + 1] << 8) | (f[pos + 2] << 16);
                const uint32_t last = h & 1, type = (h >> 1) & 3, size = h >> 3;
                if (size > kZstdBlockMax || got + size > nm) { err = 1; break; }
                if (type == 0) {
                    if (pos + 3 + size > flen) { err = 1; break; }
                    bsz[nblk] = size;
                    pos += 3 + size;
                } else if (type == 1) {
                    if (pos + 4 > flen) { err = 1; break; }
                    bsz[nblk] = size | 0x80000000u;
                    pos += 4;
                } else { err = 1; break; }
                bsrc[nblk] = 12 + (pos - (type == 0 ? size : 1));
                bdst[nblk] = got;
                got += size;
                nblk++;
                if (last) { done = 1; break; }
            }
            if (done && (got != nm || pos != flen)) err = 1;
            s_pos = pos; s_got = got; s_nblk = nblk; s_err = err; s_done = done;
        }
        __syncthreads();
        if (s_err) break;
        const uint32_t nblk = s_nblk;
        for (uint32_t k = 0; k < nblk; ++k) {
            const uint32_t sz = bsz[k] & 0x7FFFFFFFu, rle = bsz[k] >> 31;
            const uint8_t* src = rec + bsrc[k];
            uint8_t* dst = cwb + bdst[k];
            if (rle) {
                const uint8_t b = src[0];
                for (uint32_t i = tid; i < sz; i += 256) dst[i] = b;
            } else {
                for (uint32_t i = tid; i < sz; i += 256) dst[i] = src[i];
            }
        }
        __syncthreads();
    }
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
        rs.err = err;
        if (err) atomicOr(plan.err, kErrCorrupt);
    }
}

// ---------------------------------------------------------------------------
// Mask chain over time, one thread per mask word of one attribute.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_dec_mask(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t a = blockIdx.y;
    const uint32_t w = blockIdx.x * 64 + threadIdx.x;
    if (w >= plan.nwords) return;
    const uint64_t tm = tail_mask(w, plan.nwords, plan.npx);
    uint64_t mprev = 0;
    for (uint32_t t = 0; t < plan.n_scans; ++t) {
        const uint32_t r = t * plan.n_attrs + a;
        const DecItem& it = plan.items[r];
        const uint64_t c = it.cw[w];
        const uint64_t m = plan.res[r].mode ? (c ^ mprev) : c;
        if (m & ~tm) atomicOr(plan.err, kErrCorrupt);  // mask bits past the scan
        it.vw[w] = ~m & tm;
        mprev = m;
    }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_dec_scan(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t r = blockIdx.x;
    const DecItem it = plan.items[r];
    __shared__ uint32_t scratch[20];
    uint32_t carry = 0;
    for (uint32_t w0 = 0; w0 < it.nwords; w0 += 1024) {
        const uint32_t w = w0 + threadIdx.x;
        const uint32_t pc = w < it.nwords ? __popcll(it.vw[w]) : 0u;
        uint32_t total;
        const uint32_t pre = block_excl_scan<1024>(pc, scratch, &total) + carry;
        if (w < it.nwords) it.wpre[w] = pre;
        carry += total;
    }
    if (threadIdx.x == 0 && carry != plan.res[r].N) atomicOr(plan.err, kErrCorrupt);
}

// ---------------------------------------------------------------------------
// Frame unpacking.  One wave per frame: payload words and exception bytes to
// LDS, values of 128 slots, exception high parts patched in, inverse ZigZag,
// running sum inside the frame.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bits_at(const uint32_t* w, uint32_t bp, uint32_t width) {
    if (width == 0) return 0;
    const uint64_t v = (uint64_t)w[bp >> 5] | ((uint64_t)w[(bp >> 5) + 1] << 32);
    return (uint32_t)(v >> (bp & 31)) & low_mask32(width);
}

__global__ __launch_bounds__(256) void k_dec_frames(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t r = blockIdx.y;
    const DecItem it = plan.items[r];
    const DecRes rs = plan.res[r];
    const uint32_t j0 = blockIdx.x * kGroupFrames;
    if (j0 >= rs.nb) return;
    const uint32_t j1 = min(j0 + kGroupFrames, rs.nb);
    __shared__ uint32_t pw[4][130];
    __shared__ uint32_t hwb[4][132];
    __shared__ uint32_t zf[4][128];
    const uint32_t wave = threadIdx.x / kWave, l = lane_id();
    const uint32_t m = low_mask32(it.bits);
    for (uint32_t j = j0 + wave; j < j1; j += 4) {
        const uint32_t info = it.blkinfo[j];
        const uint32_t b = info & 0xFF, n = (info >> 8) & 0xFF, B = (info >> 16) & 0xFF;
        const uint32_t hwid = B - b;
        const uint32_t hb = (n * hwid + 7) / 8;
        const uint32_t real = min(kFrame, rs.N - j * kFrame);
        const uint32_t* payw = (const uint32_t*)(it.rec + rs.pay_off + it.blkoffs[3 * j]);
        const uint8_t* posp = it.rec + rs.pos_off + it.blkoffs[3 * j + 1];
        const uint8_t* highp = it.rec + rs.high_off + it.blkoffs[3 * j + 2];
        pw[wave][l] = l < 4 * b ? payw[l] : 0u;
        pw[wave][l + 64] = l + 64 < 4 * b ? payw[l + 64] : 0u;
        if (l < 2) pw[wave][128 + l] = 0;
        // high-part bytes as little-endian words
        for (uint32_t k = l; k < 132; k += 64) {
            uint32_t v = 0;
            for (uint32_t q = 0; q < 4; ++q) {
                const uint32_t bi = 4 * k + q;
                if (bi < hb) v |= (uint32_t)highp[bi] << (8 * q);
            }
            hwb[wave][k] = v;
        }
        __builtin_amdgcn_wave_barrier();
        zf[wave][l] = bits_at(pw[wave], l * b, b);
        zf[wave][l + 64] = bits_at(pw[wave], (l + 64) * b, b);
        __builtin_amdgcn_wave_barrier();
        // exceptions: ascending positions inside the frame's real values
        for (uint32_t k = l; k < n; k += 64) {
            const uint32_t p = posp[k];
            const bool ok = p < real && (k == 0 || posp[k - 1] < p);
            if (!ok) { atomicOr(plan.err, kErrCorrupt); continue; }
            zf[wave][p] |= bits_at(hwb[wave], k * hwid, hwid) << b;
        }
        __builtin_amdgcn_wave_barrier();
        const uint32_t d0 = l < real ? unzigzag(zf[wave][l], it.bits) : 0u;
        const uint32_t d1 = l + 64 < real ? unzigzag(zf[wave][l + 64], it.bits) : 0u;
        const uint32_t a0 = wave_incl_scan(d0);
        const uint32_t t0 = (uint32_t)__shfl((int)a0, 63, kWave);
        const uint32_t a1 = wave_incl_scan(d1) + t0;
        uint32_t* sb = it.sbuf + j * kFrame;
        if (l < real) sb[l] = a0 & m;
        if (l + 64 < real) sb[l + 64] = a1 & m;
        if (l == 63) it.bsum[j] = a1 & m;
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
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
// Scatter: value k of the flattened vector goes to the k-th valid pixel.
// ---------------------------------------------------------------------------
template <int WB>
__device__ __forceinline__ void dec_scatter_body(const DecPlan& plan, const DecItem& it, uint32_t mode, uint32_t p0) {
    const uint32_t w = p0 >> 6, q4 = (p0 >> 4) & 3;
    const uint64_t v = it.vw[w];
    const uint32_t bits16 = (uint32_t)(v >> (16 * q4)) & 0xFFFFu;
    uint32_t k = it.wpre[w] + __popcll(v & ((1ull << (16 * q4)) - 1ull));
    const uint32_t m = low_mask32(it.bits);
    uint32_t out[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        uint32_t val = 0;
        if (bits16 & (1u << i)) {
            val = (it.sbuf[k] + it.bsum[k >> 7]) & m;
            k++;
        }
        out[i] = val;
    }
    store16<WB>(it.out, p0, it.npx, it.aligned16, out);
    (void)plan;
    (void)mode;
}

__global__ __launch_bounds__(256) void k_dec_scatter(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t r = blockIdx.y;
    const DecItem it = plan.items[r];
    const uint32_t p0 = blockIdx.x * kTilePx + threadIdx.x * 16;
    if (p0 >= it.npx) return;
    const uint32_t mode = plan.res[r].mode;
    switch (it.wb) {
        case 4: dec_scatter_body<4>(plan, it, mode, p0); break;
        case 2: dec_scatter_body<2>(plan, it, mode, p0); break;
        default: dec_scatter_body<1>(plan, it, mode, p0); break;
    }
}

// ---------------------------------------------------------------------------
// Over time, per pixel: a P-scan adds the previous decoded scan at its valid
// pixels (Sec. III-D); then q * P, saturated to the sample width.
// ---------------------------------------------------------------------------
template <int WB>
__device__ __forceinline__ void dec_temporal_body(const DecPlan& plan, uint32_t a, uint32_t p0) {
    uint32_t qprev[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) qprev[i] = 0;
    const uint32_t A = plan.n_attrs, T = plan.n_scans;
    for (uint32_t t = 0; t < T; ++t) {
        const uint32_t r = t * A + a;
        const DecItem& it = plan.items[r];
        const uint32_t mode = plan.res[r].mode;
        const uint32_t P = it.P, bits = it.bits, m = low_mask32(bits);
        const bool next_p = (t + 1 < T) && plan.res[r + A].mode == 1;
        uint32_t v[16];
        if (mode == 1) {
            load16<WB>(it.out, p0, it.npx, it.aligned16, v);
            const uint64_t vw = it.vw[p0 >> 6];
            const uint32_t bits16 = (uint32_t)(vw >> (16 * ((p0 >> 4) & 3))) & 0xFFFFu;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t q = (bits16 & (1u << i)) ? ((v[i] + qprev[i]) & m) : 0u;
                qprev[i] = q;
                v[i] = dequantize(q, P, bits);
            }
            store16<WB>(it.out, p0, it.npx, it.aligned16, v);
        } else if (P > 1 || next_p) {
            load16<WB>(it.out, p0, it.npx, it.aligned16, v);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                qprev[i] = v[i];
                v[i] = dequantize(v[i], P, bits);
            }
            if (P > 1) store16<WB>(it.out, p0, it.npx, it.aligned16, v);
        }
    }
}

__global__ __launch_bounds__(256) void k_dec_temporal(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t a = blockIdx.y;
    const uint32_t p0 = (blockIdx.x * 256 + threadIdx.x) * 16;
    if (p0 >= plan.npx) return;
    switch (plan.items[a].wb) {
        case 4: dec_temporal_body<4>(plan, a, p0); break;
        case 2: dec_temporal_body<2>(plan, a, p0); break;
        default: dec_temporal_body<1>(plan, a, p0); break;
    }
}

hipError_t launch_decode(const DecPlan& plan, hipStream_t stream) {
    if (plan.n_items == 0) return hipSuccess;
    JIFFY_LAUNCH("k_dec_parse", k_dec_parse, dim3(plan.n_items), dim3(256), stream, plan);
    JIFFY_LAUNCH("k_dec_mask", k_dec_mask, dim3(div_up(plan.nwords, 64), plan.n_attrs), dim3(64), stream, plan);
    JIFFY_LAUNCH("k_dec_scan", k_dec_scan, dim3(plan.n_items), dim3(1024), stream, plan);
    JIFFY_LAUNCH("k_dec_frames", k_dec_frames, dim3(plan.max_groups, plan.n_items), dim3(256), stream, plan);
    JIFFY_LAUNCH("k_dec_bscan", k_dec_bscan, dim3(plan.n_items), dim3(1024), stream, plan);
    JIFFY_LAUNCH("k_dec_scatter", k_dec_scatter, dim3(plan.n_tiles, plan.n_items), dim3(256), stream, plan);
    if (plan.need_temporal)
        JIFFY_LAUNCH("k_dec_temporal", k_dec_temporal, dim3(div_up(plan.npx, 256 * 16), plan.n_attrs), dim3(256),
                     stream, plan);
    return hipGetLastError();
}

}  // namespace jiffy
