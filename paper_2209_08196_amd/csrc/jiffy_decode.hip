// Jiffy decoder kernels for gfx950.  Decoding reverses each encoding step
// (Sec. III-C: "a straightforward reversal"):
//
//   k_dec_parse    record header, mask frame (Raw/RLE Zstandard blocks) to mask
//                  bytes, residual-section header and its frame offsets
//   k_dec_mask     mask chain over time: a P-scan's mask is its content XOR
//                  the previous mask (Sec. III-D); valid-sample words
//   k_dec_scan     running count of valid samples before every tile
//   k_dec_tiles    bit unpacking, exception patching (Sec. II), inverse
//                  ZigZag (Eq. 1), running sum (undoes the delta, Sec.
//                  III-C) chained across tiles, values back to their
//                  pixels, zeros elsewhere
//   k_dec_temporal adds the previous scan for P-scans (Sec. III-D) and
//                  restores the original representation, q * P (Sec. III-A)
//   k_dec_report   the error words to host-mapped memory
//
// Every offset read from the stream is checked before it is used; a
// malformed stream raises kErrCorrupt and later kernels do nothing.
#define JIFFY_KERNEL_TU 1
#include <type_traits>

#include "jiffy_device.h"

namespace jiffy {

constexpr uint32_t kWin = 8192;             // frame positions per parsing window
constexpr uint32_t kChunk = 128;            // bytes per chunk of the chain stitching
constexpr uint32_t kWinChunks = kWin / kChunk;
constexpr uint32_t kJInvalid = 0xFFFFFFFEu; // no valid block chain continues here
constexpr uint32_t kJLast = 0xFFFFFFFDu;    // a last block that ends the frame exactly
constexpr uint32_t kSpinMax = 1u << 16;     // polls of a workgroup waiting on another before giving up

__device__ __forceinline__ uint32_t rd32(const uint8_t* p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

// ---------------------------------------------------------------------------
// Record parse.  blockIdx.y < pwin: the record header and one 8 KiB window
// of the mask frame (Raw and RLE blocks) into mask bytes; blockIdx.y = pwin:
// the residual section header into per-frame widths and section offsets.
// The two parts of a record are independent (the section starts after the
// mask frame, whose length is in the record header).
// ---------------------------------------------------------------------------
constexpr uint32_t kSeg = 32;                      // bytes per thread segment of a window
constexpr uint32_t kSegs = kWin / kSeg;            // 256: one per thread
constexpr uint16_t kXOut = 0xFFFFu;                // the chain leaves the window (a valid position)
constexpr uint16_t kXBad = 0xFFFEu;                // no valid block header here
constexpr uint16_t kXLast = 0xFFFDu;               // the last block; it ends the frame exactly
static_assert((kJInvalid & 0xFFFFu) == kXBad && (kJLast & 0xFFFFu) == kXLast && kJLast < kJInvalid,
              "a step's mark keeps its low half as the window mark");
static_assert(kWin <= 0xFFF0u && kSegs == 256, "window offsets fit 16 bits; one segment per thread");
static_assert(kWin == kParseWin, "the host sizes the parse grid with the same window");
static_assert(kChunk % kSeg == 0 && kWinChunks <= kSegs && (kChunk & (kChunk - 1)) == 0,
              "a chunk is a power of two of whole segments; a lane per chunk");

__device__ __forceinline__ uint32_t sx(uint32_t i) { return i + ((i >> 5) << 1); }

// The step a block header h (its three bytes, little-endian) at frame offset
// i takes: the next header's offset; kJLast for a last block that ends the
// frame exactly; kJInvalid for no block (type 2 or 3, a size above the
// format's maximum, no room for the header, or a block that runs past the
// frame or, being last, stops short of its end).  Type 1 (RLE) takes one
// content byte.  No branches: every byte of a window is tried.
constexpr uint32_t kHdrLim = (kZstdBlockMax + 1) << 3;  // headers with a size in range lie below
__device__ __forceinline__ uint32_t block_next(uint32_t h, uint32_t i, uint32_t flen) {
    const uint32_t last = h & 1u;
    const uint32_t n = i + 3 + ((h & 2u) ? 1u : (h >> 3));
    const bool ok = ((h & 4u) == 0) & (h < kHdrLim) & (i + 3 <= flen) & (last ? n == flen : n < flen);
    return !ok ? kJInvalid : last ? kJLast : n;
}

struct ParseLds {
    union {
        // per position, indexed through sx() (one pad entry pair per 32
        // positions keeps segments in distinct banks): first the chain
        // position at or after its segment's end, after the jumping rounds
        // the one at or after its chunk's end
        uint16_t Y[kWin + kWin / 16];
        struct {  // a block takes 3 bytes at least
            uint32_t dst[kWin / 3 + 2];  // block k: content offset of its first byte (and the end)
            uint16_t src[kWin / 3 + 1];  // block k: window offset of its content | RLE << 15
        } t;
    } u;
    uint32_t fwin[kWin / 4 + 2];  // the window's frame bytes (and the two after it)
    uint16_t seg_entry[kSegs];    // first chain position in each segment (window offset), or kXBad
    uint16_t c_entry[kWinChunks];
    uint32_t scratch[8];
    uint32_t s_err, s_done, s_next, s_pos, s_flen, s_nblk;
};

// Window states of a record's mask-frame parse: bit 63 published, bit 62
// an error before it, bit 61 the frame ended before it; else the first block
// header at or after the window's start (bits 0..31, a frame offset) and the
// content bytes before it (bits 32..60).
constexpr uint64_t kPsPub = 1ull << 63, kPsErr = 1ull << 62, kPsDone = 1ull << 61;

__device__ __forceinline__ JG uint64_t* parse_states(const DecPlan& plan, uint32_t r) {
    return (JG uint64_t*)(plan.ws + plan.item_stride * r + plan.off_pstate);
}

// Record header and mask frame.  The frame's blocks start at offset P0 (after
// the frame header); window w covers frame offsets [P0 + w kWin, P0 + (w+1) kWin)
// and is parsed by its own workgroup (windows numbered in arrival order, so a
// window's predecessors have all started).  Each builds its jump tables
// independently, then waits for the state its predecessor publishes (where
// the block chain enters the window and how much content came before),
// follows the chain through the window, publishes the state for the next
// window, and only then lists and expands its blocks.
__device__ void parse_mask(const DecPlan& plan, uint32_t r, const DecItem& it, ParseLds& P) {
    const uint8_t* rec = it.rec;
    const uint32_t L = it.rec_len;
    const uint32_t nm = div_up(it.npx, 8);
    const uint32_t tid = threadIdx.x;
    JG uint64_t* pst = parse_states(plan, r);
    __shared__ uint32_t s_win;
    __shared__ uint64_t s_state;
    if (tid == 0) {
        // the window's ticket, and with it (no wait in between) the record
        // header and the frame header through its content size,
        // record bytes 0..27, in one round of word loads (a record is 4-byte
        // aligned, at least 12 bytes and a whole number of words long; a word
        // past its end reads its last word again, and every byte taken from
        // one is ruled out by the length checks first)
        const uint32_t win = atomicAdd((JG uint32_t*)(pst + plan.pwin + 1), 1u);
        const uint32_t* rw = (const uint32_t*)rec;
        const uint32_t lw = L / 4 - 1;
        uint32_t hw[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) hw[k] = rw[min((uint32_t)k, lw)];
        s_win = win;
        auto byte = [&](uint32_t i) -> uint32_t { return (hw[i >> 2] >> (8 * (i & 3))) & 0xFFu; };
        uint32_t err = 0;
        const uint32_t mode = byte(4), attr = byte(5);
        const uint32_t resv = hw[1] >> 16;
        const uint32_t flen = hw[2];
        // the record's own length must repeat the length the index gave it
        if (hw[0] != L || mode > 1 || attr != it.attr || resv != 0 || flen > L - 12) err = 1;
        if (mode == 1 && it.t == 0) err = 1;  // nothing to predict from
        uint32_t pos = 0;
        if (!err) {  // the frame starts at record byte 12
            if (flen < 6 || hw[3] != 0xFD2FB528u) err = 1;
            else {
                const uint32_t fhd = byte(16);
                const uint32_t fcs_flag = fhd >> 6, single = (fhd >> 5) & 1;
                const uint32_t reserved = (fhd >> 3) & 1, checksum = (fhd >> 2) & 1, dict = fhd & 3;
                if (!single || reserved || checksum || dict) err = 1;
                const uint32_t fcs_len = fcs_flag == 0 ? 1 : fcs_flag == 1 ? 2 : fcs_flag == 2 ? 4 : 8;
                pos = 5;
                if (!err && pos + fcs_len > flen) err = 1;
                if (!err) {
                    uint64_t fcs = 0;  // little-endian, frame bytes 5 .. 5 + fcs_len (record bytes 17 ..)
#pragma unroll
                    for (uint32_t k = 0; k < 8; ++k)
                        if (k < fcs_len) fcs |= (uint64_t)byte(17 + k) << (8 * k);
                    if (fcs_len == 2) fcs += 256;
                    if (fcs != nm) err = 1;
                    pos += fcs_len;
                }
            }
        }
        if (!err && pos + 3 > flen) err = 1;  // no room for a block
        P.s_err = err;
        P.s_pos = pos;
        P.s_done = 0;
        P.s_flen = flen;
        if (win == 0) {
            plan.res[r].mode = mode;
            plan.res[r].flen = flen;
            plan.modes[r] = (uint8_t)mode;
        }
    }
    __syncthreads();
    const uint32_t win = s_win;
    const uint32_t flen = P.s_flen;
    const uint8_t* f = rec + 12;
    const uint8_t* fb = (const uint8_t*)P.fwin;
    uint8_t* cwb = (uint8_t*)it.cw;
    if (win == 0)  // bytes past the mask content in its last word
        for (uint32_t i = nm + tid; i < it.nwords * 8u; i += 256) cwb[i] = 0;
    if (P.s_err) {  // every window sees the header; the first reports it
        if (win == 0 && tid == 0) atomicOr(plan.err, kErrCorrupt);
        return;
    }
    const uint32_t P0 = P.s_pos;
    const uint32_t nwin = div_up(flen - P0, kWin);
    if (nwin > plan.pwin) {  // longer than any frame of this many pixels
        if (win == 0 && tid == 0) atomicOr(plan.err, kErrCorrupt);
        return;
    }
    if (win >= nwin) return;  // the frame is shorter than the most windows a record can have
    const uint32_t ws = P0 + win * kWin, we = min(ws + kWin, flen);
    // publishes the state for the next window (if the frame reaches it)
    auto publish = [&](uint64_t st) {
        if (win + 1 < nwin) __hip_atomic_store(pst + win + 1, kPsPub | st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // The block headers form a chain: each one gives the position of the
    // next.  Every thread owns a 32-byte segment of the window: walking it
    // backwards it finds, for each position, where a chain through that
    // position leaves the segment; a few rounds of pointer jumping turn that
    // into where it leaves the chunk (kChunk bytes).  One lane then follows
    // the true chain from chunk to chunk, a lane per chunk block by block
    // through its chunk (noting where the chain enters each segment), and
    // every lane walks its own segment to list the blocks; all lanes expand
    // them.
    uint32_t wbase, wlen;
    {  // stage frame bytes [ws, we + 2) with word loads (the record is 4-byte aligned), all issued first
        const uint32_t r0 = (12 + ws) & ~3u, r1 = min(12 + we + 2, L);
        const uint32_t* rw = (const uint32_t*)rec;
        constexpr int kIter = (kWin / 4 + 2 + 255) / 256;
        uint32_t v[kIter];
#pragma unroll
        for (int u = 0; u < kIter; ++u) {
            const uint32_t q = r0 / 4 + tid + 256u * u;
            v[u] = q * 4 < r1 ? rw[q] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kIter; ++u) {
            const uint32_t q = r0 / 4 + tid + 256u * u;
            if (q * 4 < r1) P.fwin[q - r0 / 4] = v[u];
        }
        wbase = r0 - 12;
        wlen = r1 - r0;
    }
    // a header at frame offset i (ws <= i < we: its bytes are staged)
    auto header = [&](uint32_t i, uint32_t& size, uint32_t& rle) -> uint32_t {
        const uint8_t* hp = fb + (i - wbase);
        const uint32_t h = (uint32_t)hp[0] | ((uint32_t)hp[1] << 8) | ((uint32_t)hp[2] << 16);
        size = h >> 3;
        rle = (h >> 1) & 1u;
        return block_next(h, i, flen);
    };
    __syncthreads();
    const uint32_t s0 = ws + tid * kSeg, s1 = min(s0 + kSeg, we);
    {
        // this segment's 32 bytes and the two after it, aligned to the segment start
        const uint32_t a = ws - wbase;  // 0..3: the window's first byte within fwin's first word
        uint32_t w[10], u[9];
#pragma unroll
        for (int k = 0; k < 10; ++k) w[k] = P.fwin[8 * tid + k];
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] = __builtin_amdgcn_alignbyte(w[k + 1], w[k], a);
        // backwards over the segment: where a chain through each position
        // leaves it.  Without branches: every position reads one entry (its
        // own when the step leaves the segment or the header is no block) and
        // writes its own; positions past the window's end get values nothing
        // reads (a valid step from inside the window past its end is kXOut).
        uint16_t* ys = P.u.Y + sx(tid * kSeg);  // the segment's entries (no pad inside a segment)
#pragma unroll
        for (int j = kSeg - 1; j >= 0; --j) {
            const uint32_t i = s0 + j;
            // bytes j .. j+2 of the segment from two whole words (a 64-bit
            // shift here makes the compiler keep u[] in memory)
            const uint32_t h = __builtin_amdgcn_alignbyte(u[(j >> 2) + 1], u[j >> 2], j & 3) & 0xFFFFFFu;
            const uint32_t n = block_next(h, i, flen);
            // the marks lie above every offset and keep their window mark in the low half
            const uint32_t c = n < we ? n - ws : n >= kJLast ? n & 0xFFFFu : kXOut;
            const bool in = n < s1;
            const uint32_t v = ys[in ? n - s0 : (uint32_t)j];
            ys[j] = (uint16_t)(in ? v : c);
        }
    }
    __syncthreads();
    // each step spans a segment at least, so log2(kChunk / kSeg) doublings reach
    // the chunk's end.  Entries only ever move forward along their chain and
    // never past the chunk's exit, so reads and writes of one round may
    // interleave freely; a thread takes its positions eight at a time, every
    // one read and rewritten (unchanged when its step leaves the chunk).  A
    // step stays in the chunk exactly when its offset agrees with the
    // position's above the chunk bits (marks never do).
    for (uint32_t span = kSeg; span < kChunk; span *= 2) {
        constexpr int kPer = kWin / 256, kGrp = 8;
#pragma unroll
        for (int g = 0; g < kPer; g += kGrp) {
            uint32_t y[kGrp];
#pragma unroll
            for (int k = 0; k < kGrp; ++k) y[k] = P.u.Y[sx(tid + 256u * (g + k))];
#pragma unroll
            for (int k = 0; k < kGrp; ++k) {
                const uint32_t i = tid + 256u * (g + k);
                const bool f = (y[k] ^ i) < kChunk;
                const uint32_t z = P.u.Y[sx(f ? y[k] : i)];
                y[k] = f ? z : y[k];
            }
#pragma unroll
            for (int k = 0; k < kGrp; ++k) P.u.Y[sx(tid + 256u * (g + k))] = (uint16_t)y[k];
        }
        __syncthreads();
    }
    // where the chain enters this window, and the content before it
    if (tid == 0) {
        uint64_t st = kPsPub | P0;  // window 0: the first block, no content before it
        if (win > 0) {
            uint32_t spins = 0;
            for (;;) {
                st = __hip_atomic_load(pst + win, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (st & kPsPub) break;
                if (++spins > kSpinMax) {  // never expected: the previous window did not publish
                    st = kPsPub | kPsErr;
                    atomicOr(plan.err, kErrCorrupt);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        s_state = st;
    }
    __syncthreads();
    const uint64_t st_in = s_state;
    const uint32_t entry = (uint32_t)st_in, content = (uint32_t)(st_in >> 32) & 0x1FFFFFFFu;
    if ((st_in & (kPsErr | kPsDone)) || entry >= we) {  // nothing of the chain here: pass the state on
        if (tid == 0) publish(st_in & ~kPsPub);
        return;
    }
    // the true chain: chunk entries (one lane), then segment entries (a lane per chunk)
    if (tid < kWinChunks) P.c_entry[tid] = kXBad;
    P.seg_entry[tid] = kXBad;
    __syncthreads();
    if (tid == 0) {
        uint32_t e = entry - ws;
        while (e < kXLast) {
            P.c_entry[e / kChunk] = (uint16_t)e;
            e = P.u.Y[sx(e)];
        }
    }
    __syncthreads();
    if (tid < kWinChunks) {  // block by block through the chunk, noting each segment's first
        uint32_t seg = kSegs;
        for (uint32_t e = P.c_entry[tid]; e < kXLast && e / kChunk == tid;) {
            if (e / kSeg != seg) {
                seg = e / kSeg;
                P.seg_entry[seg] = (uint16_t)e;
            }
            uint32_t size, rle;
            const uint32_t n = header(ws + e, size, rle);
            if (n >= we) break;  // leaves the window, ends the frame, or is no block
            e = n - ws;
        }
    }
    __syncthreads();
    // every lane: the blocks that start in its segment
    uint32_t cnt = 0, csz = 0, exit_n = 0, has_exit = 0;
    for (uint32_t e = P.seg_entry[tid]; e < kXLast && e / kSeg == tid;) {
        uint32_t size, rle;
        const uint32_t n = header(ws + e, size, rle);
        cnt++;
        csz += size;
        if (n >= we) {  // the chain leaves the window (or the frame ends) after this block
            exit_n = n;
            has_exit = 1;
            break;
        }
        e = n - ws;
    }
    uint32_t nblk, ctot;
    const uint32_t boff = block_excl_scan<256>(cnt, P.scratch, &nblk);
    const uint32_t coff = content + block_excl_scan<256>(csz, P.scratch, &ctot);
    if (has_exit) {
        if (exit_n == kJInvalid) P.s_err = 1;
        else if (exit_n == kJLast) P.s_done = 1;
        else P.s_next = exit_n;
    }
    if (tid == 0 && (nblk == 0 || content + ctot > nm)) P.s_err = 1;
    // the block table (the jump tables are no longer needed)
    {
        uint32_t k = boff, d = coff;
        for (uint32_t e = P.seg_entry[tid]; e < kXLast && e / kSeg == tid;) {
            uint32_t size, rle;
            const uint32_t n = header(ws + e, size, rle);
            P.u.t.dst[k] = d;
            P.u.t.src[k] = (uint16_t)((e + 3) | (rle << 15));
            k++;
            d += size;
            if (n >= we) break;
            e = n - ws;
        }
    }
    if (tid == 0) P.u.t.dst[nblk] = content + ctot;
    __syncthreads();
    if (tid == 0) {  // the next window's state, before this one's expansion
        uint64_t st;
        if (P.s_err) st = kPsErr;
        else if (P.s_done) st = kPsDone;
        else st = P.s_next | ((uint64_t)(content + ctot) << 32);
        if (!P.s_err && P.s_done && content + ctot != nm) {
            P.s_err = 1;
            st = kPsErr;
        }
        publish(st);
        if (P.s_err) atomicOr(plan.err, kErrCorrupt);
    }
    __syncthreads();
    if (P.s_err) return;
    // expansion: each thread writes a contiguous run of 16-byte groups of
    // content, finding its first block by binary search and walking on from
    // there; a word inside one block is one LDS word pair (raw) or the
    // repeated byte (RLE), a word across blocks is built byte by byte
    const uint32_t d0 = content, d1 = content + ctot;
    const uint32_t q0 = d0 & ~15u, ng = (d1 - q0 + 15) / 16, per = (ng + 255) / 256;
    const uint32_t qa = q0 + 16 * per * tid, qb = min(qa + 16 * per, d1);
    if (qa < qb) {
        const uint32_t first = qa < d0 ? d0 : qa;
        uint32_t lo = 0, hi = nblk - 1;  // the largest k with dst[k] <= first
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (P.u.t.dst[mid] <= first) lo = mid; else hi = mid - 1;
        }
        // the current block: content [bstart, bend), frame source | RLE << 31, RLE byte
        auto src_of = [&](uint32_t k) -> uint32_t {
            const uint32_t sv = P.u.t.src[k];
            return (ws + (sv & 0x7FFFu)) | ((sv >> 15) << 31);
        };
        auto byte_at = [&](uint32_t sb) -> uint32_t { return sb - wbase < wlen ? fb[sb - wbase] : f[sb]; };
        uint32_t k = lo, bstart = P.u.t.dst[k], bend = P.u.t.dst[k + 1], bsrc = src_of(k);
        uint32_t rv = byte_at(bsrc & 0x7FFFFFFFu);
        auto next_block = [&]() {
            ++k;
            bstart = bend;
            bend = P.u.t.dst[k + 1];
            bsrc = src_of(k);
            rv = byte_at(bsrc & 0x7FFFFFFFu);
        };
        for (uint32_t q = qa; q < qb; q += 16) {
            uint32_t wd[4];
#pragma unroll
            for (uint32_t g = 0; g < 4; ++g) {
                // the word's bytes [lo, hi) of the content, one block's part per pass
                const uint32_t qw = q + 4 * g, hi = min(qw + 4, d1);
                uint32_t word = 0;
                for (uint32_t d = max(qw, d0); d < hi;) {
                    while (d >= bend) next_block();  // blocks without content are passed over
                    const uint32_t e = min(hi, bend);
                    uint32_t v;
                    if (bsrc >> 31) v = rv * 0x01010101u;
                    else {
                        const uint32_t sb = (bsrc & 0x7FFFFFFFu) + (d - bstart);  // frame offset of byte d
                        const uint32_t so = sb - wbase;
                        if (so + 4 <= wlen)
                            v = __builtin_amdgcn_alignbyte(P.fwin[(so >> 2) + 1], P.fwin[so >> 2], so & 3);
                        else {  // past the staged bytes (a block running on beyond the window)
                            v = 0;
                            for (uint32_t b = 0; b < e - d; ++b) v |= byte_at(sb + b) << (8 * b);
                        }
                    }
                    const uint32_t nb = e - d;  // 1 .. 4 bytes, placed at byte d - qw of the word
                    const uint32_t m = nb >= 4 ? 0xFFFFFFFFu : (1u << (8 * nb)) - 1;
                    word |= (v & m) << (8 * (d - qw));
                    d = e;
                }
                wd[g] = word;
            }
            if (q >= d0 && q + 16 <= d1) *(uint4*)(cwb + q) = make_uint4(wd[0], wd[1], wd[2], wd[3]);
            else
                for (uint32_t b = 0; b < 16; ++b)
                    if (q + b >= d0 && q + b < d1) cwb[q + b] = (uint8_t)(wd[b >> 2] >> (8 * (b & 3)));
        }
    }
}

__device__ void parse_sections(const DecPlan& plan, uint32_t r, const DecItem& it, ParseLds& P) {
    const uint8_t* rec = it.rec;
    const uint32_t L = it.rec_len;
    const uint32_t tid = threadIdx.x;
    __shared__ uint32_t s_N, s_nb, s_sec, s_err;
    if (tid == 0) {
        const uint32_t flen = rd32(rec + 8);
        uint32_t err = 0, N = 0, nb = 0, sec = 0;
        if (flen > L - 12) err = 1;
        else {
            sec = align4(12 + flen);
            if (sec + 4 > L) err = 1;
            else {
                N = rd32(rec + sec);
                if (N > it.npx) err = 1;
                nb = div_up(N, kFrame);
                if (!err && sec + align4(4 + 3 * nb) > L) err = 1;
            }
        }
        s_err = err; s_N = N; s_nb = nb; s_sec = sec;
    }
    __syncthreads();
    if (s_err) {
        if (tid == 0) atomicOr(plan.err, kErrCorrupt);
        return;
    }
    const uint32_t sec = s_sec, N = s_N, nb = s_nb;
    const uint8_t* hb = rec + sec + 4;
    // kSecPer consecutive frames per thread: their width, count and maximum
    // width bytes loaded in one round (past the last frame: the last again,
    // unused), summed in order, then one three-value scan per pass
    constexpr uint32_t kSecPer = 8, kSecPass = 256 * kSecPer;
    __shared__ uint32_t s_scan[3 * (256 / kWave + 1)];
    // offsets within the record are 32-bit; the total is kept in 64 bits so
    // that widths and counts claiming more than 4 GiB cannot wrap past the check
    uint32_t cp = 0, cn = 0, ch = 0, bad = 0;
    uint64_t sum = 0;
    for (uint32_t j0 = 0; j0 < nb; j0 += kSecPass) {
        const uint32_t jb = j0 + tid * kSecPer;
        uint32_t fb[kSecPer], fn[kSecPer], fB[kSecPer];
#pragma unroll
        for (uint32_t u = 0; u < kSecPer; ++u) {
            const uint32_t j = min(jb + u, nb - 1);
            fb[u] = hb[j];
            fn[u] = hb[nb + j];
            fB[u] = hb[2 * nb + j];
        }
        uint32_t v[3] = {0u, 0u, 0u};  // payload, position and high part bytes of the thread's frames
#pragma unroll
        for (uint32_t u = 0; u < kSecPer; ++u) {
            if (jb + u >= nb) break;
            const uint32_t b = fb[u], n = fn[u], B = fB[u];
            if (B > it.bits || b > B || n > 128 || (n && b == B)) bad = 1;
            v[0] += 16 * b;
            v[1] += n;
            v[2] += (n * (B - b) + 7) / 8;
            it.blkinfo[jb + u] = b | (n << 8) | (B << 16);
        }
        uint32_t tot[3];
        block_excl_scan3<256>(v, s_scan, tot);
        uint32_t op = cp + v[0], on = cn + v[1], oh = ch + v[2];
#pragma unroll
        for (uint32_t u = 0; u < kSecPer; ++u) {
            const uint32_t j = jb + u;
            if (j >= nb) break;
            const uint32_t b = fb[u], n = fn[u], B = fB[u];
            it.blkoffs[3 * j] = op;
            it.blkoffs[3 * j + 1] = on;
            it.blkoffs[3 * j + 2] = oh;
            op += 16 * b;
            on += n;
            oh += (n * (B - b) + 7) / 8;
        }
        cp += tot[0]; cn += tot[1]; ch += tot[2];
        sum += (uint64_t)tot[0] + tot[1] + tot[2];
    }
    if (bad) atomicOr(&s_err, 1u);
    __syncthreads();
    if (tid == 0) {
        const uint32_t pay0 = sec + align4(4 + 3 * nb);
        // the record must end exactly after the padded sections
        uint32_t err = s_err;
        if (pay0 + ((sum + 3) & ~3ull) != L) err = 1;
        DecRes& rs = plan.res[r];
        rs.N = N;
        rs.nb = nb;
        rs.sec = sec;
        rs.pay_off = pay0;
        rs.pos_off = pay0 + cp;
        rs.high_off = pay0 + cp + cn;
        rs.high_end = pay0 + cp + cn + ch;
        if (err) atomicOr(plan.err, kErrCorrupt);
    }
}

__global__ __launch_bounds__(256) void k_dec_parse(DecPlan plan) {
    __shared__ ParseLds P;
    const uint32_t r = blockIdx.x;
    DecItem it = plan.items[r];
    if (plan.roff) {  // the record from the device-side index; later kernels find it in the item
        const uint64_t o = plan.roff[r];
        if (o == ~0ull) {
            if (threadIdx.x == 0 && blockIdx.y == plan.pwin) atomicOr(plan.err, kErrCorrupt);
            return;
        }
        it.rec = (const JG uint8_t*)o;
        it.rec_len = plan.rlen[r];
        if (threadIdx.x == 0 && blockIdx.y == plan.pwin) {
            plan.items[r].rec = it.rec;
            plan.items[r].rec_len = it.rec_len;
        }
    }
    if (blockIdx.y < plan.pwin) parse_mask(plan, r, it, P);
    else parse_sections(plan, r, it, P);
}

// ---------------------------------------------------------------------------
// Plan upload (blocks before the last, 16 bytes per thread from host-mapped
// memory).  The last block clears the records' parse window states and, with
// a device-side index, indexes the records: the stream header must equal the
// expected one, every table length must be a multiple of 4 of at least 12
// bytes, and the records must end exactly at the end of the stream;
// otherwise every record offset is ~0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dec_prepare(const uint4* src, uint4* dst, uint32_t n16, DecPlan plan,
                                                     uint32_t up_blocks) {
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x < up_blocks) {
        const uint32_t i = blockIdx.x * 256 + tid;
        if (i < n16) ((JG uint4*)dst)[i] = load_system16((const JG uint4*)src + i);
        return;
    }
    // one workgroup per stream (one in all without an index): its records'
    // parse window states and window tickets start at zero
    const uint32_t s = blockIdx.x - up_blocks, nsrc = plan.roff ? plan.n_src : 1u;
    const uint32_t A = plan.roff ? plan.src_attrs : plan.n_attrs, nq = plan.n_scans * A;
    auto item = [&](uint32_t qi) {  // the item of the stream's record qi = t * A + a
        const uint32_t t = qi / A, a = qi - t * A;
        return t * plan.n_attrs + s * A + a;
    };
    {
        const uint32_t per = plan.pwin + 2;  // pwin + 1 states, then the ticket word
        for (uint32_t i = tid; i < nq * per; i += 256) {
            const uint32_t qi = i / per, k = i - qi * per;
            JG uint64_t* st = parse_states(plan, item(qi));
            if (k <= plan.pwin) st[k] = 0;
            else *(JG uint32_t*)(st + k) = 0u;
        }
    }
    if (!plan.roff || s >= nsrc) return;
    __shared__ uint64_t scratch[8];
    __shared__ uint32_t s_bad;
    __shared__ uint4 s_src;
    if (tid == 0) {
        s_bad = 0;
        s_src = load_system16((const JG uint4*)(plan.srcs + s));
    }
    __syncthreads();
    const uint64_t base = (uint64_t)s_src.x | ((uint64_t)s_src.y << 32), len = (uint64_t)s_src.z | ((uint64_t)s_src.w << 32);
    const JG uint32_t* words = (const JG uint32_t*)base;
    const JG uint32_t* tab = (const JG uint32_t*)(base + plan.hdr_len);
    if (len < plan.hdr_len + 4ull * nq) s_bad = 1;  // read before any table word (all threads agree)
    __syncthreads();
    if (!s_bad) {
        if (plan.hdr_check && tid < plan.hdr_len / 4 && words[tid] != plan.hdr_words[tid]) atomicOr(&s_bad, 1u);
        uint64_t carry = (uint64_t)plan.hdr_len + 4ull * nq;
        for (uint32_t q0 = 0; q0 < nq; q0 += 256) {
            const uint32_t qi = q0 + tid;
            const uint32_t l = qi < nq ? tab[qi] : 0u;
            if (qi < nq && (l < 12 || l % 4)) atomicOr(&s_bad, 1u);
            uint64_t total;
            const uint64_t pre = block_excl_scan64<256>((uint64_t)l, scratch, &total) + carry;
            if (qi < nq) {
                plan.roff[item(qi)] = base + pre;
                plan.rlen[item(qi)] = l;
            }
            carry += total;
        }
        if (tid == 0 && carry != len) s_bad = 1;
    }
    __syncthreads();
    if (s_bad)
        for (uint32_t qi = tid; qi < nq; qi += 256) plan.roff[item(qi)] = ~0ull;  // the same thread wrote it above
}

hipError_t launch_dec_prepare(const void* host, void* dev, size_t bytes, const DecPlan& plan, hipStream_t stream) {
    const uint32_t n16 = (uint32_t)(bytes / 16);
    const uint32_t up = div_up(n16, 256);  // then one workgroup per stream (one without an index)
    const uint32_t blocks = up + (plan.roff ? plan.n_src : 1u);
    JIFFY_LAUNCH("k_dec_prepare", k_dec_prepare, dim3(blocks), dim3(256), stream, (const uint4*)host, (uint4*)dev,
                 n16, plan, up);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mask chain over time: a P-scan's mask is its content XOR the previous
// scan's mask, an I-scan's mask is its content.  A workgroup takes 64
// 32-bit halves of the mask words of one attribute over every scan; each of
// its waves takes kMaskAhead consecutive scans (their loads issued together)
// and runs the chain from a carry of 0, keeping the chunk's last mask and
// whether the chunk holds an I-scan.  The chain is linear in the carry
// (XOR), so a chunk without an I-scan ends at its last mask XOR the carry
// into it, and one with an I-scan does not depend on the carry: each wave
// folds the summaries of the chunks before it to get its own carry, then
// writes its scans' valid words.  Rounds of (waves x kMaskAhead) scans
// follow one another with the carry passed on.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t* item_words(const DecPlan& plan, uint32_t r, uint32_t off) {
    return (uint64_t*)(plan.ws + plan.item_stride * r + off);
}

constexpr int kMaskAhead = 32;
constexpr uint32_t kMaskWaves = 16;  // waves per workgroup of k_dec_mask, at most

__global__ __launch_bounds__(kMaskWaves * 64) void k_dec_mask(DecPlan plan) {
    if (*plan.err) return;
    __shared__ uint32_t s_end[kMaskWaves][64], s_reset[kMaskWaves][64];
    const uint32_t a = blockIdx.y, l = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const uint32_t h = blockIdx.x * 64 + l;  // half-word index
    const bool live = h < 2 * plan.nwords;
    const uint32_t tm = live ? (uint32_t)(tail_mask(h >> 1, plan.nwords, plan.npx) >> (32 * (h & 1))) : 0u;
    const uint32_t A = plan.n_attrs, T = plan.n_scans;
    uint32_t carry = 0;  // the mask of the scan before this round
    bool bad = false;
    for (uint32_t t_round = 0; t_round < T; t_round += nw * kMaskAhead) {
        const uint32_t t0 = t_round + w * kMaskAhead;
        // the modes are loaded with the words, and every load is issued (past
        // the last scan it reads the last scan again, unused): nothing waits alone
        uint32_t c[kMaskAhead], md[kMaskAhead];
#pragma unroll
        for (int k = 0; k < kMaskAhead; ++k) {
            const uint32_t t = min(t0 + k, T - 1);
            c[k] = live ? ((const uint32_t*)item_words(plan, t * A + a, plan.off_cw))[h] : 0u;
            md[k] = plan.modes[t * A + a];
        }
        uint32_t loc = 0, reset = 0;
#pragma unroll
        for (int k = 0; k < kMaskAhead; ++k) {
            if (t0 + k < T) {
                loc = md[k] ? (c[k] ^ loc) : c[k];
                reset |= md[k] ? 0u : 1u;
            }
        }
        s_end[w][l] = loc;
        s_reset[w][l] = reset;
        __syncthreads();
        uint32_t prev = carry;
        for (uint32_t v = 0; v < w; ++v) prev = s_reset[v][l] ? s_end[v][l] : (s_end[v][l] ^ prev);
        uint32_t next = carry;  // the carry into the next round: the last chunk's true end
        for (uint32_t v = 0; v < nw; ++v) next = s_reset[v][l] ? s_end[v][l] : (s_end[v][l] ^ next);
#pragma unroll
        for (int k = 0; k < kMaskAhead; ++k) {
            const uint32_t t = t0 + k;
            if (t < T && live) {
                const uint32_t m = md[k] ? (c[k] ^ prev) : c[k];
                bad |= (m & ~tm) != 0;  // mask bits past the scan
                ((uint32_t*)item_words(plan, t * A + a, plan.off_vw))[h] = ~m & tm;
                prev = m;
            }
        }
        carry = next;
        __syncthreads();  // the summaries are free for the next round
    }
    if (bad) atomicOr(plan.err, kErrCorrupt);
}

constexpr uint32_t kDecTileFrames = (kDecTileVals + 2 * kFrame - 2) / kFrame;  // frames a tile's values can touch
constexpr uint32_t kDecThreads = (4 * kDecTileFrames + 63) / 64 * 64;  // a quad per frame, in whole waves
constexpr uint32_t kFrameMaxWords = 160;              // a frame's packed bytes are at most 640

// ---------------------------------------------------------------------------
// Running count of valid samples (N must match the section header) and the
// record's decode tiles.  One round per kDecBlockPx-pixel block (1024 mask
// words, one per thread): the block's first pixel starts a tile, and so does
// every valid pixel whose rank is a positive multiple of kDecTileVals inside
// the block (the word that holds that rank finds its bit); the tiles are
// numbered in pixel order by counting, per block, one tile plus its rank
// boundaries.  Then each tile's descriptor (values and pixels), with the
// check that its frames' packed bytes are plausible.  The tiles' look-back
// states and the record's ticket are cleared here, before k_dec_tiles.
// ---------------------------------------------------------------------------
static_assert(kDecBlockPx == 64 * 1024, "a block is one mask word per thread of k_dec_scan");

__global__ __launch_bounds__(1024) void k_dec_scan(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t r = blockIdx.x;
    const DecItem it = plan.items[r];
    const DecRes rs = plan.res[r];
    __shared__ uint32_t scratch[20];
    for (uint32_t lt = threadIdx.x; lt < plan.nvt; lt += 1024) it.status[lt] = 0ull;
    if (threadIdx.x == 0) *it.tctr = 0u;
    uint32_t carry = 0, tiles = 0;  // valid samples and tiles before the block
    // the words of kScanAhead blocks are requested together, then the blocks
    // are counted one after another
    constexpr uint32_t kScanAhead = 8;
    for (uint32_t wa = 0; wa < it.nwords; wa += 1024 * kScanAhead) {
        uint64_t vv[kScanAhead];
#pragma unroll
        for (uint32_t u = 0; u < kScanAhead; ++u) {
            const uint32_t w = wa + 1024 * u + threadIdx.x;
            vv[u] = w < it.nwords ? it.vw[w] : 0ull;
        }
#pragma unroll
        for (uint32_t u = 0; u < kScanAhead; ++u) {
            const uint32_t w0 = wa + 1024 * u;
            if (w0 >= it.nwords) break;
            const uint32_t w = w0 + threadIdx.x;
            const uint64_t v = vv[u];
            const uint32_t c = (uint32_t)__popcll(v);
            uint32_t total;
            const uint32_t pre = block_excl_scan<1024>(c, scratch, &total) + carry;
            const uint32_t k0 = carry / kDecTileVals;
            if (threadIdx.x == 0) it.tstart[tiles] = make_uint2(64u * w0, carry);
            if (c) {  // a rank boundary in this word: at most one, a word holds 64 values
                const uint32_t k = (pre + c - 1) / kDecTileVals, R = k * kDecTileVals;
                if (k > k0 && R >= pre) it.tstart[tiles + (k - k0)] = make_uint2(64u * w + select_bit(v, R - pre), R);
            }
            tiles += 1 + (total ? (carry + total - 1) / kDecTileVals - k0 : 0u);
            carry += total;
        }
    }
    if (threadIdx.x == 0) {
        it.tstart[tiles] = make_uint2(it.npx, carry);
        plan.res[r].ntiles = tiles;
        if (carry != rs.N || tiles > plan.nvt) atomicOr(plan.err, kErrCorrupt);
    }
    __syncthreads();  // every tile start stored
    if (carry != rs.N || tiles > plan.nvt) return;
    const uint32_t sec[3] = {rs.pay_off, rs.pos_off, rs.high_off};
    const uint32_t send[3] = {rs.pos_off - rs.pay_off, rs.high_off - rs.pos_off, rs.high_end - rs.high_off};
    bool bad = false;
    for (uint32_t lt = threadIdx.x; lt < tiles; lt += 1024) {
        const uint2 a = it.tstart[lt], b = it.tstart[lt + 1];
        DecTile d;
        d.ps = a.x;
        d.kb = a.y;
        d.pe = b.x;
        d.ke = b.y;
        const uint32_t jf = d.kb >> 7, j1 = d.ke > d.kb ? ((d.ke - 1) >> 7) + 1 : jf;  // frames [jf, j1)
        uint32_t words = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const uint32_t o0 = jf < rs.nb ? it.blkoffs[3 * jf + q] : send[q];
            const uint32_t o1 = j1 < rs.nb ? it.blkoffs[3 * j1 + q] : send[q];
            words += j1 > jf ? ((sec[q] + o1 + 3) >> 2) - ((sec[q] + o0) >> 2) : 0u;
        }
        // more than 640 bytes per frame, or a tile of no pixels or too many: not a valid tile
        bad |= words > (j1 - jf) * kFrameMaxWords + 6 || d.pe <= d.ps || d.pe - d.ps > kDecBlockPx ||
               d.ke - d.kb > kDecTileVals;
        it.tdesc[lt] = d;
    }
    if (bad) atomicOr(plan.err, kErrCorrupt);
}

// ---------------------------------------------------------------------------
// Frame unpacking and the running sum, per decode tile (Sec. II, Sec. III-C
// reversed): at most kDecTileVals values and kDecBlockPx pixels of one
// record.  Workgroups are laid out tile-major (workgroup i serves record
// i mod n); the tile within the record is taken in arrival order (a ticket),
// so every tile a workgroup waits for has started, and workgroups past the
// record's tile count leave at once.
//   1. the frames' widths and offsets are loaded;
//   2. four lanes per frame unpack the low bits (lane q: values 32q..32q+31,
//      its b payload words loaded straight from the record into registers)
//      into the frame's LDS row, patch the exceptions' high parts in, and
//      undo ZigZag (Eq. 1);
//   3. a workgroup scan sums the deltas of the tile's values; the running
//      sum before the tile comes from the tiles before it (decoupled
//      look-back: each tile publishes its own sum, then the running sum
//      through it);
//   4. the tile's pixels are written: the k-th valid pixel gets value k,
//      the others zero.  Each wave writes a run of segments of contiguous
//      bytes (lane l a segment's l-th 16 bytes), so each store covers whole
//      cache lines; its valid-pixel words are requested before the
//      look-back and held in registers.  The groups at the tile's two ends
//      write only the tile's own pixels.
// For a P-scan the values are differences to the previous scan (added by
// k_dec_temporal); for P > 1 they are quantized (restored there too).
// ---------------------------------------------------------------------------
constexpr uint64_t kStAgg = 1ull << 32, kStIncl = 2ull << 32;  // look-back status flags

// The pixels are written by segments of 64 lane groups: a lane group is the
// 16 bytes of output one lane stores at once (16 / WB pixels), so one wave's
// store covers a segment's whole contiguous bytes.
template <int WB> struct SegT {
    static constexpr uint32_t kGroup = 16 / WB;              // pixels per lane
    static constexpr uint32_t kPx = kWave * kGroup;          // pixels per segment (a multiple of 64)
    static constexpr uint32_t kWords = kPx / 64;             // valid-pixel words per segment (divides 64)
    static constexpr uint32_t kSegs = kDecBlockPx / kPx + 1; // segments a tile touches, at most
    // a wave's run of segments and its words, at most, and the words each lane holds
    static constexpr uint32_t kRun = (kSegs + kDecThreads / kWave - 1) / (kDecThreads / kWave);
    static constexpr uint32_t kSlots = (kRun * kWords + kWave - 1) / kWave;
    static_assert(kWave % kWords == 0, "a segment's words lie in one slot");
};

// Valid-pixel word of a tile holding pixel p (a multiple of 64), its bits
// outside the tile's pixels [ps, pe) cleared; 0 past the tile.
__device__ __forceinline__ uint64_t tile_word(const DecItem& it, const DecTile& D, uint32_t p) {
    if (p >= D.pe || p + 64u <= D.ps) return 0;  // (a shift of 64 or more is undefined)
    uint64_t w = it.vw[p >> 6];
    if (p < D.ps) w &= ~0ull << (D.ps - p);
    if (D.pe - p < 64u) w &= (1ull << (D.pe - p)) - 1ull;
    return w;
}

template <class R>
struct DecTileLds {
    R rows[kDecTileFrames * RowT<R>::kElems];
    uint32_t info[kDecTileFrames];
    uint32_t offs[kDecTileFrames + 1][3];  // frame offsets in the three sections
    uint32_t scratch[8];
    uint32_t ticket, base, bad;
};

// `width` bits from bit bp of a little-endian word array.  Without kExact
// it may read the word after the bits; with kExact (the record itself) it
// never reads past them.
template <bool kExact, class W>
__device__ __forceinline__ uint32_t bits_at(W* w, uint32_t bp, uint32_t width) {
    const uint32_t sh = bp & 31;
    uint64_t v = w[bp >> 5];
    if (!kExact || sh + width > 32) v |= (uint64_t)w[(bp >> 5) + 1] << 32;
    return (uint32_t)(v >> sh) & low_mask32(width);
}

// One wave: publishes the tile's sum, then sums the tiles before it from the
// nearest one whose running sum is known, 64 tiles per round.  Returns the
// running sum before the tile.
__device__ uint32_t dec_lookback(JG uint64_t* st, uint32_t lt, uint32_t agg, JG uint32_t* err2) {
    const uint32_t l = lane_id();
    if (l == 0) __hip_atomic_store(st + lt, (lt ? kStAgg : kStIncl) | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lt == 0) return 0;
    uint32_t excl = 0, end = lt, spins = 0;  // tiles [0, end) not summed yet
    for (;;) {
        const int idx = (int)end - 1 - (int)l;  // lane 0: the nearest
        uint64_t s = kStIncl;                    // before the first tile: running sum 0
        if (idx >= 0) s = __hip_atomic_load(st + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t f = s & ~0xFFFFFFFFull;
        const uint64_t incl = ballot(f == kStIncl), empty = ballot(f == 0);
        const uint32_t fi = incl ? (uint32_t)__builtin_ctzll(incl) : 64u;
        const uint32_t fe = empty ? (uint32_t)__builtin_ctzll(empty) : 64u;
        if (fe < fi) {  // a nearer tile has not published: take the sums before it, poll again
            if (fe) {
                excl += wave_sum(l < fe ? (uint32_t)s : 0u);
                end -= fe;
            }
            if (++spins > kSpinMax) {  // never expected: a tile before this one did not publish
                if (l == 0) atomicOr(err2, kErrCorrupt);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_sum(l <= fi ? (uint32_t)s : 0u);
        if (fi < 64) break;
        end -= 64;
    }
    if (l == 0) __hip_atomic_store(st + lt, kStIncl | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// The low B bits of a lane's 32 values: its B payload words (from w) are
// loaded at once, then every value is taken out of them with shifts known
// at compile time.
template <int B>
__device__ __forceinline__ void unpack32(const JG uint32_t* w, uint32_t z[32]) {
    uint32_t v[B];
#pragma unroll
    for (int k = 0; k < B; ++k) v[k] = w[k];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        constexpr uint32_t kMask = B == 32 ? 0xFFFFFFFFu : ((1u << B) - 1u);
        const int bit = i * B, lo = bit >> 5, sh = bit & 31;
        uint32_t x = v[lo] >> sh;
        if (sh + B > 32) x |= v[lo + 1] << (32 - sh);
        z[i] = x & kMask;
    }
}
#define JIFFY_UNPACK_CASE(B) \
    case B: unpack32<B>(w, z); break;
__device__ __forceinline__ void unpack_lane(const JG uint32_t* w, uint32_t b, uint32_t z[32]) {
    switch (b) {
        JIFFY_UNPACK_CASE(1) JIFFY_UNPACK_CASE(2) JIFFY_UNPACK_CASE(3) JIFFY_UNPACK_CASE(4)
        JIFFY_UNPACK_CASE(5) JIFFY_UNPACK_CASE(6) JIFFY_UNPACK_CASE(7) JIFFY_UNPACK_CASE(8)
        JIFFY_UNPACK_CASE(9) JIFFY_UNPACK_CASE(10) JIFFY_UNPACK_CASE(11) JIFFY_UNPACK_CASE(12)
        JIFFY_UNPACK_CASE(13) JIFFY_UNPACK_CASE(14) JIFFY_UNPACK_CASE(15) JIFFY_UNPACK_CASE(16)
        JIFFY_UNPACK_CASE(17) JIFFY_UNPACK_CASE(18) JIFFY_UNPACK_CASE(19) JIFFY_UNPACK_CASE(20)
        JIFFY_UNPACK_CASE(21) JIFFY_UNPACK_CASE(22) JIFFY_UNPACK_CASE(23) JIFFY_UNPACK_CASE(24)
        JIFFY_UNPACK_CASE(25) JIFFY_UNPACK_CASE(26) JIFFY_UNPACK_CASE(27) JIFFY_UNPACK_CASE(28)
        JIFFY_UNPACK_CASE(29) JIFFY_UNPACK_CASE(30) JIFFY_UNPACK_CASE(31) JIFFY_UNPACK_CASE(32)
        default:  // b = 0 (a width above 32 is rejected by the section parse)
#pragma unroll
            for (int i = 0; i < 32; ++i) z[i] = 0;
    }
}
#undef JIFFY_UNPACK_CASE

constexpr uint32_t kExPre = 4;  // exceptions per lane requested with the frame's payload

// Four lanes unpack frame jf + g from the record's words: pay_w is the
// frame's first payload word, pos_b its first exception-position byte,
// high_bit its first high-part bit.  d gets the lane's running sum of the
// deltas of the tile's values.
template <class R, class W = const JG uint32_t>
__device__ __forceinline__ void dec_unpack(const DecItem& it, const DecRes& rs, DecTileLds<R>& L, W* words, uint32_t g,
                                           uint32_t q, uint32_t kb, uint32_t ke, uint32_t jf, uint32_t pay_w,
                                           uint32_t pos_b, uint32_t high_bit, uint32_t d[32], uint32_t& lane_sum) {
    const uint32_t j = jf + g;
    const uint32_t info = L.info[g];
    const uint32_t b = info & 0xFFu, n = (info >> 8) & 0xFFu, B = (info >> 16) & 0xFFu;
    const uint32_t hw = B - b, real = min(kFrame, rs.N - j * kFrame);
    R* row = L.rows + g * RowT<R>::kElems;
    const uint32_t i0 = 32u * q;
    // the lane's first kExPre exceptions (e = q, q + 4, ...) are requested
    // with the payload
    constexpr uint32_t kPre = kExPre;
    const JG uint8_t* pos = (const JG uint8_t*)words + pos_b;
    uint32_t ep[kExPre], eq[kExPre], eh[kExPre];
#pragma unroll
    for (uint32_t i = 0; i < kPre; ++i) {
        const uint32_t e = q + 4 * i;
        ep[i] = eq[i] = eh[i] = 0;
        if (e < n) {
            ep[i] = pos[e];
            eq[i] = e ? pos[e - 1] : 0u;
            eh[i] = bits_at<true>(words, high_bit + e * hw, hw);
        }
    }
    uint32_t z[32];
    unpack_lane(words + pay_w + q * b, b, z);  // lane q's values fill words q*b .. q*b + b - 1 of the frame
    row_put<R>(row, q, z);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if (n) {
        // OR each high part in without waiting for the element (positions
        // increase strictly, so no two lanes touch one element; a 16-bit
        // element is ORed into its 32-bit word, the other half unchanged)
        uint32_t bad = 0;
        auto patch = [&](uint32_t e, uint32_t p, uint32_t p_before, uint32_t high) {
            if (p >= real || (e && p_before >= p)) {
                bad = 1;
                return;
            }
            const uint32_t x = high << b, idx = roff<R>(p);
            if (sizeof(R) == 4)
                __hip_atomic_fetch_or((uint32_t*)row + idx, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            else
                __hip_atomic_fetch_or((uint32_t*)row + (idx >> 1), x << (16 * (idx & 1)), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WAVEFRONT);
        };
#pragma unroll
        for (uint32_t i = 0; i < kPre; ++i)
            if (q + 4 * i < n) patch(q + 4 * i, ep[i], eq[i], eh[i]);
        for (uint32_t e = q + 4 * kPre; e < n; e += 4)  // (e - 1 only for e > 0: it would wrap)
            patch(e, pos[e], e ? pos[e - 1] : 0u, bits_at<true>(words, high_bit + e * hw, hw));
        if (bad) atomicOr(&L.bad, 1u);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    row_get<R>(row, q, z);
    // deltas of the tile's own values, inclusive running sum over the lane:
    // bit i of `in` is set when value k0 + i lies in [kb, ke)
    const uint32_t k0 = j * kFrame + i0;
    const uint32_t lo = kb > k0 ? min(kb - k0, 32u) : 0u, hi = ke > k0 ? min(ke - k0, 32u) : 0u;
    const uint32_t in = (hi >= 32 ? ~0u : (1u << hi) - 1u) & ~(lo >= 32 ? ~0u : (1u << lo) - 1u);
    if (in == ~0u) {
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            lane_sum += unzigzag(z[i], it.bits);
            d[i] = lane_sum;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            lane_sum += ((in >> i) & 1u) ? unzigzag(z[i], it.bits) : 0u;
            d[i] = lane_sum;
        }
    }
}

// Value k sits at row element k + kPad (k >> 5) - kElems jf (a row holds
// 128 values and kPad pad elements per 32).  A lane's group of pixels
// starts at pixel p0; bit i of `bits` marks pixel p0 + i valid (only the
// tile's own pixels can be), k is the value of its first valid pixel.
// Every pixel's read is issued, without a branch (a pixel without a value
// reads the next value's element, clamped to the rows), and its zero
// selected afterwards.  A group wholly inside the tile is written with one
// 16-byte store; a group at the tile's ends pixel by pixel, its own pixels
// only.
template <int WB, class R>
__device__ __forceinline__ void dec_group_store(const DecItem& it, const DecTile& D, uint32_t p0, uint32_t bits,
                                                uint32_t k, uint32_t jf, const DecTileLds<R>& L) {
    static_assert(RowT<R>::kElems == 128 + 4 * RowT<R>::kPad, "a row is 128 values and four pads");
    constexpr uint32_t G = SegT<WB>::kGroup;
    constexpr uint32_t kLast = kDecTileFrames * RowT<R>::kElems - 1;
    using T = typename SampleT<WB>::T;
    const uint32_t rbase = RowT<R>::kElems * jf;
    uint32_t v[G];
#pragma unroll
    for (uint32_t i = 0; i < G; ++i) {
        const uint32_t on = (bits >> i) & 1u;
        const uint32_t x = L.rows[min(k + RowT<R>::kPad * (k >> 5) - rbase, kLast)];
        v[i] = on ? x : 0u;
        k += on;
    }
    if (p0 >= D.ps && p0 + G <= D.pe && it.aligned16) {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (uint32_t i = 0; i < G; ++i) w[i * WB / 4] |= (v[i] & low_mask32(8 * WB)) << (8 * ((i * WB) & 3));
        *(uint4*)((T*)it.out + p0) = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
#pragma unroll
        for (uint32_t i = 0; i < G; ++i)
            if (p0 + i >= D.ps && p0 + i < D.pe) ((T*)it.out)[p0 + i] = (T)v[i];
    }
}

// R: the row element; the workgroups serve the n records rec_list[first ..]
// (one instantiation per sample width WB: a single store path each)
template <class R, int WB>
__global__ __launch_bounds__(kDecThreads) void k_dec_tiles(DecPlan plan, uint32_t first, uint32_t n) {
    if (*plan.err) return;  // set before this launch; this kernel reports through err2
    __shared__ DecTileLds<R> L;
    const uint32_t tid = threadIdx.x;
    const uint32_t r = plan.rec_list[first + blockIdx.x % n];
    const DecItem it = plan.items[r];
    if (tid == 0) {
        L.ticket = atomicAdd(it.tctr, 1u);
        L.bad = 0;
    }
    // 1. the tile's descriptor and its frames' widths and offsets.  Workgroups
    // usually arrive in index order, so those of the tile the index names are
    // requested while the ticket (and the record's results) are on their way,
    // and requested again only when the ticket names another tile (a guess
    // past the record's tiles reads in-bounds words that are not used)
    const DecRes rs = plan.res[r];
    DecTile D;
    uint32_t mo[4];  // the thread's frame: its three section offsets and its widths
    auto tile_meta = [&](uint32_t t) {
        D = it.tdesc[t];
        const uint32_t j = (D.kb >> 7) + tid;
        if (tid <= kDecTileFrames && j < it.maxnb) {
            mo[0] = it.blkoffs[3 * j];
            mo[1] = it.blkoffs[3 * j + 1];
            mo[2] = it.blkoffs[3 * j + 2];
            mo[3] = it.blkinfo[j];
        }
    };
    const uint32_t guess = blockIdx.x / n;
    tile_meta(min(guess, plan.nvt - 1u));
    __syncthreads();
    const uint32_t lt = L.ticket;
    if (lt >= rs.ntiles) return;  // more workgroups than the record has tiles
    if (lt != guess) tile_meta(lt);
    const uint32_t m = low_mask32(it.bits);
    const uint32_t kb = D.kb, ke = D.ke;
    const uint32_t jf = kb >> 7;
    const uint32_t nf = ke > kb ? ((ke - 1) >> 7) - jf + 1 : 0u;  // frames the tile's values lie in
    if (tid <= nf && nf) {
        const uint32_t j = jf + tid;
        if (j < rs.nb) {
            L.offs[tid][0] = mo[0];
            L.offs[tid][1] = mo[1];
            L.offs[tid][2] = mo[2];
            if (tid < nf) L.info[tid] = mo[3];
        } else {  // the ends of the sections
            L.offs[tid][0] = rs.pos_off - rs.pay_off;
            L.offs[tid][1] = rs.high_off - rs.pos_off;
            L.offs[tid][2] = rs.high_end - rs.high_off;
        }
    }
    __syncthreads();
    // 2. unpack: quad g decodes frame jf + g, straight from the record
    const uint32_t g = tid >> 2, q = tid & 3u;
    uint32_t d[32];
    uint32_t lane_sum = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) d[i] = 0;
    if (g < nf)
        dec_unpack<R>(it, rs, L, (const JG uint32_t*)it.rec, g, q, kb, ke, jf, (rs.pay_off + L.offs[g][0]) >> 2,
                      rs.pos_off + L.offs[g][1], 8 * (rs.high_off + L.offs[g][2]), d, lane_sum);
    // the tile's valid-pixel words, requested now and used in step 4: wave
    // w writes the segments [s0, s1) (from the segment holding the tile's
    // first pixel), whose words lane l holds from the l-th on, every 64th
    constexpr uint32_t S = SegT<WB>::kPx, kW = SegT<WB>::kWords, kSlots = SegT<WB>::kSlots;
    const uint32_t P0 = D.ps & ~(S - 1u), nseg = div_up(D.pe - P0, S);
    const uint32_t wv = tid / kWave, l = tid % kWave, run = div_up(nseg, kDecThreads / kWave);
    const uint32_t s0 = min(wv * run, nseg), s1 = min(s0 + run, nseg);
    uint64_t held[kSlots];
    uint32_t cnt = 0;
#pragma unroll
    for (uint32_t k = 0; k < kSlots; ++k) {
        const uint32_t wi = s0 * kW + l + kWave * k;  // word index from P0
        held[k] = wi < s1 * kW ? tile_word(it, D, P0 + 64u * wi) : 0ull;
    }
    // 3. running sum: lanes are in value order (quads in frame order)
    uint32_t agg;
    const uint32_t excl = block_excl_scan<kDecThreads>(lane_sum, L.scratch, &agg);
    if (tid < kWave) {
        const uint32_t base = dec_lookback(it.status, lt, agg, plan.err2);
        if (tid == 0) L.base = base;
    }
    __syncthreads();
    if (tid == 0 && L.bad) atomicOr(plan.err2, kErrCorrupt);
    if (g < nf) {
        const uint32_t v0 = L.base + excl;
#pragma unroll
        for (int i = 0; i < 32; ++i) d[i] = (v0 + d[i]) & m;
        row_put<R>(L.rows + g * RowT<R>::kElems, q, d);
    }
    // 4. the tile's pixels: the k-th valid pixel gets value k.  A wave's
    // first value follows the valid pixels of the waves before it; segment
    // by segment, lane l takes the l-th group of pixels, its word fetched
    // from the lane that holds it
#pragma unroll
    for (uint32_t k = 0; k < kSlots; ++k) cnt += __popcll(held[k]);
    uint32_t total;
    const uint32_t before = block_excl_scan<kDecThreads>(cnt, L.scratch, &total);
    uint32_t next = kb + (uint32_t)__builtin_amdgcn_readfirstlane((int)before);  // lane 0's: the waves before
    constexpr uint32_t G = SegT<WB>::kGroup;
    for (uint32_t i = 0; s0 + i < s1; ++i) {
        const uint32_t j = i * kW + l * G / 64, slot = i * kW / kWave;  // slot: the same for the whole wave
        uint64_t h = held[0];
#pragma unroll
        for (uint32_t k = 1; k < kSlots; ++k)
            if (slot == k) h = held[k];
        const uint32_t src = j % kWave;
        const uint64_t w = (uint64_t)(uint32_t)__shfl((int)(uint32_t)h, (int)src, kWave) |
                           ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(h >> 32), (int)src, kWave) << 32);
        const uint32_t bits = (uint32_t)(w >> ((l * G) & 63u)) & low_mask32(G);
        const uint32_t c = __popc(bits), inc = wave_incl_scan(c);
        const uint32_t p0 = P0 + (s0 + i) * S + l * G;
        if (p0 < D.pe) dec_group_store<WB, R>(it, D, p0, bits, next + inc - c, jf, L);
        next += (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
    }
}

// ---------------------------------------------------------------------------
// Over time, per pixel: a P-scan adds the previous decoded scan at its valid
// pixels (Sec. III-D); then q * P, saturated to the sample width.  The
// attribute's list of scans to read is built in LDS: a scan is read only
// when it is a P-scan, precedes one, or has P > 1.
// ---------------------------------------------------------------------------
constexpr uint32_t kModeLds = 8192;

// The scans that must be read: P-scans, scans followed by a P-scan, and
// every scan when P > 1; taken in order, with the next kTempAhead - 1 scans'
// samples in flight while the current one is finished (the loads do not
// depend on each other, only the sums do).  A thread takes one 32-bit word
// of every scan: 4 / WB pixels.
constexpr int kTempAhead = 8;
template <int WB>
__device__ __forceinline__ void dec_temporal_body(const DecPlan& plan, uint32_t a, uint8_t* out, uint32_t P,
                                                  uint32_t p0, const uint16_t* list, uint32_t tb, uint32_t nlist,
                                                  uint32_t qprev[4 / WB]) {
    constexpr int NP = 4 / WB;
    const uint32_t A = plan.n_attrs;
    const uint32_t bits = 8 * WB, m = low_mask32(bits);
    const uint64_t stride = (uint64_t)plan.npx * WB;
    const bool whole = ((uintptr_t)out % 4 == 0) && (stride % 4 == 0) && p0 + NP <= plan.npx;
    using T = typename SampleT<WB>::T;
    // e: a list entry (the scan, and bit 15 set for a P-scan).  The loads land
    // in registers that nothing reads before the scan's turn, so the next
    // scans' loads stay in flight meanwhile.
    auto fetch = [&](uint32_t e, uint32_t& w, uint64_t& vw) {
        const uint32_t t = tb + (e & 0x7FFFu);
        const uint8_t* s = out + stride * t + (uint64_t)p0 * WB;
        if (whole) w = *(const uint32_t*)s;
        else {
            w = 0;
            for (int i = 0; i < NP; ++i)
                if (p0 + i < plan.npx) w |= (uint32_t)((const T*)s)[i] << (8 * WB * i);
        }
        // the valid-sample words exist for every record; an I-scan's is not used
        vw = item_words(plan, t * A + a, plan.off_vw)[p0 >> 6];
    };
    auto put = [&](uint32_t t, const uint32_t v[NP]) {
        uint8_t* d = out + stride * t + (uint64_t)p0 * WB;
        if (whole) {
            uint32_t w = 0;
#pragma unroll
            for (int i = 0; i < NP; ++i) w |= v[i] << (8 * WB * i);
            *(uint32_t*)d = w;
        } else {
            for (int i = 0; i < NP; ++i)
                if (p0 + i < plan.npx) ((T*)d)[i] = (T)v[i];
        }
    };
    uint32_t buf[kTempAhead];
    uint64_t bw[kTempAhead];
#pragma unroll
    for (int j = 0; j < kTempAhead; ++j)
        if ((uint32_t)j < nlist) fetch(list[j], buf[j], bw[j]);
    for (uint32_t k0 = 0; k0 < nlist; k0 += kTempAhead) {
#pragma unroll
        for (int j = 0; j < kTempAhead; ++j) {
            const uint32_t k = k0 + j;
            if (k >= nlist) break;
            const uint32_t e = list[k], t = tb + (e & 0x7FFFu);
            const bool pscan = e >> 15;
            const uint32_t cb = (uint32_t)(bw[j] >> (p0 & 63));
            uint32_t v[NP];
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const uint32_t r = (buf[j] >> (8 * WB * i)) & m;
                // P-scan: the previous scan added at the valid pixels; I-scan: the sample itself
                const uint32_t q = !pscan ? r : (cb >> i) & 1u ? ((r + qprev[i]) & m) : 0u;
                qprev[i] = q;
                v[i] = dequantize(q, P, bits);
            }
            if (pscan || P > 1) put(t, v);
            if (k + kTempAhead < nlist) fetch(list[k + kTempAhead], buf[j], bw[j]);
        }
    }
}

__global__ __launch_bounds__(256) void k_dec_temporal(DecPlan plan) {
    if (*plan.err) return;
    const uint32_t a = blockIdx.y;
    __shared__ uint16_t list[kModeLds];  // the scans to read: offset from tb, bit 15 for a P-scan
    __shared__ uint32_t scratch[8];
    const uint32_t A = plan.n_attrs, T = plan.n_scans;
    // the column's planes, width and precision from its first scan's record
    uint8_t* const out = (uint8_t*)plan.items[a].out;
    const uint32_t P = plan.items[a].P, wb = plan.items[a].wb;
    const bool all = P > 1;
    const uint32_t p0 = (blockIdx.x * 256 + threadIdx.x) * (4 / wb);
    if (blockIdx.x * 256 * (4 / wb) >= plan.npx) return;  // the grid is sized for 32-bit samples
    uint32_t qprev[4] = {0u, 0u, 0u, 0u};
    for (uint32_t tb = 0; tb < T; tb += kModeLds) {  // kModeLds scans at a time
        const uint32_t te = min(T, tb + kModeLds);
        uint32_t nlist = 0;  // the scans to read, in order
        for (uint32_t t0 = tb; t0 < te; t0 += 256) {
            const uint32_t t = t0 + threadIdx.x;
            uint32_t need = 0, pscan = 0;
            if (t < te) {
                pscan = plan.modes[t * A + a];
                need = all || pscan || (t + 1 < T && plan.modes[(t + 1) * A + a]);
            }
            uint32_t tot;
            const uint32_t o = block_excl_scan<256>(need, scratch, &tot);
            if (need) list[nlist + o] = (uint16_t)((t - tb) | (pscan ? 0x8000u : 0u));
            nlist += tot;
        }
        __syncthreads();
        if (p0 < plan.npx) {
            switch (wb) {
                case 4: dec_temporal_body<4>(plan, a, out, P, p0, list, tb, nlist, qprev); break;
                case 2: dec_temporal_body<2>(plan, a, out, P, p0, list, tb, nlist, qprev); break;
                default: dec_temporal_body<1>(plan, a, out, P, p0, list, tb, nlist, qprev); break;
            }
        }
        __syncthreads();
    }
}

// A decode's error words to host-mapped memory: the host reads them once the
// stream has synchronized, with no copy call.  Kernel parameters are plain
// pointers (an address-space qualifier would change the device symbol).
__global__ __launch_bounds__(64) void k_dec_report(const uint32_t* err, uint32_t* host, uint32_t n) {
    const uint32_t i = threadIdx.x;
    if (i < n) store_system((JG uint32_t*)host + i, ((const JG uint32_t*)err)[i]);
}

hipError_t launch_dec_report(const void* dev_err, void* host, uint32_t n, hipStream_t stream) {
    JIFFY_LAUNCH("k_dec_report", k_dec_report, dim3(1), dim3(64), stream, (const uint32_t*)dev_err, (uint32_t*)host, n);
    return hipGetLastError();
}

hipError_t launch_decode(const DecPlan& plan, hipStream_t stream) {
    if (plan.n_items == 0) return hipSuccess;
    JIFFY_LAUNCH("k_dec_parse", k_dec_parse, dim3(plan.n_items, plan.pwin + 1), dim3(256), stream, plan);
    const uint32_t mask_waves = min(kMaskWaves, div_up(plan.n_scans, (uint32_t)kMaskAhead));
    JIFFY_LAUNCH("k_dec_mask", k_dec_mask, dim3(div_up(2 * plan.nwords, 64), plan.n_attrs), dim3(64 * mask_waves),
                 stream, plan);
    JIFFY_LAUNCH("k_dec_scan", k_dec_scan, dim3(plan.n_items), dim3(1024), stream, plan);
    // records of 32-bit samples (32-bit rows), then 16-bit, then 8-bit ones (16-bit rows)
    const uint32_t n8 = plan.n_items - plan.n_wide - plan.n_w16;
    if (plan.n_wide)
        JIFFY_LAUNCH("k_dec_tiles_w32", (k_dec_tiles<uint32_t, 4>), dim3(plan.n_wide * plan.nvt), dim3(kDecThreads),
                     stream, plan, 0u, plan.n_wide);
    if (plan.n_w16)
        JIFFY_LAUNCH("k_dec_tiles_w16", (k_dec_tiles<uint16_t, 2>), dim3(plan.n_w16 * plan.nvt), dim3(kDecThreads),
                     stream, plan, plan.n_wide, plan.n_w16);
    if (n8)
        JIFFY_LAUNCH("k_dec_tiles_w8", (k_dec_tiles<uint16_t, 1>), dim3(n8 * plan.nvt), dim3(kDecThreads), stream,
                     plan, plan.n_wide + plan.n_w16, n8);
    if (plan.need_temporal)
        JIFFY_LAUNCH("k_dec_temporal", k_dec_temporal, dim3(div_up(plan.npx, 256), plan.n_attrs), dim3(256),
                     stream, plan);
    return hipGetLastError();
}

}  // namespace jiffy
