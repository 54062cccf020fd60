// Internal declarations shared by the Jiffy HIP kernels and the C-ABI host
// code.  gfx950 only: wave64, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// In the kernels' device compilation every pointer in the structures below
// points to global memory: declaring that lets the compiler emit global
// (not flat) loads and stores, which do not hold up LDS waits.  Host code
// sees plain pointers; the layout is the same.
#if defined(__HIP_DEVICE_COMPILE__) && defined(JIFFY_KERNEL_TU)
#define JG __attribute__((address_space(1)))
#else
#define JG
#endif

namespace jiffy {

constexpr int kWave = 64;
constexpr uint32_t kFrame = 128;            // values per packed frame (Sec. II: frames of 128)
constexpr uint32_t kSlotBytes = 640;        // a packed frame (at most 16 * 32 bytes), or a frame that
                                            // straddles tiles: its 128 residuals and their predecessor;
                                            // five 128-byte lines, so that a frame of up to 128 bytes
                                            // (most are) starts and ends in one line
constexpr uint32_t kFTile = 8192;           // pixels per encode / decode tile
constexpr uint32_t kNoFix = 0xFFFFFFFFu;    // a tile with no straddling frame to finish
constexpr uint32_t kAsmFrames = 64;         // frames copied into the stream by one workgroup
constexpr uint32_t kZstdBlockMax = 131072;  // largest Zstandard block (RFC 8878)
constexpr uint32_t kRleMinRun = 8;          // runs this long become RLE blocks
constexpr uint32_t kParseWin = 8192;        // mask-frame bytes per parsing window (one workgroup each)

// Error bits raised by kernels (ORed into a device word).
enum : uint32_t { kErrCorrupt = 1u, kErrCapacity = 2u, kErrStall = 4u };  // stall: a bounded wait ran out

inline __host__ __device__ uint32_t align4(uint32_t x) { return (x + 3u) & ~3u; }
inline __host__ __device__ uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// Worst-case size of the mask frame for n content bytes.
inline __host__ __device__ uint32_t frame_bound(uint32_t n) { return 16u + n + 4u * (n / kZstdBlockMax + 1u); }

// Division by a run-time invariant P (Granlund & Montgomery, "Division by
// invariant integers using multiplication", 1994): n / P = (t + ((n - t) >> s1)) >> s2,
// t = mulhi(m, n), exact for every 32-bit n.
struct Divisor {
    uint32_t P, magic, s1, s2, half_up;  // half_up = ceil(P / 2)
};

inline Divisor make_divisor(uint32_t P) {
    Divisor d;
    uint32_t l = 0;
    while ((1ull << l) < P) l++;
    d.P = P;
    d.magic = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - P)) / P + 1);
    d.s1 = l < 1 ? l : 1;
    d.s2 = l > 1 ? l - 1 : 0;
    d.half_up = P - P / 2;
    return d;
}

// One (scan, attribute) record to encode.
struct EncItem {
    const JG void* x;            // current scan, npx samples
    const JG void* xprev;        // previous scan (raw or quantized), or null
    JG void* qout;               // if set, the quantized scan is stored here
    JG uint64_t* vw;             // valid-sample words of this scan (bit = 1: nonzero)
    const JG uint64_t* vwprev;   // valid-sample words of the previous scan
    JG uint32_t* tfix;           // [ntiles] frame that starts in the tile and ends after it, or kNoFix
    JG uint64_t* tstat;          // [ntiles] look-back state of each kFTile tile
    JG uint32_t* tctr;           // k_enc_tiles ticket counter of the record
    JG uint32_t* blkinfo;        // [maxnb] b | n << 8 | B << 16
    JG uint32_t* blkoffs;        // [3 * maxnb] payload / position / high offsets
    JG uint8_t* slots;           // [maxnb * kSlotBytes] packed frames
    JG uint8_t* frame;           // mask frame staging
    JG uint32_t* segs;           // [seg_cap] frame segment starts (bit 31: run)
    JG uint32_t* segoff;         // [seg_cap] frame segment output offsets
    Divisor div;
    uint32_t npx, nwords, height, width;
    uint32_t wb, bits, attr, out_id;
    uint32_t has_prev, prev_quantized, mode_req, trial_rows;
    uint32_t maxnb, frame_cap, seg_cap, aligned16;
    uint32_t ntiles;
    uint32_t prev_item;          // the record in this launch whose valid words are vwprev, or kNoFix
};

// Per-record results of an encode.
struct EncRes {
    uint32_t N, nb, mode, flen;
    uint32_t pay, pos, high, rec_len;
    uint32_t nseg, pad0;
    uint64_t rec_off;
};

// One output buffer of an encode call (the whole stream, or one stream's
// records in a batch step).
struct EncOut {
    JG uint8_t* base;
    uint64_t cap;
    uint32_t first_item, n_items;
    uint32_t hdr_len;         // stream header + length table, or 0
    uint32_t n_scans, n_attrs, height, width;
    uint32_t ok;
    uint64_t len;
    uint64_t gbase;           // global prefix of the first record (scratch)
    uint8_t attr_wb[8];
    uint32_t attr_p[8];
};

// A decode tile: its values [kb, ke) and, for the payload, exception
// position and exception high-part sections, the first record word and the
// number of words that hold the tile's frames.
// A decode tile: values [kb, ke) of its record, pixels [ps, pe).  Tiles are
// cut at every kDecTileVals-th value and at the start of every
// kDecBlockPx-pixel block, so a tile holds at most kDecTileVals values (the
// frame rows of one workgroup) and at most kDecBlockPx pixels.
struct DecTile {
    uint32_t kb, ke, ps, pe;
};
constexpr uint32_t kDecTileVals = 8064;  // 63 frames: a tile's values touch at most 64 frames, one per quad of 256 threads
constexpr uint32_t kDecBlockPx = 65536;
// tiles a record of npx pixels can have, at most
inline __host__ __device__ uint32_t dec_tile_slots(uint32_t npx) {
    return (npx + kDecBlockPx - 1) / kDecBlockPx + (npx + kDecTileVals - 1) / kDecTileVals;
}

// One record to decode.
struct DecItem {
    const JG uint8_t* rec;
    uint32_t rec_len;
    JG void* out;                // [npx] output samples
    JG uint64_t* cw;             // unframed mask content (XOR form for a P-scan)
    JG uint64_t* vw;             // valid-sample words
    JG uint32_t* blkinfo;        // [maxnb]
    JG uint32_t* blkoffs;        // [3 * maxnb]
    JG uint2* tstart;            // [nvt + 1] each tile's first pixel and first value, then (npx, N)
    JG DecTile* tdesc;           // [nvt]
    JG uint32_t* tctr;           // k_dec_tiles ticket counter of the record
    JG uint64_t* status;         // [nvt] look-back state of each tile
    uint32_t npx, nwords, wb, bits;
    uint32_t attr, t, P, maxnb;
    uint32_t aligned16, pad0;
};

struct DecRes {
    uint32_t mode, flen, N, nb;
    uint32_t sec, pay_off, pos_off, high_off;
    uint32_t high_end, err, ntiles, pad0;
};

// ---- kernel timing hooks (jiffy_api.hip) ----------------------------------
void prof_begin(const char* name, hipStream_t stream);
void prof_end(hipStream_t stream);

#define JIFFY_LAUNCH(name, kern, grid, block, stream, ...)                 \
    do {                                                                     \
        ::jiffy::prof_begin(name, stream);                                   \
        hipLaunchKernelGGL(kern, grid, block, 0, stream, __VA_ARGS__);       \
        ::jiffy::prof_end(stream);                                           \
    } while (0)

// ---- kernel launchers (defined in the .hip files) -------------------------
struct EncPlan {
    const JG EncItem* items;     // device
    JG EncRes* res;              // device
    JG EncOut* outs;             // device
    JG uint32_t* err;            // device
    const JG uint32_t* ftile_item;  // device: item of each kFTile tile
    const JG uint32_t* ftile_first; // device: first kFTile tile of each item
    JG uint8_t* host_res;        // host-mapped results (or null): per output {u64 len, u32 ok, u32 -}, then
                                 // per record its mode (u32), then the error word, then per record its
                                 // length (u32)
    uint32_t ftpi;               // kFTile tiles per record when every record has the same size (the
                                 // maps above are then unused), else 0
    uint32_t n_items, n_outs, n_ftiles;
    uint32_t max_asm;         // max over items of ceil(maxnb / kAsmFrames)
    // the fused persistent launch (k_enc_fused); all zeroed by the plan upload
    JG uint32_t* fctl;           // [2] next work item, workgroups finished
    JG uint32_t* fdep;           // [4 * n_items] per record: decision made, tiles done, mask frame done, sizes done
    JG uint64_t* fstat;          // [n_items] look-back states of the record offsets
    JG uint32_t* ffix;           // [n_fix] tile-crossing frame groups done
    JG uint32_t* fout;           // [n_outs] output length known
    const JG uint32_t* fasm;     // [n_items + 1] first assembly item of each record (null: max_asm + 1 each)
    uint32_t n_fix, n_asm;       // tile-crossing frame groups, assembly items
};
hipError_t launch_encode(const EncPlan& plan, hipStream_t stream);
// The same encode as one persistent launch of `grid` workgroups.
hipError_t launch_encode_fused(const EncPlan& plan, uint32_t grid, hipStream_t stream);
// Workgroups of the fused launch one compute unit holds at once.
hipError_t fused_occupancy(int* per_cu);
constexpr uint32_t kFixGroup = 64;  // tile entries per group of tile-crossing frames

// One record copy of a brute-force encode (32 bytes; the job list lives in
// host-mapped memory).
struct CopyJob {
    uint64_t src, dst;
    uint32_t len, pad0;
    uint64_t pad1;
};
// Copies every job's bytes (device to device) with a kernel on `stream`.
hipError_t launch_copy_records(const CopyJob* host_jobs, uint32_t n, hipStream_t stream);

// Ablated codecs (Sec. IV-H, Table IV) and the run-length mask codec: byte
// sums per record r (scan-major, attribute-minor) in acc[8 r + k]: k = 0, 1, 2
// the packed bytes of every pixel's frames coded as values, differences
// (modulo 2^bits), ZigZag-coded differences; 3, 4 the packed bytes and the
// value count of the run-length section of the record's zero bitmask; 5, 6
// the same for that mask XOR the previous scan's (left 0 for the first scan).
struct AblAttr {
    const void* x;  // [T][H][W] samples of wb bytes
    uint32_t wb, bits;
    Divisor div;
};
struct AblArgs {
    AblAttr attr[8];
    uint32_t A, T, npx, nb;  // nb: frames per record
    uint32_t chunks;         // 64-frame chunks per record (workgroups of the level kernel per record)
    uint64_t* acc;           // [8 T A], zeroed by launch_ablate
    uint32_t* runs;          // npx words per workgroup of the run-length kernel
};
// Input standardization (Sec. III-A): points of n_scans scans, n_points
// each, into range and attribute images of height x width cells.
struct StdArgs {
    const float* xyz;            // [n_scans][n_points][3]
    const void* attr_in[8];      // [n_scans][n_points] each
    void* range;                 // [n_scans][cells] of range_bytes
    void* attr_out[8];           // [n_scans][cells] each
    uint64_t* keys;              // [n_scans][cells] workspace
    uint32_t n_scans, n_points, height, width, cells;
    uint32_t range_bytes, n_attrs;
    uint32_t attr_bytes[8];
    double elev_hi, span, unit, qmax;  // span = elev_hi - elev_lo; qmax = 2^(8 range_bytes) - 1
};
hipError_t launch_standardize(const StdArgs& g, hipStream_t stream);

// Zeroes acc, then launches the level kernel over every chunk of every
// record and the run-length kernel with `run_groups` workgroups.
hipError_t launch_ablate(const AblArgs& a, uint32_t run_groups, hipStream_t stream);

// Copies `bytes` (a multiple of 16) from host-mapped memory into device
// memory with a kernel on `stream` (no copy engine, so no cross-queue wait).
hipError_t launch_copy_in(const void* host, void* dev, size_t bytes, hipStream_t stream);

// One stream of a device-indexed decode (in host-mapped memory).
struct DecSrc {
    uint64_t src, len;  // device address and length of the stream
};

struct DecPlan {
    JG DecItem* items;
    JG DecRes* res;
    JG uint32_t* err;
    JG uint32_t* err2;           // errors found by k_dec_tiles
    JG uint8_t* modes;           // [n_items] 0 = I, 1 = P (written by the parse)
    JG uint8_t* ws;              // per-record workspace, item_stride bytes each
    uint64_t item_stride;
    uint32_t off_cw, off_vw;  // offsets of the mask words inside a record's workspace
    uint32_t n_items, n_scans, n_attrs;
    uint32_t nwords, npx;
    uint32_t nvt;             // decode tile slots per record (dec_tile_slots)
    const JG uint32_t* rec_list; // the records with 32-bit samples, then 16-bit, then 8-bit
    uint32_t n_wide;          // how many have 32-bit samples
    uint32_t n_w16;           // how many have 16-bit samples (they follow the 32-bit ones, the 8-bit ones follow them)
    uint32_t need_temporal;   // per-pixel pass over time needed
    uint32_t pwin;            // mask-frame windows per record (parse workgroups), at most
    uint32_t off_pstate;      // offset in a record's workspace of its window states ([pwin + 1] u64,
                              // then the window ticket counter)
    // Record index built on the device (null roff: the host filled rec /
    // rec_len).  The plan decodes n_src streams of src_attrs attributes and
    // n_scans scans each; the record of scan t, attribute a of stream s is
    // item t * n_attrs + s * src_attrs + a (n_attrs = n_src * src_attrs
    // columns).  srcs (host-mapped) gives each stream's bytes; its length
    // table follows a header of hdr_len bytes.  roff[r] = the record's
    // address, rlen[r] its length, or roff[r] = ~0 when its stream's index is
    // bad.
    const DecSrc* srcs;
    JG uint64_t* roff;
    JG uint32_t* rlen;
    uint32_t n_src, src_attrs;
    uint32_t hdr_len;         // header bytes before the table
    uint32_t hdr_check;       // compare them with hdr_words
    uint32_t hdr_words[(20 + 8 * 8) / 4];  // the expected header
};
hipError_t launch_decode(const DecPlan& plan, hipStream_t stream);

// Upload of the decode plan (as launch_copy_in), clearing of the parse
// window states and, when plan.roff is set, the device-side record index of
// every stream, in one launch.
hipError_t launch_dec_prepare(const void* host, void* dev, size_t bytes, const DecPlan& plan, hipStream_t stream);
// Copies n error words of a decode to host-mapped memory (system-scope stores).
hipError_t launch_dec_report(const void* dev_err, void* host, uint32_t n, hipStream_t stream);

}  // namespace jiffy
