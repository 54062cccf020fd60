// C ABI of the Jiffy codec (include/jiffy.h): argument checks, workspace
// layout, kernel planning, stream headers, resident stream state.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/jiffy.h"
#include "jiffy_internal.h"

using namespace jiffy;

// Device scratch of jiffy_encode_noalloc: that entry point's whole encoder
// workspace (plan image, results, per-record buffers), of a fixed size, one
// copy per device, held until the process ends.  Host code uses the address
// hipGetSymbolAddress returns for it on each device (DevCtx::scratch), never
// the array's own name.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

// Host staging of jiffy_encode_noalloc (ordinary static memory, not pinned):
// the plan image it copies to the device and the results it copies back.
constexpr size_t kNoallocUpBytes = 1u << 20;
constexpr size_t kNoallocResBytes = 256u << 10;
alignas(256) uint8_t g_noalloc_up[kNoallocUpBytes];
alignas(256) uint8_t g_noalloc_res[kNoallocResBytes];
std::mutex g_noalloc_mu;  // guards the two staging buffers (taken after a device's lock)

void prof_collect();

constexpr size_t kAlign = 256;
size_t al(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};
// Pinned host memory; d is its device address (kernels read the plan
// uploads and write the encode results through it, with system-scope
// accesses).
struct HostBuf {
    void* p = nullptr;
    void* d = nullptr;
    size_t cap = 0;
};

hipError_t grow(DevBuf& b, size_t need) {
    if (need <= b.cap) return hipSuccess;
    size_t cap = need + need / 4;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.cap = 0;
    }
    hipError_t e = hipMalloc(&b.p, cap);
    if (e == hipSuccess) b.cap = cap;
    return e;
}
hipError_t host_alloc(void** p, void** d, size_t bytes) {
    *p = *d = nullptr;
    hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    e = hipHostGetDevicePointer(d, *p, 0);
    if (e != hipSuccess) {
        (void)hipHostFree(*p);
        *p = *d = nullptr;
    }
    return e;
}
hipError_t grow(HostBuf& b, size_t need) {
    if (need <= b.cap) return hipSuccess;
    size_t cap = need + need / 4;
    if (b.p) {
        hipError_t e = hipHostFree(b.p);
        if (e != hipSuccess) return e;
        b.p = b.d = nullptr;
        b.cap = 0;
    }
    hipError_t e = host_alloc(&b.p, &b.d, cap);
    if (e == hipSuccess) b.cap = cap;
    return e;
}

// Per-device workspace.  Calls on one device are serialized by `mu` and
// synchronize their stream before returning, so the buffers are free again.
// Per device: the encoder's and the decoder's workspaces (separate, so that a
// decode leaves the encoder's plan image in place), the pinned host buffers,
// and the number of encoder plan uploads so far (a plan reused with no other
// upload since needs no upload).
struct DevCtx {
    std::mutex mu;
    DevBuf ws, ws_dec;
    DevBuf brute;     // the two staging streams of a brute-force encode
    DevBuf abl;       // jiffy_ablate: per-record sums and run-start lists
    DevBuf std_keys;  // jiffy_standardize: one 64-bit key per cell
    HostBuf up, down, res;
    HostBuf jobs;     // its record copy list
    uint64_t enc_gen = 0;
    uint8_t* scratch = nullptr;  // this device's copy of `scratch` (jiffy_encode_noalloc), once looked up
};
DevCtx g_ctx[64];

int current_device(int* dev) {
    if (hipGetDevice(dev) != hipSuccess || *dev < 0 || *dev >= 64) return JIFFY_E_DEVICE;
    return JIFFY_OK;
}

// Worst-case bytes of one record of npx samples of `bits` bits: header, mask
// frame, section header and every frame packed at full width, each part
// padded to 4 bytes.
uint64_t record_bound(uint64_t npx, uint32_t bits) {
    const uint64_t nm = (npx + 7) / 8, nb = (npx + kFrame - 1) / kFrame;
    return 12 + (16 + nm + 4 * (nm / kZstdBlockMax + 1)) + 3 + 4 + 3 * nb + 3 + nb * 16 * bits + 3;
}

bool layout_ok(const jiffy_layout* L) {
    if (!L || L->n_attrs < 1 || L->n_attrs > JIFFY_MAX_ATTRS || L->height == 0 || L->width == 0) return false;
    const uint64_t npx = (uint64_t)L->height * L->width;
    if (npx >= (1ull << 31)) return false;
    for (uint32_t a = 0; a < L->n_attrs; ++a) {
        const uint32_t wb = L->width_bytes[a];
        if (wb != 1 && wb != 2 && wb != 4) return false;
        if (L->precision[a] == 0) return false;
        // record lengths, section sizes and offsets are 32-bit fields of the stream
        if (record_bound(npx, 8 * wb) >= (1ull << 32)) return false;
    }
    return true;
}

uint32_t header_len(uint32_t A, uint32_t T) { return 20 + 8 * A + 4 * T * A; }

// The stream header without its length table (20 + 8 A bytes): magic,
// version 1, attribute count, height, width, scan count (0: records follow
// one another with no table), then per attribute its sample width and P.
void write_header(uint8_t* h, const jiffy_layout* L, uint32_t T) {
    const uint32_t A = L->n_attrs;
    memset(h, 0, 20 + 8 * A);
    memcpy(h, "JFY1", 4);
    h[4] = 1;
    h[6] = (uint8_t)A;
    memcpy(h + 8, &L->height, 4);
    memcpy(h + 12, &L->width, 4);
    memcpy(h + 16, &T, 4);
    for (uint32_t a = 0; a < A; ++a) {
        h[20 + 8 * a] = L->width_bytes[a];
        memcpy(h + 24 + 8 * a, &L->precision[a], 4);
    }
}

// ---------------------------------------------------------------------------
// encode planning
// ---------------------------------------------------------------------------
struct EncSpec {
    const void* x;
    const void* xprev;
    void* qout;
    uint64_t* vw_fixed;          // resident valid words (stream state) or null
    const uint64_t* vwprev_fixed;
    int prev_item;               // item whose valid words are the previous ones, or -1
    uint32_t H, W, wb, P, attr, out_id;
    uint32_t has_prev, prev_quantized, mode_req, trial_rows;
};

struct OutSpec {
    uint8_t* base;
    uint64_t cap;
    uint32_t first_item, n_items, hdr_len, n_scans;
    const jiffy_layout* layout;
};

struct EncResult {
    uint32_t err = 0;
    std::vector<uint64_t> lens;
    std::vector<uint8_t> ok;
    std::vector<uint8_t> modes;
    std::vector<uint32_t> rec_lens;
};

// Where everything of one encode launch sequence lives in its device
// workspace: [res][err][outs][items][tile maps] (the part uploaded from the
// host, from `err` on) then per record its buffers.
struct EncLayout {
    uint32_t n = 0, no = 0, n_ftiles = 0, max_asm = 1;
    uint32_t ftpi = 0;  // tiles per record when all records have the same size (no tile maps)
    uint32_t n_fix = 0, n_asm = 0;
    std::vector<uint32_t> ftile_first, asm_first;  // asm_first: empty when every record has max_asm + 1 items
    size_t o_res = 0, o_err = 0, o_outs = 0, o_items = 0, o_ftfirst = 0, o_ftitem = 0;
    size_t o_fctl = 0, o_fdep = 0, o_fstat = 0, o_ffix = 0, o_fout = 0, o_fasm = 0;
    size_t up_end = 0, total = 0;
    std::vector<size_t> o_vw, o_blk, o_slots, o_frame, o_segs;
    size_t up_bytes() const { return up_end - o_err; }
    // host results: per output len/ok, per record its mode, the error word, per record its length
    size_t res_bytes() const { return 16ull * no + 8ull * n + 4; }
};

EncLayout enc_layout(const std::vector<EncSpec>& specs, const std::vector<OutSpec>& outs) {
    EncLayout Lo;
    const uint32_t n = (uint32_t)specs.size(), no = (uint32_t)outs.size();
    Lo.n = n;
    Lo.no = no;
    Lo.ftile_first.resize(n);
    for (uint32_t r = 0; r < n; ++r) {
        Lo.ftile_first[r] = Lo.n_ftiles;
        const uint32_t npx = specs[r].H * specs[r].W;
        Lo.n_ftiles += div_up(npx, kFTile);
        const uint32_t asmg = div_up(div_up(npx, kFrame), kAsmFrames);
        if (asmg > Lo.max_asm) Lo.max_asm = asmg;
    }
    bool uniform = true;
    for (uint32_t r = 1; r < n; ++r)
        if (specs[r].H * specs[r].W != specs[0].H * specs[0].W) uniform = false;
    if (n && uniform) {
        Lo.ftpi = div_up(specs[0].H * specs[0].W, kFTile);
    }
    const uint32_t n_maps = Lo.ftpi ? 0u : n, n_ftmap = Lo.ftpi ? 0u : Lo.n_ftiles;
    // the fused launch's work items: assembly parts per record, tile-crossing frame groups
    Lo.n_fix = div_up(Lo.n_ftiles, kFixGroup);
    if (Lo.ftpi) {
        Lo.n_asm = n * (Lo.max_asm + 1);
    } else {
        Lo.asm_first.resize(n + 1);
        uint32_t a = 0;
        for (uint32_t r = 0; r < n; ++r) {
            Lo.asm_first[r] = a;
            a += 1 + div_up(div_up(specs[r].H * specs[r].W, kFrame), kAsmFrames);
        }
        Lo.asm_first[n] = a;
        Lo.n_asm = a;
    }
    size_t off = 0;
    Lo.o_res = off; off = al(off + sizeof(EncRes) * n);
    Lo.o_err = off; off = al(off + sizeof(uint32_t));
    Lo.o_outs = off; off = al(off + sizeof(EncOut) * no);
    Lo.o_items = off; off = al(off + sizeof(EncItem) * n);
    Lo.o_ftfirst = off; off = al(off + sizeof(uint32_t) * n_maps);
    Lo.o_ftitem = off; off = al(off + sizeof(uint32_t) * n_ftmap);
    Lo.o_fctl = off; off = al(off + 4 * sizeof(uint32_t));
    Lo.o_fdep = off; off = al(off + 4 * sizeof(uint32_t) * n);
    Lo.o_fstat = off; off = al(off + sizeof(uint64_t) * n);
    Lo.o_ffix = off; off = al(off + sizeof(uint32_t) * Lo.n_fix);
    Lo.o_fout = off; off = al(off + sizeof(uint32_t) * no);
    Lo.o_fasm = off; off = al(off + sizeof(uint32_t) * Lo.asm_first.size());
    Lo.up_end = off;
    Lo.o_vw.resize(n); Lo.o_blk.resize(n); Lo.o_slots.resize(n); Lo.o_frame.resize(n); Lo.o_segs.resize(n);
    for (uint32_t r = 0; r < n; ++r) {
        const uint32_t npx = specs[r].H * specs[r].W;
        const uint32_t nwords = div_up(npx, 64), maxnb = div_up(npx, kFrame), nm = div_up(npx, 8);
        Lo.o_vw[r] = off; off = al(off + (specs[r].vw_fixed ? 0 : 8ull * nwords));
        Lo.o_blk[r] = off; off = al(off + 4ull * maxnb * 4 + 4ull * div_up(npx, kFTile)) + al(8ull * div_up(npx, kFTile) + 4);
        Lo.o_slots[r] = off; off = al(off + (size_t)kSlotBytes * maxnb);
        Lo.o_frame[r] = off; off = al(off + frame_bound(nm));
        Lo.o_segs[r] = off; off = al(off + 8ull * (nm / 4 + 4));
    }
    Lo.total = off;
    return Lo;
}

// The host image of the uploaded part (records, outputs, tile maps, zeroed
// error word and output states), written into `up` (up_bytes() bytes).
void enc_fill(const EncLayout& Lo, const std::vector<EncSpec>& specs, const std::vector<OutSpec>& outs,
              uint8_t* dev, uint8_t* up) {
    const uint32_t n = Lo.n, no = Lo.no;
    memset(up, 0, Lo.up_bytes());
    auto U = [&](size_t o) { return up + (o - Lo.o_err); };
    EncOut* hout = (EncOut*)U(Lo.o_outs);
    for (uint32_t k = 0; k < no; ++k) {
        EncOut& o = hout[k];
        o.base = outs[k].base;
        o.cap = outs[k].cap;
        o.first_item = outs[k].first_item;
        o.n_items = outs[k].n_items;
        o.hdr_len = outs[k].hdr_len;
        o.n_scans = outs[k].n_scans;
        const jiffy_layout* L = outs[k].layout;
        o.n_attrs = L->n_attrs;
        o.height = L->height;
        o.width = L->width;
        for (uint32_t a = 0; a < L->n_attrs; ++a) {
            o.attr_wb[a] = L->width_bytes[a];
            o.attr_p[a] = L->precision[a];
        }
    }
    EncItem* hit = (EncItem*)U(Lo.o_items);
    for (uint32_t r = 0; r < n; ++r) {
        const EncSpec& s = specs[r];
        EncItem& it = hit[r];
        const uint32_t npx = s.H * s.W;
        it.x = s.x;
        it.xprev = s.xprev;
        it.qout = s.qout;
        it.vw = s.vw_fixed ? s.vw_fixed : (uint64_t*)(dev + Lo.o_vw[r]);
        if (s.vwprev_fixed) it.vwprev = s.vwprev_fixed;
        else if (s.prev_item >= 0) it.vwprev = specs[s.prev_item].vw_fixed ? specs[s.prev_item].vw_fixed
                                                                         : (uint64_t*)(dev + Lo.o_vw[s.prev_item]);
        else it.vwprev = nullptr;
        const uint32_t maxnb = div_up(npx, kFrame), nm = div_up(npx, 8);
        uint32_t* blk = (uint32_t*)(dev + Lo.o_blk[r]);
        const uint32_t nft = div_up(npx, kFTile);
        it.blkinfo = blk;
        it.blkoffs = blk + maxnb;
        it.tfix = blk + 4 * maxnb;
        it.tstat = (uint64_t*)(dev + Lo.o_blk[r] + al(4ull * maxnb * 4 + 4ull * nft));
        it.tctr = (uint32_t*)(it.tstat + nft);
        it.ntiles = nft;
        it.slots = dev + Lo.o_slots[r];
        it.frame = dev + Lo.o_frame[r];
        it.seg_cap = nm / 4 + 4;
        it.segs = (uint32_t*)(dev + Lo.o_segs[r]);
        it.segoff = it.segs + it.seg_cap;
        it.div = make_divisor(s.P);
        it.npx = npx;
        it.nwords = div_up(npx, 64);
        it.height = s.H;
        it.width = s.W;
        it.wb = s.wb;
        it.bits = 8 * s.wb;
        it.attr = s.attr;
        it.out_id = s.out_id;
        it.has_prev = s.has_prev;
        it.prev_quantized = s.prev_quantized;
        it.mode_req = s.mode_req;
        it.trial_rows = s.trial_rows;
        it.maxnb = maxnb;
        it.frame_cap = frame_bound(nm);
        bool al16 = ((uintptr_t)s.x % 16 == 0) && (!s.xprev || (uintptr_t)s.xprev % 16 == 0) &&
                    (!s.qout || (uintptr_t)s.qout % 16 == 0);
        it.aligned16 = al16 ? 1u : 0u;
        it.prev_item = (!s.vwprev_fixed && s.prev_item >= 0) ? (uint32_t)s.prev_item : kNoFix;
    }
    if (!Lo.asm_first.empty())
        memcpy(U(Lo.o_fasm), Lo.asm_first.data(), sizeof(uint32_t) * Lo.asm_first.size());
    if (Lo.ftpi) return;  // tiles are found by division
    uint32_t* hftf = (uint32_t*)U(Lo.o_ftfirst);
    uint32_t* hfti = (uint32_t*)U(Lo.o_ftitem);
    for (uint32_t r = 0; r < n; ++r) {
        const uint32_t npx = specs[r].H * specs[r].W;
        hftf[r] = Lo.ftile_first[r];
        for (uint32_t k = 0, nt = div_up(npx, kFTile); k < nt; ++k) hfti[Lo.ftile_first[r] + k] = r;
    }
}

EncPlan enc_plan(const EncLayout& Lo, uint8_t* dev, uint8_t* host_res) {
    EncPlan plan;
    plan.host_res = host_res;
    plan.ftpi = Lo.ftpi;
    plan.items = (const EncItem*)(dev + Lo.o_items);
    plan.res = (EncRes*)(dev + Lo.o_res);
    plan.outs = (EncOut*)(dev + Lo.o_outs);
    plan.err = (uint32_t*)(dev + Lo.o_err);
    plan.ftile_item = (const uint32_t*)(dev + Lo.o_ftitem);
    plan.ftile_first = (const uint32_t*)(dev + Lo.o_ftfirst);
    plan.n_ftiles = Lo.n_ftiles;
    plan.n_items = Lo.n;
    plan.n_outs = Lo.no;
    plan.max_asm = Lo.max_asm;
    plan.fctl = (uint32_t*)(dev + Lo.o_fctl);
    plan.fdep = (uint32_t*)(dev + Lo.o_fdep);
    plan.fstat = (uint64_t*)(dev + Lo.o_fstat);
    plan.ffix = (uint32_t*)(dev + Lo.o_ffix);
    plan.fout = (uint32_t*)(dev + Lo.o_fout);
    plan.fasm = Lo.asm_first.empty() ? nullptr : (const uint32_t*)(dev + Lo.o_fasm);
    plan.n_fix = Lo.n_fix;
    plan.n_asm = Lo.n_asm;
    return plan;
}

// Everything one call enqueues (also what a batch captures in its graph):
// the upload of the plan image by a kernel reading `up_dev` (the device
// address of the host image), then the kernels; k_enc_offsets writes the
// lengths and modes to the host results.
// The encode's launch configuration (the autotuner's knobs; jiffy_set_tuning):
// the kernel chain, or one fused persistent launch of wgs_per_cu workgroups
// per compute unit (0: as many as one holds).
jiffy_tuning g_tuning = {0u, 0u};
std::mutex g_tune_mu;
struct FusedShape {
    int cus = 0, per_cu = 0;  // looked up once per device
};
FusedShape g_fshape[64];

// Workgroups of a fused launch on the current device under tuning t, or 0
// for the kernel chain (also when the device cannot be queried).
uint32_t fused_grid(const jiffy_tuning& t) {
    if (!t.fused) return 0;
    int dev;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    FusedShape& f = g_fshape[dev];
    if (!f.cus) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            fused_occupancy(&per) != hipSuccess || cus <= 0 || per <= 0)
            return 0;
        f.per_cu = per;
        f.cus = cus;
    }
    const uint32_t per = t.wgs_per_cu ? std::min<uint32_t>(t.wgs_per_cu, (uint32_t)f.per_cu) : (uint32_t)f.per_cu;
    return per * (uint32_t)f.cus;
}

jiffy_tuning current_tuning() {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    return g_tuning;
}

hipError_t enc_enqueue(const EncLayout& Lo, const EncPlan& plan, uint8_t* dev, const void* up_dev, hipStream_t stream,
                       bool upload = true, uint32_t fgrid = 0) {
    if (upload) {
        hipError_t e = launch_copy_in(up_dev, dev + Lo.o_err, Lo.up_bytes(), stream);
        if (e != hipSuccess) return e;
    }
    return fgrid ? launch_encode_fused(plan, fgrid, stream) : launch_encode(plan, stream);
}

// Results k_enc_offsets wrote to host memory.
void enc_results(const EncLayout& Lo, const uint8_t* hres, EncResult& result) {
    memcpy(&result.err, hres + 16ull * Lo.no + 4ull * Lo.n, 4);
    result.lens.resize(Lo.no);
    result.ok.resize(Lo.no);
    result.modes.resize(Lo.n);
    for (uint32_t k = 0; k < Lo.no; ++k) {
        uint64_t len;
        uint32_t ok;
        memcpy(&len, hres + 16 * k, 8);
        memcpy(&ok, hres + 16 * k + 8, 4);
        result.lens[k] = len;
        result.ok[k] = (uint8_t)ok;
    }
    const uint32_t* m = (const uint32_t*)(hres + 16ull * Lo.no);
    result.rec_lens.resize(Lo.n);
    for (uint32_t r = 0; r < Lo.n; ++r) {
        result.modes[r] = (uint8_t)m[r];
        result.rec_lens[r] = m[Lo.n + 1 + r];
    }
}

// An encode plan: the layout and the plan image in `up`, valid for the
// workspace at `ws`.
struct EncPrepared {
    bool valid = false;
    void* ws = nullptr;
    uint64_t gen = 0;  // the device's upload count when this plan's image was last uploaded
    EncLayout Lo;
};

int enc_prepare(DevCtx& ctx, HostBuf& up, const std::vector<EncSpec>& specs, const std::vector<OutSpec>& outs,
                EncPrepared& P) {
    P.valid = false;
    ++ctx.enc_gen;  // the workspace may move or be rewritten: no earlier image is known to be there
    P.Lo = enc_layout(specs, outs);
    if (grow(ctx.ws, P.Lo.total) != hipSuccess) return JIFFY_E_DEVICE;
    if (grow(up, P.Lo.up_bytes()) != hipSuccess) return JIFFY_E_DEVICE;
    enc_fill(P.Lo, specs, outs, (uint8_t*)ctx.ws.p, (uint8_t*)up.p);
    P.ws = ctx.ws.p;
    P.valid = true;
    return JIFFY_OK;
}

// upload = false: the plan's image is still in the workspace (nothing was
// uploaded or prepared on this device since), so the kernels start at once.
int enc_execute(DevCtx& ctx, const HostBuf& up, const EncPrepared& P, hipStream_t stream, EncResult& result,
                bool upload = true) {
    if (grow(ctx.res, P.Lo.res_bytes()) != hipSuccess) return JIFFY_E_DEVICE;
    uint8_t* dev = (uint8_t*)ctx.ws.p;
    const EncPlan plan = enc_plan(P.Lo, dev, (uint8_t*)ctx.res.d);
    if (upload) ++ctx.enc_gen;
    // the fused launch needs its control words zeroed by the upload of the plan image
    const uint32_t fgrid = fused_grid(current_tuning());
    if (fgrid) {
        if (!upload) ++ctx.enc_gen;
        upload = true;
    }
    if (enc_enqueue(P.Lo, plan, dev, up.d, stream, upload, fgrid) != hipSuccess) return JIFFY_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
    prof_collect();
    enc_results(P.Lo, (const uint8_t*)ctx.res.p, result);
    return (result.err & kErrStall) ? JIFFY_E_DEVICE : JIFFY_OK;
}

int run_encode(DevCtx& ctx, const std::vector<EncSpec>& specs, const std::vector<OutSpec>& outs, hipStream_t stream,
               EncResult& result) {
    EncPrepared P;
    if (int rc = enc_prepare(ctx, ctx.up, specs, outs, P)) return rc;
    return enc_execute(ctx, ctx.up, P, stream, result);
}

// The records of one scan sequence (jiffy_encode): scan t of attribute a
// predicts from scan t-1 of the same plane; one output, the whole stream.
void sequence_specs(const jiffy_layout* L, uint32_t mode, uint32_t K, uint32_t T, const void* const* d_planes,
                    void* d_out, size_t cap, std::vector<EncSpec>& specs, std::vector<OutSpec>& outs) {
    const uint32_t A = L->n_attrs;
    const size_t npx = (size_t)L->height * L->width;
    specs.resize((size_t)T * A);
    for (uint32_t t = 0; t < T; ++t) {
        for (uint32_t a = 0; a < A; ++a) {
            EncSpec& s = specs[(size_t)t * A + a];
            const size_t step = npx * L->width_bytes[a];
            s.x = (const uint8_t*)d_planes[a] + t * step;
            s.xprev = t ? (const uint8_t*)d_planes[a] + (t - 1) * step : nullptr;
            s.qout = nullptr;
            s.vw_fixed = nullptr;
            s.vwprev_fixed = nullptr;
            s.prev_item = t ? (int)((t - 1) * A + a) : -1;
            s.H = L->height;
            s.W = L->width;
            s.wb = L->width_bytes[a];
            s.P = L->precision[a];
            s.attr = a;
            s.out_id = 0;
            s.has_prev = t ? 1u : 0u;
            s.prev_quantized = 0;
            s.mode_req = mode;
            s.trial_rows = K;
        }
    }
    outs.assign(1, OutSpec{(uint8_t*)d_out, cap, 0, T * A, header_len(A, T), T, L});
}

// Arguments of jiffy_encode / jiffy_encode_noalloc; JIFFY_OK or JIFFY_E_INVALID.
int check_encode_args(const jiffy_layout* L, const jiffy_options* opt, uint32_t T, const void* const* d_planes,
                      void* d_out, size_t* h_out_len, uint32_t max_mode = JIFFY_MODE_P_ONLY) {
    if (!layout_ok(L) || !h_out_len || !d_out || (uintptr_t)d_out % 4) return JIFFY_E_INVALID;
    if (opt && opt->mode > max_mode) return JIFFY_E_INVALID;
    if ((uint64_t)T * L->n_attrs > (1u << 24)) return JIFFY_E_INVALID;
    if (T && !d_planes) return JIFFY_E_INVALID;
    for (uint32_t a = 0; T && a < L->n_attrs; ++a)
        if (!d_planes[a] || (uintptr_t)d_planes[a] % L->width_bytes[a]) return JIFFY_E_INVALID;
    return JIFFY_OK;
}

// Sec. III-E, the brute-force choice: every record is coded as an I- and
// as a P-record in one launch sequence (two staging streams of records),
// the smaller of each pair is kept (equal sizes: the I-record; the first
// scan has no P-record), and a copy kernel assembles the stream: header
// and length table, then the kept records in order.
int encode_brute(DevCtx& ctx, const jiffy_layout* L, uint32_t K, uint32_t T, const void* const* d_planes,
                 void* d_out, size_t cap, size_t* h_out_len, uint8_t* h_modes, hipStream_t stream) {
    const uint32_t A = L->n_attrs, n = T * A;
    const size_t hl = header_len(A, T);
    size_t body = 0;
    for (uint32_t a = 0; a < A; ++a) body += record_bound((uint64_t)L->height * L->width, 8u * L->width_bytes[a]) * T;
    if (grow(ctx.brute, 2 * al(body)) != hipSuccess) return JIFFY_E_DEVICE;
    uint8_t* stage[2] = {(uint8_t*)ctx.brute.p, (uint8_t*)ctx.brute.p + al(body)};
    std::vector<EncSpec> specs, half;
    std::vector<OutSpec> outs(2), o1;
    for (uint32_t kind = 0; kind < 2; ++kind) {  // 0: every record an I-record, 1: a P-record where possible
        sequence_specs(L, kind ? JIFFY_MODE_P_ONLY : JIFFY_MODE_I_ONLY, K, T, d_planes, stage[kind], body, half, o1);
        for (EncSpec& e : half) {
            e.out_id = kind;
            if (e.prev_item >= 0) e.prev_item += (int)(kind * n);
        }
        specs.insert(specs.end(), half.begin(), half.end());
        outs[kind] = OutSpec{stage[kind], body, kind * n, n, 0, T, L};
    }
    EncResult res;
    if (int rc = run_encode(ctx, specs, outs, stream, res)) return rc;
    if (!res.ok[0] || !res.ok[1]) return JIFFY_E_DEVICE;  // the staging streams hold every record's bound
    // the kept records and their places
    if (grow(ctx.jobs, sizeof(CopyJob) * (n + 1) + hl) != hipSuccess) return JIFFY_E_DEVICE;
    CopyJob* jobs = (CopyJob*)ctx.jobs.p;
    uint8_t* hdr = (uint8_t*)ctx.jobs.p + sizeof(CopyJob) * (n + 1);
    write_header(hdr, L, T);
    uint64_t src[2] = {0, 0}, dst = hl;
    for (uint32_t r = 0; r < n; ++r) {
        const uint32_t li = res.rec_lens[r], lp = res.rec_lens[n + r];
        const bool p = r >= A && lp < li;
        const uint32_t len = p ? lp : li;
        memcpy(hdr + 20 + 8 * A + 4 * r, &len, 4);
        jobs[r] = CopyJob{(uint64_t)(uintptr_t)(stage[p ? 1 : 0] + src[p ? 1 : 0]), (uint64_t)(uintptr_t)d_out + dst,
                          len, 0, 0};
        if (h_modes) h_modes[r] = p ? 1 : 0;
        src[0] += li;
        src[1] += lp;
        dst += len;
    }
    *h_out_len = dst;
    if (dst > cap) return JIFFY_E_CAPACITY;
    ++ctx.enc_gen;  // the encoder workspace now holds this call's plan, not a cached one
    if (hipMemcpyAsync(d_out, hdr, hl, hipMemcpyHostToDevice, stream) != hipSuccess) return JIFFY_E_DEVICE;
    if (launch_copy_records((const CopyJob*)ctx.jobs.d, n, stream) != hipSuccess) return JIFFY_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
    prof_collect();
    return JIFFY_OK;
}

// The last jiffy_encode's arguments and plan (per device): a call with the
// same arguments on the same workspace reuses the plan image.
struct EncKey {
    jiffy_layout L;
    uint32_t mode, K, T, pad;
    const void* planes[JIFFY_MAX_ATTRS];
    void* out;
    size_t cap;
};
struct EncCache {
    EncKey key;
    EncPrepared prep;
    HostBuf up;
};
EncCache g_enc_cache[64];
// The same for jiffy_encode_many, keyed by every stream's planes and output.
struct EncManyCache {
    std::vector<uint64_t> key;
    EncPrepared prep;
    HostBuf up;
};
EncManyCache g_enc_many_cache[64];

// ---------------------------------------------------------------------------
// header parsing (host memory)
// ---------------------------------------------------------------------------
uint32_t rd32(const uint8_t* p) { return p[0] | (p[1] << 8) | (p[2] << 16) | ((uint32_t)p[3] << 24); }
uint16_t rd16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }

int parse_header(const uint8_t* h, size_t len, jiffy_layout* L, uint32_t* T, size_t* hdr) {
    if (len < 20 || memcmp(h, "JFY1", 4) != 0 || rd16(h + 4) != 1) return JIFFY_E_CORRUPT;
    const uint32_t A = rd16(h + 6);
    if (A < 1 || A > JIFFY_MAX_ATTRS || len < 20 + 8ull * A) return JIFFY_E_CORRUPT;
    memset(L, 0, sizeof *L);
    L->n_attrs = A;
    L->height = rd32(h + 8);
    L->width = rd32(h + 12);
    *T = rd32(h + 16);
    for (uint32_t a = 0; a < A; ++a) {
        const uint8_t* d = h + 20 + 8 * a;
        if (d[1] || d[2] || d[3]) return JIFFY_E_CORRUPT;
        L->width_bytes[a] = d[0];
        L->precision[a] = rd32(d + 4);
    }
    if (!layout_ok(L)) return JIFFY_E_CORRUPT;
    *hdr = 20 + 8 * A;
    return JIFFY_OK;
}

// ---------------------------------------------------------------------------
// kernel timing: events around each launch, read back after the call's sync
// ---------------------------------------------------------------------------
struct ProfEntry {
    const char* name;
    hipEvent_t start, stop;
};
struct ProfTotal {
    char name[32];
    double ms;
    uint32_t launches;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfEntry> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
std::vector<ProfTotal> g_prof_totals;

hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// called after the stream of the pending launches has been synchronized
void prof_collect() {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    for (ProfEntry& p : g_prof_pending) {
        float ms = 0.f;
        if (p.start && p.stop && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            ProfTotal* t = nullptr;
            for (ProfTotal& x : g_prof_totals)
                if (strncmp(x.name, p.name, sizeof x.name) == 0) t = &x;
            if (!t) {
                g_prof_totals.push_back(ProfTotal{});
                t = &g_prof_totals.back();
                strncpy(t->name, p.name, sizeof t->name - 1);
            }
            t->ms += ms;
            t->launches++;
        }
        if (p.start) g_prof_pool.push_back(p.start);
        if (p.stop) g_prof_pool.push_back(p.stop);
    }
    g_prof_pending.clear();
}

}  // namespace

namespace jiffy {
// launches go into a graph, or the call may not create events: no timing events
thread_local bool t_no_events = false;

void prof_begin(const char* name, hipStream_t stream) {
    if (t_no_events) return;
    std::lock_guard<std::mutex> lock(g_prof_mu);
    if (!g_prof_on) return;
    ProfEntry e{name, prof_event(), prof_event()};
    if (e.start) (void)hipEventRecord(e.start, stream);
    g_prof_pending.push_back(e);
}
void prof_end(hipStream_t stream) {
    if (t_no_events) return;
    std::lock_guard<std::mutex> lock(g_prof_mu);
    if (!g_prof_on || g_prof_pending.empty()) return;
    ProfEntry& e = g_prof_pending.back();
    if (e.stop) (void)hipEventRecord(e.stop, stream);
}
}  // namespace jiffy

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int jiffy_profile_enable(int enable) {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof_on = enable != 0;
    if (g_prof_on) g_prof_totals.clear();
    return JIFFY_OK;
}

int jiffy_profile_read(uint32_t max_kernels, char* names, double* total_ms, uint32_t* launches) {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    const uint32_t n = (uint32_t)g_prof_totals.size();
    for (uint32_t k = 0; k < n && k < max_kernels; ++k) {
        if (names) memcpy(names + 32 * k, g_prof_totals[k].name, 32);
        if (total_ms) total_ms[k] = g_prof_totals[k].ms;
        if (launches) launches[k] = g_prof_totals[k].launches;
    }
    return (int)n;
}

int jiffy_set_tuning(const jiffy_tuning* t) {
    if (!t || t->fused > 1 || t->wgs_per_cu > 64) return JIFFY_E_INVALID;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuning = *t;
    return JIFFY_OK;
}

int jiffy_get_tuning(jiffy_tuning* t, uint32_t* max_wgs_per_cu) {
    if (t) *t = current_tuning();
    if (max_wgs_per_cu) {
        *max_wgs_per_cu = 0;
        int dev;
        if (current_device(&dev)) return JIFFY_E_DEVICE;
        const jiffy_tuning probe = {1u, 0u};
        if (!fused_grid(probe)) return JIFFY_E_DEVICE;
        *max_wgs_per_cu = (uint32_t)g_fshape[dev].per_cu;
    }
    return JIFFY_OK;
}

const char* jiffy_status_string(int s) {
    switch (s) {
        case JIFFY_OK: return "ok";
        case JIFFY_E_INVALID: return "invalid argument";
        case JIFFY_E_CAPACITY: return "output buffer too small";
        case JIFFY_E_CORRUPT: return "corrupt stream";
        case JIFFY_E_DEVICE: return "HIP runtime error";
        case JIFFY_E_SHAPE: return "planes do not match the stream";
        case JIFFY_E_SCRATCH: return "request exceeds the fixed scratch buffer of jiffy_encode_noalloc";
        default: return "unknown status";
    }
}

size_t jiffy_encode_bound(const jiffy_layout* L, uint32_t n_scans) {
    if (!layout_ok(L)) return 0;
    const size_t npx = (size_t)L->height * L->width;
    size_t total = header_len(L->n_attrs, n_scans);
    for (uint32_t a = 0; a < L->n_attrs; ++a) total += record_bound(npx, 8u * L->width_bytes[a]) * n_scans;
    return total;
}

int jiffy_encode(const jiffy_layout* L, const jiffy_options* opt, uint32_t T, const void* const* d_planes,
                 void* d_out, size_t cap, size_t* h_out_len, uint8_t* h_modes, hipStream_t stream) {
    if (int rc = check_encode_args(L, opt, T, d_planes, d_out, h_out_len, JIFFY_MODE_BRUTE)) return rc;
    const uint32_t mode = opt ? opt->mode : 0;
    const uint32_t K = (opt && opt->trial_rows) ? opt->trial_rows : 4;
    const uint32_t A = L->n_attrs;
    int dev;
    if (current_device(&dev)) return JIFFY_E_DEVICE;
    DevCtx& ctx = g_ctx[dev];
    std::lock_guard<std::mutex> lock(ctx.mu);
    if (mode == JIFFY_MODE_BRUTE && T) return encode_brute(ctx, L, K, T, d_planes, d_out, cap, h_out_len, h_modes, stream);
    if (T == 0) {
        // a header with no records
        const uint32_t hl = header_len(A, 0);
        *h_out_len = hl;
        if (cap < hl) return JIFFY_E_CAPACITY;
        if (grow(ctx.up, hl) != hipSuccess) return JIFFY_E_DEVICE;
        uint8_t* h = (uint8_t*)ctx.up.p;
        write_header(h, L, 0);
        if (hipMemcpyAsync(d_out, h, hl, hipMemcpyHostToDevice, stream) != hipSuccess) return JIFFY_E_DEVICE;
        if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
        return JIFFY_OK;
    }
    EncCache& C = g_enc_cache[dev];
    EncKey key;
    memset(&key, 0, sizeof key);
    key.L = *L;
    key.mode = mode;
    key.K = K;
    key.T = T;
    for (uint32_t a = 0; a < A; ++a) key.planes[a] = d_planes[a];
    key.out = d_out;
    key.cap = cap;
    EncResult res;
    if (C.prep.valid && C.prep.ws == ctx.ws.p && memcmp(&key, &C.key, sizeof key) == 0) {
        const bool resident = C.prep.gen == ctx.enc_gen;  // no other upload or plan on this device since
        if (int rc = enc_execute(ctx, C.up, C.prep, stream, res, !resident)) return rc;
        C.prep.gen = ctx.enc_gen;
        *h_out_len = res.lens[0];
        if (!res.ok[0]) return JIFFY_E_CAPACITY;
        if (h_modes) memcpy(h_modes, res.modes.data(), (size_t)T * A);
        return JIFFY_OK;
    }
    std::vector<EncSpec> specs;
    std::vector<OutSpec> outs;
    sequence_specs(L, mode, K, T, d_planes, d_out, cap, specs, outs);
    if (int rc = enc_prepare(ctx, C.up, specs, outs, C.prep)) return rc;
    C.key = key;
    if (int rc = enc_execute(ctx, C.up, C.prep, stream, res)) return rc;
    C.prep.gen = ctx.enc_gen;
    *h_out_len = res.lens[0];
    if (!res.ok[0]) return JIFFY_E_CAPACITY;
    if (h_modes) memcpy(h_modes, res.modes.data(), (size_t)T * A);
    return JIFFY_OK;
}

int jiffy_encode_many(const jiffy_layout* L, const jiffy_options* opt, uint32_t n_streams, uint32_t T,
                      const void* const* const* d_planes, void* const* d_outs, const size_t* caps, size_t* h_out_lens,
                      uint8_t* h_modes, hipStream_t stream) {
    if (!layout_ok(L) || !h_out_lens || (n_streams && (!d_planes || !d_outs || !caps))) return JIFFY_E_INVALID;
    if (opt && opt->mode > JIFFY_MODE_P_ONLY) return JIFFY_E_INVALID;
    if (n_streams == 0) return JIFFY_OK;
    const uint32_t A = L->n_attrs;
    if ((uint64_t)T * A * n_streams > (1u << 24) || T == 0) return JIFFY_E_INVALID;
    for (uint32_t s = 0; s < n_streams; ++s)
        if (int rc = check_encode_args(L, opt, T, d_planes[s], d_outs[s], h_out_lens)) return rc;
    const uint32_t mode = opt ? opt->mode : 0;
    const uint32_t K = (opt && opt->trial_rows) ? opt->trial_rows : 4;
    int dev;
    if (current_device(&dev)) return JIFFY_E_DEVICE;
    DevCtx& ctx = g_ctx[dev];
    std::lock_guard<std::mutex> lock(ctx.mu);
    // the plan of the last call is reused when the arguments and the workspace are the same
    std::vector<uint64_t> key(sizeof(jiffy_layout) / 8 + 1, 0);
    memcpy(key.data(), L, sizeof *L);
    key.push_back(mode);
    key.push_back(K);
    key.push_back(T);
    for (uint32_t s = 0; s < n_streams; ++s) {
        for (uint32_t a = 0; a < A; ++a) key.push_back((uint64_t)(uintptr_t)d_planes[s][a]);
        key.push_back((uint64_t)(uintptr_t)d_outs[s]);
        key.push_back(caps[s]);
    }
    EncManyCache& C = g_enc_many_cache[dev];
    EncResult res;
    const bool hit = C.prep.valid && C.prep.ws == ctx.ws.p && key == C.key;
    if (hit) {
        if (int rc = enc_execute(ctx, C.up, C.prep, stream, res, C.prep.gen != ctx.enc_gen)) return rc;
    } else {
        std::vector<EncSpec> specs, half;
        std::vector<OutSpec> outs, o1;
        const uint32_t per = T * A;
        for (uint32_t s = 0; s < n_streams; ++s) {
            sequence_specs(L, mode, K, T, d_planes[s], d_outs[s], caps[s], half, o1);
            for (EncSpec& e : half) {
                e.out_id = s;
                if (e.prev_item >= 0) e.prev_item += (int)(s * per);
            }
            specs.insert(specs.end(), half.begin(), half.end());
            o1[0].first_item = s * per;
            outs.push_back(o1[0]);
        }
        if (int rc = enc_prepare(ctx, C.up, specs, outs, C.prep)) return rc;
        C.key = std::move(key);
        if (int rc = enc_execute(ctx, C.up, C.prep, stream, res)) return rc;
    }
    C.prep.gen = ctx.enc_gen;
    int rc = JIFFY_OK;
    for (uint32_t s = 0; s < n_streams; ++s) {
        h_out_lens[s] = res.lens[s];
        if (!res.ok[s]) rc = JIFFY_E_CAPACITY;
    }
    if (h_modes) memcpy(h_modes, res.modes.data(), (size_t)n_streams * T * A);
    return rc;
}

int jiffy_standardize(const jiffy_grid* G, uint32_t n_scans, uint32_t n_points, const float* d_xyz,
                      const void* const* d_attrs_in, void* d_range, void* const* d_attrs_out, hipStream_t stream) {
    static_assert(JIFFY_MAX_ATTRS <= 8, "StdArgs holds 8 attributes");
    if (!G || G->height == 0 || G->width == 0 || G->n_attrs > JIFFY_MAX_ATTRS) return JIFFY_E_INVALID;
    const uint32_t rb = G->range_bytes;
    if (rb != 1 && rb != 2 && rb != 4) return JIFFY_E_INVALID;
    if (!(G->elev_lo < G->elev_hi) || !(G->range_unit > 0.0) || !(G->elev_hi - G->elev_lo < 1e300) ||
        !(G->range_unit < 1e300))
        return JIFFY_E_INVALID;
    const uint64_t cells = (uint64_t)G->height * G->width;
    if (cells >= (1ull << 32)) return JIFFY_E_INVALID;
    const uint64_t tot_cells = cells * n_scans, tot_pts = (uint64_t)n_points * n_scans;
    if (tot_cells > (1ull << 38) || tot_pts > (1ull << 38)) return JIFFY_E_INVALID;
    if (n_scans == 0) return JIFFY_OK;
    if (!d_range || (uintptr_t)d_range % rb) return JIFFY_E_INVALID;
    if (n_points && (!d_xyz || (uintptr_t)d_xyz % 4)) return JIFFY_E_INVALID;
    if (G->n_attrs && (!d_attrs_out || (n_points && !d_attrs_in))) return JIFFY_E_INVALID;
    StdArgs g;
    memset(&g, 0, sizeof g);
    for (uint32_t a = 0; a < G->n_attrs; ++a) {
        const uint32_t ab = G->attr_bytes[a];
        if (ab != 1 && ab != 2 && ab != 4) return JIFFY_E_INVALID;
        if (!d_attrs_out[a] || (uintptr_t)d_attrs_out[a] % ab) return JIFFY_E_INVALID;
        if (n_points && (!d_attrs_in[a] || (uintptr_t)d_attrs_in[a] % ab)) return JIFFY_E_INVALID;
        g.attr_in[a] = n_points ? d_attrs_in[a] : nullptr;
        g.attr_out[a] = d_attrs_out[a];
        g.attr_bytes[a] = ab;
    }
    g.xyz = d_xyz;
    g.range = d_range;
    g.n_scans = n_scans;
    g.n_points = n_points;
    g.height = G->height;
    g.width = G->width;
    g.cells = (uint32_t)cells;
    g.range_bytes = rb;
    g.n_attrs = G->n_attrs;
    g.elev_hi = G->elev_hi;
    g.span = G->elev_hi - G->elev_lo;
    g.unit = G->range_unit;
    g.qmax = (double)((1ull << (8 * rb)) - 1);
    int dev;
    if (current_device(&dev)) return JIFFY_E_DEVICE;
    DevCtx& ctx = g_ctx[dev];
    std::lock_guard<std::mutex> lock(ctx.mu);
    if (grow(ctx.std_keys, 8 * tot_cells) != hipSuccess) return JIFFY_E_DEVICE;
    g.keys = (uint64_t*)ctx.std_keys.p;
    if (launch_standardize(g, stream) != hipSuccess) return JIFFY_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
    prof_collect();
    return JIFFY_OK;
}

int jiffy_ablate(const jiffy_layout* L, uint32_t T, const void* const* d_planes, uint64_t* h_sizes,
                 hipStream_t stream) {
    static_assert(JIFFY_MAX_ATTRS <= 8, "AblArgs holds 8 attributes");
    if (!layout_ok(L) || !h_sizes || (T && !d_planes)) return JIFFY_E_INVALID;
    const uint32_t A = L->n_attrs;
    const uint64_t n = (uint64_t)T * A;
    if (n > (1u << 24)) return JIFFY_E_INVALID;
    for (uint32_t a = 0; T && a < A; ++a)
        if (!d_planes[a] || (uintptr_t)d_planes[a] % L->width_bytes[a]) return JIFFY_E_INVALID;
    if (n == 0) return JIFFY_OK;
    const uint32_t npx = L->height * L->width;
    const uint32_t nb = div_up(npx, kFrame);
    AblArgs g;
    memset(&g, 0, sizeof g);
    g.A = A;
    g.T = T;
    g.npx = npx;
    g.nb = nb;
    g.chunks = div_up(nb, 64u);
    if (n * g.chunks >= (1ull << 31)) return JIFFY_E_INVALID;
    for (uint32_t a = 0; a < A; ++a) {
        g.attr[a].x = d_planes[a];
        g.attr[a].wb = L->width_bytes[a];
        g.attr[a].bits = 8u * L->width_bytes[a];
        g.attr[a].div = make_divisor(L->precision[a]);
    }
    const uint32_t groups = (uint32_t)(n < 256 ? n : 256);
    int dev;
    if (current_device(&dev)) return JIFFY_E_DEVICE;
    DevCtx& ctx = g_ctx[dev];
    std::lock_guard<std::mutex> lock(ctx.mu);
    const size_t acc_bytes = al(64 * n);
    if (grow(ctx.abl, acc_bytes + (size_t)groups * npx * 4) != hipSuccess) return JIFFY_E_DEVICE;
    g.acc = (uint64_t*)ctx.abl.p;
    g.runs = (uint32_t*)((uint8_t*)ctx.abl.p + acc_bytes);
    if (launch_ablate(g, groups, stream) != hipSuccess) return JIFFY_E_DEVICE;
    std::vector<uint64_t> acc(8 * n);
    if (hipMemcpyAsync(acc.data(), g.acc, 64 * n, hipMemcpyDeviceToHost, stream) != hipSuccess) return JIFFY_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
    prof_collect();
    // section = u32 N, three bytes per frame padded to 4, the frames' packed bytes
    auto section = [](uint64_t values, uint64_t packed) { return 4 + ((3 * ((values + 127) / 128) + 3) & ~3ull) + packed; };
    auto pad4 = [](uint64_t x) { return (x + 3) & ~3ull; };
    for (uint64_t r = 0; r < n; ++r) {
        const uint64_t* c = &acc[8 * r];
        uint64_t* o = h_sizes + JIFFY_ABL_SIZES * r;
        for (int k = 0; k < 3; ++k) o[k] = 12 + pad4(section(npx, c[k]));
        o[3] = pad4(section(c[4], c[3]));
        o[4] = r >= A ? pad4(section(c[6], c[5])) : o[3];
    }
    return JIFFY_OK;
}

int jiffy_encode_noalloc(const jiffy_layout* L, const jiffy_options* opt, uint32_t T, const void* const* d_planes,
                         void* d_out, size_t cap, size_t* h_out_len, uint8_t* h_modes, hipStream_t stream) {
    if (int rc = check_encode_args(L, opt, T, d_planes, d_out, h_out_len)) return rc;
    const uint32_t mode = opt ? opt->mode : 0;
    const uint32_t K = (opt && opt->trial_rows) ? opt->trial_rows : 4;
    const uint32_t A = L->n_attrs;
    const uint32_t hl = header_len(A, T);
    std::vector<EncSpec> specs;
    std::vector<OutSpec> outs;
    EncLayout Lo;
    if (T) {  // the workspace this call needs must fit the fixed scratch and staging buffers
        sequence_specs(L, mode, K, T, d_planes, d_out, cap, specs, outs);
        Lo = enc_layout(specs, outs);
        if (Lo.total > kScratchBytes || Lo.up_bytes() > kNoallocUpBytes || Lo.o_items - Lo.o_res > kNoallocResBytes) {
            *h_out_len = 0;
            return JIFFY_E_SCRATCH;
        }
    } else if (hl > kNoallocUpBytes) {
        return JIFFY_E_SCRATCH;
    }
    int dev;
    if (current_device(&dev)) return JIFFY_E_DEVICE;
    DevCtx& ctx = g_ctx[dev];
    std::lock_guard<std::mutex> lock(ctx.mu);
    std::lock_guard<std::mutex> hlock(g_noalloc_mu);
    if (!ctx.scratch) {  // first call on this device (it is current): where its copy of the array lives
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return JIFFY_E_DEVICE;
        ctx.scratch = (uint8_t*)p;
    }
    if (T == 0) {  // a header with no records
        *h_out_len = hl;
        if (cap < hl) return JIFFY_E_CAPACITY;
        write_header(g_noalloc_up, L, 0);
        if (hipMemcpyAsync(d_out, g_noalloc_up, hl, hipMemcpyHostToDevice, stream) != hipSuccess) return JIFFY_E_DEVICE;
        return hipStreamSynchronize(stream) == hipSuccess ? JIFFY_OK : JIFFY_E_DEVICE;
    }
    uint8_t* ws = ctx.scratch;
    // the plan image (records, outputs, tile maps; the error word and the output
    // states zeroed) is written on the host and copied in; everything else the
    // kernels read is written or cleared by this call's kernels first
    enc_fill(Lo, specs, outs, ws, g_noalloc_up);
    const EncPlan plan = enc_plan(Lo, ws, nullptr);  // no host-mapped results: they are copied back below
    t_no_events = true;                              // no timing events either
    hipError_t e = hipMemcpyAsync(ws + Lo.o_err, g_noalloc_up, Lo.up_bytes(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_encode(plan, stream);
    t_no_events = false;
    if (e != hipSuccess) return JIFFY_E_DEVICE;
    // results: per record its mode, the error word, the output's length and fit flag
    if (hipMemcpyAsync(g_noalloc_res, ws + Lo.o_res, Lo.o_items - Lo.o_res, hipMemcpyDeviceToHost, stream) !=
        hipSuccess)
        return JIFFY_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
    uint32_t err;
    memcpy(&err, g_noalloc_res + (Lo.o_err - Lo.o_res), 4);
    if (err & kErrStall) return JIFFY_E_DEVICE;
    EncOut o;
    memcpy(&o, g_noalloc_res + (Lo.o_outs - Lo.o_res), sizeof o);
    *h_out_len = o.len;
    if (!o.ok) return JIFFY_E_CAPACITY;
    if (h_modes) {
        for (uint32_t r = 0; r < Lo.n; ++r) {
            EncRes rs;
            memcpy(&rs, g_noalloc_res + sizeof(EncRes) * r, sizeof rs);
            h_modes[r] = (uint8_t)rs.mode;
        }
    }
    return JIFFY_OK;
}

int jiffy_peek(const void* h_in, size_t len, jiffy_layout* L, uint32_t* n_scans) {
    if (!h_in || !L) return JIFFY_E_INVALID;
    const uint8_t* h = (const uint8_t*)h_in;
    uint32_t T;
    size_t p;
    int rc = parse_header(h, len, L, &T, &p);
    if (rc) return rc;
    if (T) {
        const size_t nrec = (size_t)T * L->n_attrs;
        if (len < p + 4 * nrec) return JIFFY_E_CORRUPT;
        size_t total = p + 4 * nrec;
        for (size_t r = 0; r < nrec; ++r) total += rd32(h + p + 4 * r);
        if (total != len) return JIFFY_E_CORRUPT;
    } else {
        size_t q = p, nrec = 0;
        while (q < len) {
            if (q + 4 > len) return JIFFY_E_CORRUPT;
            const uint32_t rl = rd32(h + q);
            if (rl < 12 || rl % 4 || rl > len - q) return JIFFY_E_CORRUPT;
            q += rl;
            nrec++;
        }
        if (nrec % L->n_attrs) return JIFFY_E_CORRUPT;
        T = (uint32_t)(nrec / L->n_attrs);
    }
    if (n_scans) *n_scans = T;
    return JIFFY_OK;
}

}  // extern "C"

namespace {
// Decodes T scans of layout L from the stream at din (in_len bytes).  Record
// offsets come from the host (roff / rlen) or, with roff null, from the
// length table after `p` header bytes, indexed on the device (hdr: the
// expected header bytes to check there, or null when the host has read it).
// A decode plan: the plan image in `up` (uploaded by k_dec_prepare) and the
// kernels' arguments, valid for the workspace at `ws`.
struct DecPrepared {
    bool valid = false;
    void* ws = nullptr;
    DecPlan plan;
    size_t o_err = 0, up_bytes = 0;
};
// The last device-indexed decode's arguments and plan (per device): a call
// with the same arguments on the same workspace reuses the plan image.  The
// key lists the layout, the scan and stream counts, whether the header is
// checked, and every stream's bytes and output planes.
struct DecCache {
    std::vector<uint64_t> key;
    DecPrepared prep;
    HostBuf up;
};
DecCache g_dec_cache[64];

// A decode plan for S streams of layout L and T scans each (items scan-major,
// then stream, then attribute).  With roff (records walked on the host; S =
// 1) record r is at dins[0] + roff[r]; otherwise the records are indexed on
// the device from each stream's length table.
int dec_prepare(DevCtx& ctx, HostBuf& upbuf, const jiffy_layout& L, uint32_t S, uint32_t T,
                const uint8_t* const* dins, const size_t* in_lens, const uint64_t* roff, const uint32_t* rlen,
                size_t p, const uint8_t* hdr, void* const* const* planes_out, DecPrepared& P) {
    P.valid = false;
    const uint32_t A = L.n_attrs, C = S * A;  // attributes per stream, columns

    const uint32_t n = T * C;
    const uint32_t npx = L.height * L.width, nwords = div_up(npx, 64), maxnb = div_up(npx, kFrame);
    const uint32_t nvt = dec_tile_slots(npx);
    size_t off = 0;
    const size_t o_res = off; off = al(off + sizeof(DecRes) * n);
    const size_t o_roff = off; off = al(off + (roff ? 0 : sizeof(uint64_t) * n));
    const size_t o_rlen = off; off = al(off + (roff ? 0 : sizeof(uint32_t) * n));
    const size_t o_err = off; off = al(off + sizeof(uint32_t) * 2);  // err, err2
    const size_t o_items = off; off = al(off + sizeof(DecItem) * n);
    const size_t o_list = off; off = al(off + sizeof(uint32_t) * n);
    const size_t o_srcs = off; off = al(off + sizeof(DecSrc) * S);
    const size_t up_end = off;
    const uint32_t pwin = div_up(frame_bound(div_up(npx, 8)), kParseWin);
    const size_t per_item = al(8ull * nwords) * 2 + al(4ull * maxnb * 4) + al(8ull * (nvt + 1)) + al(8ull * nvt) +
                            al(sizeof(DecTile) * nvt) + al(4) + al(8ull * (pwin + 1) + 4);
    const size_t o_modes = off; off = al(off + n);
    const size_t o_data = off;
    off += per_item * n;
    if (grow(ctx.ws_dec, off) != hipSuccess) return JIFFY_E_DEVICE;
    const size_t up_bytes = up_end - o_err;
    if (grow(upbuf, up_bytes) != hipSuccess) return JIFFY_E_DEVICE;
    uint8_t* dev = (uint8_t*)ctx.ws_dec.p;
    uint8_t* up = (uint8_t*)upbuf.p;
    memset(up, 0, up_bytes);
    DecItem* hit = (DecItem*)(up + (o_items - o_err));
    bool need_temporal = T > 1;
    for (uint32_t t = 0; t < T; ++t) {
        for (uint32_t c = 0; c < C; ++c) {
            const uint32_t r = t * C + c, st = c / A, a = c - st * A;
            DecItem& it = hit[r];
            uint8_t* base = dev + o_data + per_item * r;
            it.rec = roff ? dins[0] + roff[r] : nullptr;
            it.rec_len = roff ? rlen[r] : 0;
            const size_t step = (size_t)npx * L.width_bytes[a];
            it.out = (uint8_t*)planes_out[st][a] + t * step;
            it.cw = (uint64_t*)base; base += al(8ull * nwords);
            it.vw = (uint64_t*)base; base += al(8ull * nwords);
            it.blkinfo = (uint32_t*)base;
            it.blkoffs = it.blkinfo + maxnb;
            base += al(4ull * maxnb * 4);
            it.tstart = (uint2*)base;
            base += al(8ull * (nvt + 1));
            it.status = (uint64_t*)base;
            base += al(8ull * nvt);
            it.tdesc = (DecTile*)base;
            base += al(sizeof(DecTile) * nvt);
            it.tctr = (uint32_t*)base;
            base += al(4);
            it.npx = npx;
            it.nwords = nwords;
            it.wb = L.width_bytes[a];
            it.bits = 8 * it.wb;
            it.attr = a;
            it.t = t;
            it.P = L.precision[a];
            it.maxnb = maxnb;
            it.aligned16 = ((uintptr_t)it.out % 16 == 0) ? 1u : 0u;
            if (it.P > 1) need_temporal = true;
        }
    }
    // records with 32-bit samples first (their tiles use 32-bit LDS rows), then 16-bit, then 8-bit ones
    uint32_t* hlist = (uint32_t*)(up + (o_list - o_err));
    uint32_t k_list = 0;
    for (uint32_t w : {4u, 2u, 1u})
        for (uint32_t r = 0; r < n; ++r)
            if (hit[r].wb == w) hlist[k_list++] = r;
    uint32_t n_wide = 0, n_w16 = 0;
    for (uint32_t r = 0; r < n; ++r) {
        n_wide += hit[r].wb == 4;
        n_w16 += hit[r].wb == 2;
    }
    DecPlan plan;
    memset(&plan, 0, sizeof plan);
    plan.items = (DecItem*)(dev + o_items);
    plan.res = (DecRes*)(dev + o_res);
    plan.err = (uint32_t*)(dev + o_err);
    plan.err2 = plan.err + 1;
    plan.nvt = nvt;
    plan.rec_list = (const uint32_t*)(dev + o_list);
    plan.n_wide = n_wide;
    plan.n_w16 = n_w16;
    plan.n_items = n;
    plan.n_scans = T;
    plan.n_attrs = C;
    plan.n_src = S;
    plan.src_attrs = A;
    plan.nwords = nwords;
    plan.npx = npx;
    plan.need_temporal = need_temporal ? 1u : 0u;
    plan.modes = dev + o_modes;
    plan.ws = dev + o_data;
    plan.item_stride = per_item;
    plan.pwin = pwin;
    plan.off_pstate = (uint32_t)(al(8ull * nwords) * 2 + al(4ull * maxnb * 4) + al(8ull * (nvt + 1)) + al(8ull * nvt) +
                                 al(sizeof(DecTile) * nvt) + al(4));
    plan.off_cw = 0;
    plan.off_vw = (uint32_t)al(8ull * nwords);
    if (!roff) {
        DecSrc* hs = (DecSrc*)(up + (o_srcs - o_err));
        for (uint32_t st = 0; st < S; ++st) hs[st] = DecSrc{(uint64_t)(uintptr_t)dins[st], (uint64_t)in_lens[st]};
        plan.srcs = (const DecSrc*)((uint8_t*)upbuf.d + (o_srcs - o_err));  // read from host-mapped memory
        plan.roff = (uint64_t*)(dev + o_roff);
        plan.rlen = (uint32_t*)(dev + o_rlen);
        plan.hdr_len = (uint32_t)p;
        plan.hdr_check = hdr ? 1u : 0u;
        if (hdr) memcpy(plan.hdr_words, hdr, p);
    }
    P.plan = plan;
    P.o_err = o_err;
    P.up_bytes = up_bytes;
    P.ws = ctx.ws_dec.p;
    P.valid = true;
    return JIFFY_OK;
}

int dec_execute(DevCtx& ctx, const HostBuf& upbuf, const DecPrepared& P, hipStream_t stream) {
    uint8_t* dev = (uint8_t*)ctx.ws_dec.p;
    if (grow(ctx.down, 64) != hipSuccess) return JIFFY_E_DEVICE;
    if (launch_dec_prepare(upbuf.d, dev + P.o_err, P.up_bytes, P.plan, stream) != hipSuccess) return JIFFY_E_DEVICE;
    if (launch_decode(P.plan, stream) != hipSuccess) return JIFFY_E_DEVICE;
    if (launch_dec_report(dev + P.o_err, ctx.down.d, 2, stream) != hipSuccess) return JIFFY_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
    prof_collect();
    const volatile uint32_t* errs = (const volatile uint32_t*)ctx.down.p;
    return (errs[0] | errs[1]) ? JIFFY_E_CORRUPT : JIFFY_OK;
}

// Decodes T scans of layout L from the stream at din (in_len bytes).  Record
// offsets come from the host (roff / rlen) or, with roff null, from the
// length table after `p` header bytes, indexed on the device (hdr: the
// expected header bytes to check there, or null when the host has read it);
// a device-indexed call with the arguments of the previous one reuses its
// plan.
int run_decode(DevCtx& ctx, const jiffy_layout& L, uint32_t S, uint32_t T, const uint8_t* const* dins,
               const size_t* in_lens, const uint64_t* roff, const uint32_t* rlen, size_t p, const uint8_t* hdr,
               void* const* const* planes_out, hipStream_t stream) {
    const uint32_t A = L.n_attrs;
    if (T == 0 || S == 0) return JIFFY_OK;
    if (!planes_out) return JIFFY_E_INVALID;
    for (uint32_t st = 0; st < S; ++st) {
        if (!planes_out[st]) return JIFFY_E_INVALID;
        for (uint32_t a = 0; a < A; ++a)
            if (!planes_out[st][a] || (uintptr_t)planes_out[st][a] % L.width_bytes[a]) return JIFFY_E_INVALID;
    }
    if (roff) {  // host-walked records: no reuse
        DecPrepared P;
        if (int rc = dec_prepare(ctx, ctx.up, L, S, T, dins, in_lens, roff, rlen, p, hdr, planes_out, P)) return rc;
        return dec_execute(ctx, ctx.up, P, stream);
    }
    DecCache& C = g_dec_cache[&ctx - g_ctx];
    std::vector<uint64_t> key(sizeof(jiffy_layout) / 8 + 1, 0);
    memcpy(key.data(), &L, sizeof L);
    key.push_back(T);
    key.push_back(S);
    key.push_back(hdr ? 1u : 0u);
    for (uint32_t st = 0; st < S; ++st) {
        key.push_back((uint64_t)(uintptr_t)dins[st]);
        key.push_back(in_lens[st]);
        for (uint32_t a = 0; a < A; ++a) key.push_back((uint64_t)(uintptr_t)planes_out[st][a]);
    }
    const bool hit = C.prep.valid && C.prep.ws == ctx.ws_dec.p && key == C.key &&
                     (!hdr || memcmp(C.prep.plan.hdr_words, hdr, p) == 0);
    if (!hit) {
        if (int rc = dec_prepare(ctx, C.up, L, S, T, dins, in_lens, nullptr, nullptr, p, hdr, planes_out, C.prep))
            return rc;
        C.key = std::move(key);
    }
    return dec_execute(ctx, C.up, C.prep, stream);
}
}  // namespace

extern "C" {

int jiffy_decode(const void* d_in, size_t in_len, void* const* d_planes_out, hipStream_t stream) {
    if (!d_in || (uintptr_t)d_in % 4) return JIFFY_E_INVALID;
    if (in_len < 20) return JIFFY_E_CORRUPT;
    int devid;
    if (current_device(&devid)) return JIFFY_E_DEVICE;
    DevCtx& ctx = g_ctx[devid];
    std::lock_guard<std::mutex> lock(ctx.mu);
    const uint8_t* din = (const uint8_t*)d_in;
    // header
    const size_t h0 = in_len < 20 + 8 * JIFFY_MAX_ATTRS ? in_len : 20 + 8 * JIFFY_MAX_ATTRS;
    if (grow(ctx.down, 4096) != hipSuccess) return JIFFY_E_DEVICE;
    uint8_t* hb = (uint8_t*)ctx.down.p;
    if (hipMemcpyAsync(hb, din, h0, hipMemcpyDeviceToHost, stream) != hipSuccess) return JIFFY_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
    jiffy_layout L;
    uint32_t T_hdr;
    size_t p;
    int rc = parse_header(hb, h0, &L, &T_hdr, &p);
    if (rc) return rc;
    const uint32_t A = L.n_attrs;
    if (T_hdr) {  // a length table: the records are indexed on the device
        if ((uint64_t)T_hdr * A > (1u << 24) || in_len < p + 4ull * T_hdr * A) return JIFFY_E_CORRUPT;
        return run_decode(ctx, L, 1, T_hdr, &din, &in_len, nullptr, nullptr, p, nullptr, &d_planes_out, stream);
    }
    // no table: walk the records
    std::vector<uint64_t> roff;
    std::vector<uint32_t> rlen;
    uint64_t q = p;
    uint8_t* tb = (uint8_t*)ctx.down.p;
    while (q < in_len) {
        if (q + 4 > in_len) return JIFFY_E_CORRUPT;
        if (hipMemcpyAsync(tb, din + q, 4, hipMemcpyDeviceToHost, stream) != hipSuccess) return JIFFY_E_DEVICE;
        if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
        const uint32_t rl = rd32(tb);
        if (rl < 12 || rl % 4 || rl > in_len - q) return JIFFY_E_CORRUPT;
        roff.push_back(q);
        rlen.push_back(rl);
        q += rl;
        if (roff.size() > (1u << 24)) return JIFFY_E_CORRUPT;
    }
    if (roff.size() % A) return JIFFY_E_CORRUPT;
    const uint32_t T = (uint32_t)(roff.size() / A);
    return run_decode(ctx, L, 1, T, &din, &in_len, roff.data(), rlen.data(), p, nullptr, &d_planes_out, stream);
}

int jiffy_decode_layout(const jiffy_layout* layout, uint32_t n_scans, const void* d_in, size_t in_len,
                        void* const* d_planes_out, hipStream_t stream) {
    if (!layout_ok(layout) || !d_in || (uintptr_t)d_in % 4 || n_scans == 0) return JIFFY_E_INVALID;
    const uint32_t A = layout->n_attrs;
    if ((uint64_t)n_scans * A > (1u << 24)) return JIFFY_E_INVALID;
    const size_t p = 20 + 8 * A;
    if (in_len < p + 4ull * n_scans * A) return JIFFY_E_CORRUPT;
    int devid;
    if (current_device(&devid)) return JIFFY_E_DEVICE;
    DevCtx& ctx = g_ctx[devid];
    std::lock_guard<std::mutex> lock(ctx.mu);
    uint8_t hdr[20 + 8 * JIFFY_MAX_ATTRS];
    write_header(hdr, layout, n_scans);
    const uint8_t* din = (const uint8_t*)d_in;
    return run_decode(ctx, *layout, 1, n_scans, &din, &in_len, nullptr, nullptr, p, hdr, &d_planes_out, stream);
}

int jiffy_decode_many(const jiffy_layout* layout, uint32_t n_streams, uint32_t n_scans, const void* const* d_ins,
                      const size_t* in_lens, void* const* const* d_planes_out, hipStream_t stream) {
    if (!layout_ok(layout) || n_scans == 0 || !d_ins || !in_lens) return JIFFY_E_INVALID;
    if (n_streams == 0) return JIFFY_OK;
    const uint32_t A = layout->n_attrs;
    if ((uint64_t)n_scans * A * n_streams > (1u << 24)) return JIFFY_E_INVALID;
    const size_t p = 20 + 8 * A;
    for (uint32_t s = 0; s < n_streams; ++s) {
        if (!d_ins[s] || (uintptr_t)d_ins[s] % 4) return JIFFY_E_INVALID;
        if (in_lens[s] < p + 4ull * n_scans * A) return JIFFY_E_CORRUPT;
    }
    int devid;
    if (current_device(&devid)) return JIFFY_E_DEVICE;
    DevCtx& ctx = g_ctx[devid];
    std::lock_guard<std::mutex> lock(ctx.mu);
    uint8_t hdr[20 + 8 * JIFFY_MAX_ATTRS];
    write_header(hdr, layout, n_scans);
    return run_decode(ctx, *layout, n_streams, n_scans, (const uint8_t* const*)d_ins, in_lens, nullptr, nullptr, p,
                      hdr, d_planes_out, stream);
}

// ---------------------------------------------------------------------------
// stateful streams
// ---------------------------------------------------------------------------
struct jiffy_stream {
    jiffy_layout layout;
    jiffy_options opt;
    int device;
    void* q[2][JIFFY_MAX_ATTRS];
    uint64_t* v[2][JIFFY_MAX_ATTRS];
    int cur;
    int has_prev;
    bool owns;  // the state buffers were allocated by the library (else they live in the caller's memory)
    bool busy;  // in a submitted step that has not finished
};

}  // extern "C"

namespace {
// The resident state of a stream, in order: for each half k and attribute a
// the quantized samples (npx * width + 16 bytes), then the valid-sample words
// (8 bytes per 64 samples), each part 256-byte aligned.
size_t state_layout(const jiffy_layout* L, jiffy_stream* s, uint8_t* base) {
    const size_t npx = (size_t)L->height * L->width, nwords = (npx + 63) / 64;
    size_t off = 0;
    for (int k = 0; k < 2; ++k) {
        for (uint32_t a = 0; a < L->n_attrs; ++a) {
            if (s) s->q[k][a] = base + off;
            off = al(off + npx * L->width_bytes[a] + 16);
            if (s) s->v[k][a] = (uint64_t*)(base + off);
            off = al(off + 8 * nwords);
        }
    }
    return off;
}

jiffy_stream* new_stream(const jiffy_layout* L, const jiffy_options* opt) {
    jiffy_stream* s = new (std::nothrow) jiffy_stream();
    if (!s) return nullptr;
    s->layout = *L;
    s->opt.mode = opt ? opt->mode : 0;
    s->opt.trial_rows = (opt && opt->trial_rows) ? opt->trial_rows : 4;
    s->cur = 0;
    s->has_prev = 0;
    s->busy = false;
    return s;
}
}  // namespace

extern "C" {

size_t jiffy_stream_state_bytes(const jiffy_layout* L) {
    if (!layout_ok(L)) return 0;
    return state_layout(L, nullptr, nullptr);
}

int jiffy_stream_create(const jiffy_layout* L, const jiffy_options* opt, jiffy_stream** out) {
    if (!layout_ok(L) || !out) return JIFFY_E_INVALID;
    if (opt && opt->mode > 2) return JIFFY_E_INVALID;
    jiffy_stream* s = new_stream(L, opt);
    if (!s) return JIFFY_E_INVALID;
    s->owns = true;
    if (current_device(&s->device)) { delete s; return JIFFY_E_DEVICE; }
    const size_t npx = (size_t)L->height * L->width, nwords = (npx + 63) / 64;
    for (int k = 0; k < 2; ++k) {
        for (uint32_t a = 0; a < L->n_attrs; ++a) {
            if (hipMalloc(&s->q[k][a], npx * L->width_bytes[a] + 16) != hipSuccess ||
                hipMalloc((void**)&s->v[k][a], 8 * nwords) != hipSuccess) {
                jiffy_stream_destroy(s);
                return JIFFY_E_DEVICE;
            }
        }
    }
    *out = s;
    return JIFFY_OK;
}

int jiffy_stream_create_at(const jiffy_layout* L, const jiffy_options* opt, void* d_state, size_t state_bytes,
                           jiffy_stream** out) {
    if (!layout_ok(L) || !out || !d_state || (uintptr_t)d_state % kAlign) return JIFFY_E_INVALID;
    if (opt && opt->mode > 2) return JIFFY_E_INVALID;
    if (state_bytes < state_layout(L, nullptr, nullptr)) return JIFFY_E_INVALID;
    jiffy_stream* s = new_stream(L, opt);
    if (!s) return JIFFY_E_INVALID;
    s->owns = false;
    if (current_device(&s->device)) { delete s; return JIFFY_E_DEVICE; }
    state_layout(L, s, (uint8_t*)d_state);
    *out = s;
    return JIFFY_OK;
}

int jiffy_stream_reset(jiffy_stream* s) {
    if (!s || s->busy) return JIFFY_E_INVALID;
    s->has_prev = 0;
    return JIFFY_OK;
}

void jiffy_stream_destroy(jiffy_stream* s) {
    if (!s) return;
    if (s->owns)
        for (int k = 0; k < 2; ++k)
            for (uint32_t a = 0; a < JIFFY_MAX_ATTRS; ++a) {
                if (s->q[k][a]) (void)hipFree(s->q[k][a]);
                if (s->v[k][a]) (void)hipFree(s->v[k][a]);
            }
    delete s;
}

}  // extern "C"

namespace {
// Checks a batch's arguments; JIFFY_OK or an error status.
int check_batch(jiffy_stream* const* streams, uint32_t n, const void* const* const* d_planes, void* const* d_out,
                const size_t* caps, int dev) {
    if (!streams || !d_planes || !d_out || !caps) return JIFFY_E_INVALID;
    for (uint32_t i = 0; i < n; ++i) {
        const jiffy_stream* s = streams[i];
        if (!s || !d_planes[i] || !d_out[i] || (uintptr_t)d_out[i] % 4) return JIFFY_E_INVALID;
        if (s->device != dev) return JIFFY_E_SHAPE;
        if (s->busy) return JIFFY_E_INVALID;  // in a submitted step that has not finished
        for (uint32_t a = 0; a < s->layout.n_attrs; ++a)
            if (!d_planes[i][a] || (uintptr_t)d_planes[i][a] % s->layout.width_bytes[a]) return JIFFY_E_INVALID;
        for (uint32_t k = 0; k < i; ++k)
            if (streams[k] == s) return JIFFY_E_INVALID;
    }
    return JIFFY_OK;
}

// One record per attribute of each stream's next scan, predicting from the
// resident previous scan; the new scan's quantized samples and valid words
// go to the other half of the stream's state.
// With `packed` every record goes to the one output d_out[0] (caps[0] bytes),
// stream after stream, each right after the one before.
void stream_specs(jiffy_stream* const* streams, uint32_t n, const void* const* const* d_planes, void* const* d_out,
                  const size_t* caps, std::vector<EncSpec>& specs, std::vector<OutSpec>& outs, bool packed = false) {
    specs.clear();
    outs.resize(packed ? 1 : n);
    uint32_t total = 0;
    for (uint32_t i = 0; i < n; ++i) total += streams[i]->layout.n_attrs;
    if (packed) outs[0] = OutSpec{(uint8_t*)d_out[0], caps[0], 0, total, 0, 1, &streams[0]->layout};
    for (uint32_t i = 0; i < n; ++i) {
        const jiffy_stream* s = streams[i];
        const jiffy_layout& L = s->layout;
        if (!packed) outs[i] = OutSpec{(uint8_t*)d_out[i], caps[i], (uint32_t)specs.size(), L.n_attrs, 0, 1, &s->layout};
        for (uint32_t a = 0; a < L.n_attrs; ++a) {
            EncSpec e;
            e.x = d_planes[i][a];
            e.xprev = s->has_prev ? s->q[s->cur][a] : nullptr;
            e.qout = s->q[s->cur ^ 1][a];
            e.vw_fixed = s->v[s->cur ^ 1][a];
            e.vwprev_fixed = s->has_prev ? s->v[s->cur][a] : nullptr;
            e.prev_item = -1;
            e.H = L.height;
            e.W = L.width;
            e.wb = L.width_bytes[a];
            e.P = L.precision[a];
            e.attr = a;
            e.out_id = packed ? 0u : i;
            e.has_prev = s->has_prev ? 1u : 0u;
            e.prev_quantized = 1;
            e.mode_req = s->opt.mode;
            e.trial_rows = s->opt.trial_rows;
            specs.push_back(e);
        }
    }
}

// lengths, modes and status of a finished step; the streams advance only
// when every output fitted
int finish_step(jiffy_stream* const* streams, uint32_t n, const EncResult& res, size_t* h_lens, uint8_t* h_modes) {
    int status = JIFFY_OK;
    for (uint32_t i = 0; i < n; ++i) {
        h_lens[i] = res.lens[i];
        if (!res.ok[i]) status = JIFFY_E_CAPACITY;
    }
    if (h_modes) memcpy(h_modes, res.modes.data(), res.modes.size());
    if (status == JIFFY_OK) {
        for (uint32_t i = 0; i < n; ++i) {
            streams[i]->cur ^= 1;
            streams[i]->has_prev = 1;
        }
    }
    return status;
}
}  // namespace

extern "C" {

int jiffy_batch_encode_step(jiffy_stream* const* streams, uint32_t n, const void* const* const* d_planes,
                            void* const* d_out, const size_t* caps, size_t* h_lens, uint8_t* h_modes,
                            hipStream_t stream) {
    if (n == 0) return JIFFY_OK;
    if (!h_lens) return JIFFY_E_INVALID;
    int dev;
    if (current_device(&dev)) return JIFFY_E_DEVICE;
    if (int rc = check_batch(streams, n, d_planes, d_out, caps, dev)) return rc;
    DevCtx& ctx = g_ctx[dev];
    std::lock_guard<std::mutex> lock(ctx.mu);
    std::vector<EncSpec> specs;
    std::vector<OutSpec> outs;
    stream_specs(streams, n, d_planes, d_out, caps, specs, outs);
    EncResult res;
    if (int rc = run_encode(ctx, specs, outs, stream, res)) return rc;
    return finish_step(streams, n, res, h_lens, h_modes);
}

// ---------------------------------------------------------------------------
// batches: a fixed set of streams whose step is one replay of a HIP graph
// ---------------------------------------------------------------------------
struct jiffy_batch {
    int device = 0;
    std::vector<jiffy_stream*> streams;
    std::vector<std::vector<const void*>> planes;
    std::vector<const void* const*> plane_ptrs;
    std::vector<void*> outs;
    std::vector<size_t> caps;
    EncLayout Lo;
    uint8_t* dev = nullptr;
    uint8_t* up = nullptr;   // host image of the plan, read by the graph's upload kernel
    void* up_d = nullptr;
    uint8_t* res = nullptr;  // host results, written by the graph's offsets kernel
    void* res_d = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t fgrid = 0;  // the fused launch's workgroups (the tuning at creation), or 0: the kernel chain
};

int jiffy_batch_create(jiffy_stream* const* streams, uint32_t n, const void* const* const* d_planes,
                       void* const* d_out, const size_t* caps, jiffy_batch** out) {
    if (!out || n == 0) return JIFFY_E_INVALID;
    int dev;
    if (current_device(&dev)) return JIFFY_E_DEVICE;
    if (int rc = check_batch(streams, n, d_planes, d_out, caps, dev)) return rc;
    DevCtx& ctx = g_ctx[dev];
    std::lock_guard<std::mutex> lock(ctx.mu);  // the streams' state is read while the batch is planned
    jiffy_batch* b = new (std::nothrow) jiffy_batch();
    if (!b) return JIFFY_E_INVALID;
    b->device = dev;
    b->streams.assign(streams, streams + n);
    b->planes.resize(n);
    for (uint32_t i = 0; i < n; ++i) b->planes[i].assign(d_planes[i], d_planes[i] + streams[i]->layout.n_attrs);
    for (uint32_t i = 0; i < n; ++i) b->plane_ptrs.push_back(b->planes[i].data());
    b->outs.assign(d_out, d_out + n);
    b->caps.assign(caps, caps + n);
    b->fgrid = fused_grid(current_tuning());
    std::vector<EncSpec> specs;
    std::vector<OutSpec> outs;
    stream_specs(b->streams.data(), n, b->plane_ptrs.data(), b->outs.data(), b->caps.data(), specs, outs);
    b->Lo = enc_layout(specs, outs);
    int rc = JIFFY_E_DEVICE;
    if (hipMalloc((void**)&b->dev, b->Lo.total) == hipSuccess &&
        host_alloc((void**)&b->up, &b->up_d, b->Lo.up_bytes()) == hipSuccess &&
        host_alloc((void**)&b->res, &b->res_d, b->Lo.res_bytes()) == hipSuccess &&
        hipStreamCreate(&b->cap_stream) == hipSuccess) {
        enc_fill(b->Lo, specs, outs, b->dev, b->up);
        const EncPlan plan = enc_plan(b->Lo, b->dev, (uint8_t*)b->res_d);
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            t_no_events = true;
            const hipError_t e = enc_enqueue(b->Lo, plan, b->dev, b->up_d, b->cap_stream, true, b->fgrid);
            t_no_events = false;
            const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &b->graph);
            if (e == hipSuccess && e2 == hipSuccess &&
                hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess)
                rc = JIFFY_OK;
        }
    }
    if (rc != JIFFY_OK) {
        jiffy_batch_destroy(b);
        return rc;
    }
    *out = b;
    return JIFFY_OK;
}

int jiffy_batch_run(jiffy_batch* b, const void* const* const* d_planes, size_t* h_lens, uint8_t* h_modes,
                    hipStream_t stream) {
    if (!b || !h_lens) return JIFFY_E_INVALID;
    int dev;
    if (current_device(&dev)) return JIFFY_E_DEVICE;
    if (dev != b->device) return JIFFY_E_SHAPE;
    DevCtx& ctx = g_ctx[dev];
    std::lock_guard<std::mutex> lock(ctx.mu);  // the streams' resident state changes with the step
    const uint32_t n = (uint32_t)b->streams.size();
    if (d_planes) {
        if (int rc = check_batch(b->streams.data(), n, d_planes, b->outs.data(), b->caps.data(), dev)) return rc;
        for (uint32_t i = 0; i < n; ++i)
            b->planes[i].assign(d_planes[i], d_planes[i] + b->streams[i]->layout.n_attrs);
    }
    std::vector<EncSpec> specs;
    std::vector<OutSpec> outs;
    stream_specs(b->streams.data(), n, b->plane_ptrs.data(), b->outs.data(), b->caps.data(), specs, outs);
    enc_fill(b->Lo, specs, outs, b->dev, b->up);
    if (hipGraphLaunch(b->exec, stream) != hipSuccess) return JIFFY_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return JIFFY_E_DEVICE;
    EncResult res;
    enc_results(b->Lo, b->res, res);
    if (res.err & kErrStall) return JIFFY_E_DEVICE;
    return finish_step(b->streams.data(), n, res, h_lens, h_modes);
}

void jiffy_batch_destroy(jiffy_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->dev) (void)hipFree(b->dev);
    if (b->up) (void)hipHostFree(b->up);
    if (b->res) (void)hipHostFree(b->res);
    delete b;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// asynchronous steps: a step context owns a workspace sized once; submit
// enqueues a batch and returns, finish waits for it and reads the results
// ---------------------------------------------------------------------------
namespace {
// Upper bounds of what enc_layout needs for any batch of at most R records
// of at most S samples in all, with one (packed) output and resident valid
// words: every per-record part is at most its linear size plus one alignment
// unit, and ceil(npx / k) summed over records is at most S / k + R.
struct StepBound {
    size_t dev, up, res;
};
// Limits of a step context: with them every size below fits in 64 bits.
constexpr uint64_t kStepMaxRecords = 1ull << 24, kStepMaxSamples = 1ull << 40;

StepBound step_bound(uint64_t R, uint64_t S) {
    const uint64_t nb = S / kFrame + R, nft = S / kFTile + R, nm = S / 8 + R;
    StepBound b;
    const size_t fixed_up = 4 + sizeof(EncOut) + sizeof(EncItem) * R + 4 * R + 4 * nft + 5 * kAlign;
    b.up = fixed_up;
    b.dev = sizeof(EncRes) * R + kAlign + fixed_up                             // results, then the uploaded part
            + 16 * nb + 4 * nft + 8 * nft + 4 * R + 2 * kAlign * R              // frame info, offsets, tile states
            + (size_t)kSlotBytes * nb + kAlign * R                              // frame slots
            + (16 + 4 + 4) * R + nm + 4 * (nm / kZstdBlockMax + R) + kAlign * R  // mask frames
            + 8 * (nm / 4 + 4 * R + R) + kAlign * R;                            // segment tables
    b.res = 16 + 8 * R + 4;
    return b;
}
}  // namespace

struct jiffy_step {
    int device = 0;
    uint32_t max_records = 0;
    uint64_t max_samples = 0;
    DevBuf ws;
    HostBuf up, res;
    bool pending = false;
    hipStream_t stream = nullptr;
    std::vector<jiffy_stream*> streams;
    EncLayout Lo;
};

extern "C" {

size_t jiffy_step_workspace_bytes(uint32_t max_records, uint64_t max_samples) {
    if (max_records == 0 || max_samples == 0 || max_records > kStepMaxRecords || max_samples > kStepMaxSamples)
        return 0;
    return step_bound(max_records, max_samples).dev;
}

int jiffy_step_create(uint32_t max_records, uint64_t max_samples, jiffy_step** out) {
    if (!out || max_records == 0 || max_samples == 0 || max_records > kStepMaxRecords ||
        max_samples > kStepMaxSamples)
        return JIFFY_E_INVALID;
    jiffy_step* st = new (std::nothrow) jiffy_step();
    if (!st) return JIFFY_E_INVALID;
    if (current_device(&st->device)) { delete st; return JIFFY_E_DEVICE; }
    st->max_records = max_records;
    st->max_samples = max_samples;
    const StepBound b = step_bound(max_records, max_samples);
    if (hipMalloc(&st->ws.p, b.dev) != hipSuccess) { delete st; return JIFFY_E_DEVICE; }
    st->ws.cap = b.dev;
    if (host_alloc(&st->up.p, &st->up.d, b.up) != hipSuccess || host_alloc(&st->res.p, &st->res.d, b.res) != hipSuccess) {
        jiffy_step_destroy(st);
        return JIFFY_E_DEVICE;
    }
    st->up.cap = b.up;
    st->res.cap = b.res;
    *out = st;
    return JIFFY_OK;
}

int jiffy_step_submit(jiffy_step* st, jiffy_stream* const* streams, uint32_t n, const void* const* const* d_planes,
                      void* d_out, size_t out_capacity, hipStream_t stream) {
    if (!st || st->pending || n == 0 || !d_out) return JIFFY_E_INVALID;
    int dev;
    if (current_device(&dev)) return JIFFY_E_DEVICE;
    if (dev != st->device) return JIFFY_E_SHAPE;
    void* const outs1[1] = {d_out};
    const size_t caps1[1] = {out_capacity};
    if (!streams || !d_planes || (uintptr_t)d_out % 4) return JIFFY_E_INVALID;
    uint64_t recs = 0, samples = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const jiffy_stream* s = streams[i];
        if (!s || !d_planes[i]) return JIFFY_E_INVALID;
        if (s->device != dev) return JIFFY_E_SHAPE;
        if (s->busy) return JIFFY_E_INVALID;
        for (uint32_t a = 0; a < s->layout.n_attrs; ++a)
            if (!d_planes[i][a] || (uintptr_t)d_planes[i][a] % s->layout.width_bytes[a]) return JIFFY_E_INVALID;
        for (uint32_t k = 0; k < i; ++k)
            if (streams[k] == s) return JIFFY_E_INVALID;
        recs += s->layout.n_attrs;
        samples += (uint64_t)s->layout.n_attrs * s->layout.height * s->layout.width;
    }
    if (recs > st->max_records || samples > st->max_samples) return JIFFY_E_CAPACITY;
    std::vector<EncSpec> specs;
    std::vector<OutSpec> outs;
    stream_specs(streams, n, d_planes, outs1, caps1, specs, outs, true);
    EncLayout Lo = enc_layout(specs, outs);
    if (Lo.total > st->ws.cap || Lo.up_bytes() > st->up.cap || Lo.res_bytes() > st->res.cap) return JIFFY_E_CAPACITY;
    enc_fill(Lo, specs, outs, (uint8_t*)st->ws.p, (uint8_t*)st->up.p);
    const EncPlan plan = enc_plan(Lo, (uint8_t*)st->ws.p, (uint8_t*)st->res.d);
    t_no_events = true;  // the step completes after this call returns: no timing events
    const hipError_t e = enc_enqueue(Lo, plan, (uint8_t*)st->ws.p, st->up.d, stream, true, fused_grid(current_tuning()));
    t_no_events = false;
    if (e != hipSuccess) return JIFFY_E_DEVICE;
    st->streams.assign(streams, streams + n);
    for (jiffy_stream* s : st->streams) s->busy = true;
    st->Lo = std::move(Lo);
    st->stream = stream;
    st->pending = true;
    return JIFFY_OK;
}

int jiffy_step_finish(jiffy_step* st, size_t* h_lens, uint8_t* h_modes) {
    if (!st || !st->pending || !h_lens) return JIFFY_E_INVALID;
    const hipError_t e = hipStreamSynchronize(st->stream);
    st->pending = false;
    for (jiffy_stream* s : st->streams) s->busy = false;
    if (e != hipSuccess) return JIFFY_E_DEVICE;
    EncResult res;
    enc_results(st->Lo, (const uint8_t*)st->res.p, res);
    if (res.err & kErrStall) return JIFFY_E_DEVICE;
    const uint32_t n = (uint32_t)st->streams.size();
    for (uint32_t i = 0, r = 0; i < n; ++i) {
        size_t len = 0;
        for (uint32_t a = 0; a < st->streams[i]->layout.n_attrs; ++a, ++r) {
            len += res.rec_lens[r];
            if (h_modes) h_modes[r] = res.modes[r];
        }
        h_lens[i] = len;
    }
    if (!res.ok[0]) return JIFFY_E_CAPACITY;
    for (jiffy_stream* s : st->streams) {
        s->cur ^= 1;
        s->has_prev = 1;
    }
    return JIFFY_OK;
}

void jiffy_step_destroy(jiffy_step* st) {
    if (!st) return;
    if (st->pending) {  // an unfinished step: wait for it; its streams do not advance
        (void)hipStreamSynchronize(st->stream);
        for (jiffy_stream* s : st->streams) s->busy = false;
    }
    if (st->ws.p) (void)hipFree(st->ws.p);
    if (st->up.p) (void)hipHostFree(st->up.p);
    if (st->res.p) (void)hipHostFree(st->res.p);
    delete st;
}

}  // extern "C"
