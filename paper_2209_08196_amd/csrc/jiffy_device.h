// Device helpers for the Jiffy kernels (gfx950, wave64).
#pragma once

#include "jiffy_internal.h"

namespace jiffy {

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// number of set bits of m below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Cross-lane moves through DPP (no LDS): row_shr:n moves within rows of 16
// lanes, row_bcast:15 / :31 carry a row's last lane into the next rows.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, false);
}
template <class Op>
__device__ __forceinline__ uint32_t wave_incl_op(uint32_t v, Op op) {
    const uint32_t l = lane_id(), rl = l & 15u;
    uint32_t t;
    t = dpp_mov<0x111>(v); if (rl >= 1) v = op(v, t);
    t = dpp_mov<0x112>(v); if (rl >= 2) v = op(v, t);
    t = dpp_mov<0x114>(v); if (rl >= 4) v = op(v, t);
    t = dpp_mov<0x118>(v); if (rl >= 8) v = op(v, t);
    t = dpp_mov<0x142>(v); if ((l & 31u) >= 16) v = op(v, t);
    t = dpp_mov<0x143>(v); if (l >= 32) v = op(v, t);
    return v;
}
// inclusive prefix sum over the wave (wrapping u32)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    return wave_incl_op(v, [](uint32_t a, uint32_t b) { return a + b; });
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
    v = wave_incl_op(v, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = wave_incl_op(v, [](uint32_t a, uint32_t b) { return a < b ? a : b; });
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint64_t t = __shfl_up(v, o, kWave);
        if (l >= (uint32_t)o) v += t;
    }
    return v;
}

// Accesses to host memory at system scope: they bypass the device's caches,
// so a load sees what the host wrote before the launch and a store reaches
// host memory by the time the kernel completes, whatever caching mode the
// host allocation has.
__device__ __forceinline__ uint4 load_system16(const JG uint4* p) {
    const uint64_t* q = (const uint64_t*)p;
    const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
}
__device__ __forceinline__ void store_system(JG uint32_t* p, uint32_t v) {
    __hip_atomic_store((uint32_t*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Exclusive prefix sum over a workgroup of NT threads.  `scratch` holds
// NT/64 + 1 words of LDS.  Returns the exclusive prefix; *total gets the sum.
// Every thread of the workgroup must call it.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* scratch, uint32_t* total) {
    constexpr int NW = NT / kWave;
    const uint32_t l = lane_id(), w = threadIdx.x / kWave;
    uint32_t inc = wave_incl_scan(v);
    if (l == kWave - 1) scratch[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t s = l < (uint32_t)NW ? scratch[l] : 0u;
        uint32_t si = wave_incl_scan(s);
        if (l < (uint32_t)NW) scratch[l] = si - s;
        if (l == NW - 1) scratch[NW] = si;
    }
    __syncthreads();
    uint32_t r = scratch[w] + inc - v;
    *total = scratch[NW];
    __syncthreads();
    return r;
}

// Exclusive prefix sums of three values over the workgroup at once
// (3 * (NT/64 + 1) words of LDS); tot gets the three sums.
template <int NT>
__device__ __forceinline__ void block_excl_scan3(uint32_t v[3], uint32_t* scratch, uint32_t tot[3]) {
    constexpr int NW = NT / kWave;
    static_assert(NW >= 3 && NW <= kWave, "one wave per value combines the wave sums");
    const uint32_t l = lane_id(), w = threadIdx.x / kWave;
    uint32_t inc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        inc[c] = wave_incl_scan(v[c]);
        if (l == kWave - 1) scratch[c * (NW + 1) + w] = inc[c];
    }
    __syncthreads();
    if (w < 3) {  // wave c combines the wave sums of value c
        uint32_t* sc = scratch + w * (NW + 1);
        const uint32_t x = l < (uint32_t)NW ? sc[l] : 0u;
        const uint32_t xi = wave_incl_scan(x);
        if (l < (uint32_t)NW) sc[l] = xi - x;
        if (l == NW - 1) sc[NW] = xi;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v[c] = scratch[c * (NW + 1) + w] + inc[c] - v[c];
        tot[c] = scratch[c * (NW + 1) + NW];
    }
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t v, uint64_t* scratch, uint64_t* total) {
    constexpr int NW = NT / kWave;
    const uint32_t l = lane_id(), w = threadIdx.x / kWave;
    uint64_t inc = wave_incl_scan64(v);
    if (l == kWave - 1) scratch[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint64_t s = l < (uint32_t)NW ? scratch[l] : 0ull;
        uint64_t si = wave_incl_scan64(s);
        if (l < (uint32_t)NW) scratch[l] = si - s;
        if (l == NW - 1) scratch[NW] = si;
    }
    __syncthreads();
    uint64_t r = scratch[w] + inc - v;
    *total = scratch[NW];
    __syncthreads();
    return r;
}

// Exclusive running maximum over a workgroup (same contract as block_excl_scan).
template <int NT>
__device__ __forceinline__ uint32_t block_excl_max(uint32_t v, uint32_t* scratch, uint32_t* total) {
    constexpr int NW = NT / kWave;
    const uint32_t l = lane_id(), w = threadIdx.x / kWave;
    auto mx = [](uint32_t a, uint32_t b) { return a > b ? a : b; };
    uint32_t inc = wave_incl_op(v, mx);
    uint32_t exc = (uint32_t)__shfl_up((int)inc, 1, kWave);
    if (l == 0) exc = 0;
    if (l == kWave - 1) scratch[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t s = l < (uint32_t)NW ? scratch[l] : 0u;
        uint32_t si = wave_incl_op(s, mx);
        uint32_t se = (uint32_t)__shfl_up((int)si, 1, kWave);
        if (l == 0) se = 0;
        if (l < (uint32_t)NW) scratch[l] = se;
        if (l == NW - 1) scratch[NW] = si;
    }
    __syncthreads();
    uint32_t r = max(scratch[w], exc);
    *total = scratch[NW];
    __syncthreads();
    return r;
}

// position of the r-th (0-based) set bit of v; v must have more than r bits set
__device__ __forceinline__ uint32_t select_bit(uint64_t v, uint32_t r) {
    uint32_t pos = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        uint64_t lowmask = (width == 64) ? ~0ull : ((1ull << width) - 1);
        uint32_t c = __popcll(v & lowmask);
        if (r >= c) {
            r -= c;
            v >>= width;
            pos += width;
        }
    }
    return pos;
}

__device__ __forceinline__ uint32_t low_mask32(uint32_t bits) { return bits >= 32 ? 0xFFFFFFFFu : ((1u << bits) - 1u); }

// Sec. III-B: nearest multiple of P, halves up; zero stays zero, valid stays >= 1.
__device__ __forceinline__ uint32_t quantize(uint32_t x, const Divisor& d) {
    if (d.P == 1) return x;
    uint32_t t = __umulhi(d.magic, x);
    uint32_t a = (t + ((x - t) >> d.s1)) >> d.s2;  // x / P
    uint32_t r = x - a * d.P;
    uint32_t q = a + (r >= d.half_up ? 1u : 0u);
    return x == 0 ? 0u : max(q, 1u);
}
__device__ __forceinline__ uint32_t dequantize(uint32_t q, uint32_t P, uint32_t bits) {
    uint64_t v = (uint64_t)q * P;
    uint64_t top = (bits >= 32) ? 0xFFFFFFFFull : ((1ull << bits) - 1);
    return (uint32_t)(v > top ? top : v);
}

// Eq. 1 (standard ZigZag) on w-bit two's-complement values.
__device__ __forceinline__ uint32_t zigzag(uint32_t d, uint32_t bits) {
    int32_t s = (int32_t)(d << (32 - bits)) >> (32 - bits);
    return ((uint32_t)s << 1) ^ (uint32_t)(s >> 31);
}
__device__ __forceinline__ uint32_t unzigzag(uint32_t z, uint32_t bits) {
    return ((z >> 1) ^ (0u - (z & 1u))) & low_mask32(bits);
}

// Frame-width choice for 128 values held two per lane (Sec. II):
// B = width of the maximum; n(b) = values >= 2^b;
// cost(b) = 16 b + [n > 0] (n + ceil(n (B - b) / 8)); ties go to the larger b.
// The values' bit widths are counted by ballots, one distinct width at a
// time (lane v ends up holding the count of width v); a prefix sum gives
// n(b) on lane b, which evaluates cost(b); a wave minimum picks the width.
// Called by a whole wave.
struct FrameChoice {
    uint32_t b, n, B, cost;
};
__device__ __forceinline__ FrameChoice choose_frame(uint32_t z0, uint32_t z1) {
    const uint32_t l = lane_id();
    const uint32_t w0 = z0 ? 32u - __clz(z0) : 0u;
    const uint32_t w1 = z1 ? 32u - __clz(z1) : 0u;
    uint64_t rem0 = ~0ull, rem1 = ~0ull;
    uint32_t hc = 0, B = 0;
    while (rem0 | rem1) {
        const uint32_t v = rem0 ? (uint32_t)__builtin_amdgcn_readlane((int)w0, (int)__builtin_ctzll(rem0))
                                : (uint32_t)__builtin_amdgcn_readlane((int)w1, (int)__builtin_ctzll(rem1));
        const uint64_t m0 = ballot(w0 == v) & rem0, m1 = ballot(w1 == v) & rem1;
        if (l == v) hc = (uint32_t)(__popcll(m0) + __popcll(m1));
        B = v > B ? v : B;
        rem0 &= ~m0;
        rem1 &= ~m1;
    }
    const uint32_t n = 128u - wave_incl_scan(hc);  // values wider than l bits
    uint32_t key = 0xFFFFFFFFu;
    if (l <= B) {
        const uint32_t cost = 16u * l + (n ? n + (n * (B - l) + 7u) / 8u : 0u);
        key = (cost << 6) | (63u - l);
    }
    key = wave_min(key);
    const uint32_t b = 63u - (key & 63u);
    const uint32_t nb = (uint32_t)__builtin_amdgcn_readlane((int)n, (int)b);
    return FrameChoice{b, nb, B, key >> 6};
}

// ---- frame rows (a frame of 128 values in LDS, four lanes per frame) -----
constexpr uint32_t kRow = kFrame + 16;  // LDS words per frame row
static_assert(kRow % 4 == 0 && 4 * kRow <= kSlotBytes, "a frame row holds 128 values, padded every 32, and fits a slot");

// word of value i in a frame row: four pad words after every 32 values, so
// that each lane's 32 values start 16-byte aligned in distinct banks
__device__ __forceinline__ uint32_t row_off(uint32_t i) { return i + ((i >> 5) << 2); }

// DPP quad permutations
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E;
template <int Q> __device__ __forceinline__ uint32_t quad_bcast(uint32_t v) { return dpp_mov<0x55 * Q>(v); }

constexpr uint32_t kTileFrames = kFTile / kFrame + 1;  // frames a tile's values can touch
constexpr uint32_t kTileQuads = kFTile / kFrame;       // frames a tile can hold whole

// value kb.. of a tile: frame (k >> 7) - jf of the tile's rows, element
// row_off(k & 127).  A row is 128 values and four pads per 32, so this is
// k + 4 (k >> 5) - kRow jf: two operations and a uniform term per value.
static_assert(kRow == kFrame + 16, "a row is 128 values and four pads per 32");
__device__ __forceinline__ uint32_t tile_word(uint32_t k, uint32_t jf) { return k + ((k >> 5) << 2) - kRow * jf; }

// Frame rows of 32-bit values (32-bit samples) or 16-bit values (8- and
// 16-bit samples, whose residuals and running sums fit 16 bits): each lane's
// 32 values start 16-byte aligned.
template <class R> struct RowT;
template <> struct RowT<uint32_t> { static constexpr uint32_t kElems = kRow, kLane = 36, kPad = 4; };
template <> struct RowT<uint16_t> { static constexpr uint32_t kElems = 160, kLane = 40, kPad = 8; };
template <class R> __device__ __forceinline__ uint32_t roff(uint32_t i) { return i + RowT<R>::kPad * (i >> 5); }
template <class R> __device__ __forceinline__ uint32_t tword(uint32_t k, uint32_t jf) {
    return ((k >> 7) - jf) * RowT<R>::kElems + roff<R>(k & 127u);
}
// lane q's 32 values of a row, in and out
template <class R> __device__ __forceinline__ void row_put(R* row, uint32_t q, const uint32_t v[32]) {
    uint4* r4 = (uint4*)(row + RowT<R>::kLane * q);
    if (sizeof(R) == 4) {
#pragma unroll
        for (int c = 0; c < 8; ++c) r4[c] = make_uint4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            r4[c] = make_uint4((v[8 * c] & 0xFFFFu) | (v[8 * c + 1] << 16), (v[8 * c + 2] & 0xFFFFu) | (v[8 * c + 3] << 16),
                               (v[8 * c + 4] & 0xFFFFu) | (v[8 * c + 5] << 16), (v[8 * c + 6] & 0xFFFFu) | (v[8 * c + 7] << 16));
    }
}
template <class R> __device__ __forceinline__ void row_get(const R* row, uint32_t q, uint32_t v[32]) {
    const uint4* r4 = (const uint4*)(row + RowT<R>::kLane * q);
    if (sizeof(R) == 4) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint4 t = r4[c];
            v[4 * c] = t.x; v[4 * c + 1] = t.y; v[4 * c + 2] = t.z; v[4 * c + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint4 t = r4[c];
            const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                v[8 * c + 2 * h] = w[h] & 0xFFFFu;
                v[8 * c + 2 * h + 1] = w[h] >> 16;
            }
        }
    }
}

// ---- 16-sample vector access -------------------------------------------
template <int WB> struct SampleT;
template <> struct SampleT<1> { using T = uint8_t; };
template <> struct SampleT<2> { using T = uint16_t; };
template <> struct SampleT<4> { using T = uint32_t; };

template <int WB>
__device__ __forceinline__ uint32_t load1(const void* base, uint32_t p) {
    return ((const typename SampleT<WB>::T*)base)[p];
}

// v[i] = sample p0 + i (0 beyond npx).  p0 must be a multiple of 16.
template <int WB>
__device__ __forceinline__ void load16(const void* base, uint32_t p0, uint32_t npx, bool aligned, uint32_t v[16]) {
    using T = typename SampleT<WB>::T;
    const T* b = (const T*)base;
    if (aligned && p0 + 16 <= npx) {
        const uint4* q = (const uint4*)(b + p0);
        uint32_t w[4 * WB];
#pragma unroll
        for (int i = 0; i < WB; ++i) {
            uint4 t = q[i];
            w[4 * i + 0] = t.x;
            w[4 * i + 1] = t.y;
            w[4 * i + 2] = t.z;
            w[4 * i + 3] = t.w;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (WB == 4) v[i] = w[i];
            else if (WB == 2) v[i] = (w[i >> 1] >> (16 * (i & 1))) & 0xFFFFu;
            else v[i] = (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = (p0 + i < npx) ? (uint32_t)b[p0 + i] : 0u;
    }
}

template <int WB>
__device__ __forceinline__ void store16(void* base, uint32_t p0, uint32_t npx, bool aligned, const uint32_t v[16]) {
    using T = typename SampleT<WB>::T;
    T* b = (T*)base;
    if (aligned && p0 + 16 <= npx) {
        uint32_t w[4 * WB];
#pragma unroll
        for (int i = 0; i < 4 * WB; ++i) w[i] = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (WB == 4) w[i] = v[i];
            else if (WB == 2) w[i >> 1] |= (v[i] & 0xFFFFu) << (16 * (i & 1));
            else w[i >> 2] |= (v[i] & 0xFFu) << (8 * (i & 3));
        }
        uint4* q = (uint4*)(b + p0);
#pragma unroll
        for (int i = 0; i < WB; ++i) q[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (p0 + i < npx) b[p0 + i] = (T)v[i];
    }
}

// valid-bit word mask for the last, partial word
__device__ __forceinline__ uint64_t tail_mask(uint32_t w, uint32_t nwords, uint32_t npx) {
    uint32_t r = npx & 63u;
    return (w == nwords - 1 && r) ? ((1ull << r) - 1ull) : ~0ull;
}

}  // namespace jiffy
