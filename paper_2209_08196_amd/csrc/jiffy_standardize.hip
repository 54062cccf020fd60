// Input standardization for gfx950 (Sec. III-A): Cartesian points of many
// scans become range images on the codec's canonical H x W grid, and the
// points' attributes become attribute images of the same grid.
//
//   k_std_clear   every cell's key to "empty"
//   k_std_points  per point: spherical coordinates in double, the cell (row
//                 by elevation, column by azimuth), the range quantized to
//                 the image's unsigned width; a valid point offers the key
//                 q << 32 | point index to its cell with a 64-bit atomic
//                 minimum, so the nearest point wins and, among points of
//                 equal q, the earliest
//   k_std_gather  per cell: the winner's q and its attributes, zeros for an
//                 empty cell
//
// The arithmetic that decides a cell or a range is done in IEEE double with
// one rounding per operation in a fixed order (no contraction into fused
// multiply-adds), so only atan2 (not correctly rounded) can place a point
// lying within a few units in the last place of a bin edge differently from
// another implementation.  The points kernel reads 12 bytes per point and
// the key array stays in L2 for scans of a few hundred thousand cells.
#define JIFFY_KERNEL_TU 1
#include "jiffy_device.h"

namespace jiffy {

constexpr double kTwoPi = 2.0 * 3.14159265358979323846;

__global__ __launch_bounds__(256) void k_std_clear(StdArgs g) {
    const uint64_t n = (uint64_t)g.n_scans * g.cells;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        g.keys[i] = ~0ull;
}

// Cell index (row * W + col) and q of one point, or false when the point is
// dropped (a non-finite coordinate, outside the band, q out of range).
__device__ __forceinline__ bool std_bin(const StdArgs& g, float fx, float fy, float fz, uint32_t& cell,
                                        uint32_t& q) {
#pragma clang fp contract(off)
    const double x = fx, y = fy, z = fz;
    const double h2 = x * x + y * y;
    const double h = sqrt(h2);
    const double r = sqrt(h2 + z * z);
    const double e = atan2(z, h);
    double a = atan2(y, x);
    if (a < 0.0) a = a + kTwoPi;
    const double fr = floor(((g.elev_hi - e) * (double)g.height) / g.span);
    double fc = floor((a * (double)g.width) / kTwoPi);
    if (fc == (double)g.width) fc = 0.0;
    const double fq = floor(r / g.unit + 0.5);
    // comparisons are false for NaN, so a non-finite value drops the point
    if (!(fr >= 0.0 && fr < (double)g.height && fc >= 0.0 && fc < (double)g.width && fq >= 1.0 && fq <= g.qmax))
        return false;
    cell = (uint32_t)fr * g.width + (uint32_t)fc;
    q = (uint32_t)fq;
    return true;
}

__global__ __launch_bounds__(256) void k_std_points(StdArgs g) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t n = (uint64_t)g.n_scans * g.n_points;
    if (i >= n) return;
    const float* p = g.xyz + 3 * i;
    const float fx = p[0], fy = p[1], fz = p[2];
    uint32_t cell, q;
    if (!std_bin(g, fx, fy, fz, cell, q)) return;
    const uint64_t s = i / g.n_points;
    const uint32_t idx = (uint32_t)(i - s * g.n_points);
    atomicMin((unsigned long long*)(g.keys + s * g.cells + cell), ((unsigned long long)q << 32) | idx);
}

template <typename T>
__device__ __forceinline__ uint32_t ld_any(const void* base, uint64_t i) {
    return ((const T*)base)[i];
}
template <typename T>
__device__ __forceinline__ void st_any(void* base, uint64_t i, uint32_t v) {
    ((T*)base)[i] = (T)v;
}
__device__ __forceinline__ uint32_t ld_w(const void* base, uint32_t wb, uint64_t i) {
    return wb == 1 ? ld_any<uint8_t>(base, i) : wb == 2 ? ld_any<uint16_t>(base, i) : ld_any<uint32_t>(base, i);
}
__device__ __forceinline__ void st_w(void* base, uint32_t wb, uint64_t i, uint32_t v) {
    if (wb == 1) st_any<uint8_t>(base, i, v);
    else if (wb == 2) st_any<uint16_t>(base, i, v);
    else st_any<uint32_t>(base, i, v);
}

__global__ __launch_bounds__(256) void k_std_gather(StdArgs g) {
    const uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t n = (uint64_t)g.n_scans * g.cells;
    if (c >= n) return;
    const uint64_t key = g.keys[c];
    const bool hit = key != ~0ull;
    const uint64_t s = c / g.cells;
    const uint64_t src = s * g.n_points + (uint32_t)key;
    st_w(g.range, g.range_bytes, c, hit ? (uint32_t)(key >> 32) : 0u);
    for (uint32_t a = 0; a < g.n_attrs; ++a)
        st_w(g.attr_out[a], g.attr_bytes[a], c, hit ? ld_w(g.attr_in[a], g.attr_bytes[a], src) : 0u);
}

hipError_t launch_standardize(const StdArgs& g, hipStream_t stream) {
    const uint64_t cells = (uint64_t)g.n_scans * g.cells, pts = (uint64_t)g.n_scans * g.n_points;
    if (cells == 0) return hipSuccess;
    const uint32_t cb = (uint32_t)((cells + 255) / 256);
    JIFFY_LAUNCH("k_std_clear", k_std_clear, dim3(cb < 4096 ? cb : 4096), dim3(256), stream, g);
    if (pts) JIFFY_LAUNCH("k_std_points", k_std_points, dim3((uint32_t)((pts + 255) / 256)), dim3(256), stream, g);
    JIFFY_LAUNCH("k_std_gather", k_std_gather, dim3(cb), dim3(256), stream, g);
    return hipGetLastError();
}

}  // namespace jiffy
