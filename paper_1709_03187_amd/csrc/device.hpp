// Device building blocks shared by the ACO kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aco {

constexpr int kWave = 64;
constexpr uint32_t kNoSlot = 255;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11).  Ten rounds of the two-multiply S-box; the key advances
// by the Weyl constants after every round.  Only word 0 of the output block is
// needed by the colony.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = c0 * 0xD2511F53u;
        const uint32_t hi0 = __umulhi(c0, 0xD2511F53u);
        const uint32_t lo1 = c2 * 0xCD9E8D57u;
        const uint32_t hi1 = __umulhi(c2, 0xCD9E8D57u);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

// Word for (seed, iteration, ant, step): counter (step, ant, iteration, 0).
__device__ __forceinline__ uint32_t colony_draw(uint64_t seed, uint32_t iteration, uint32_t ant,
                                                uint32_t step)
{
    return philox_word0(step, ant, iteration, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------------------
// Exact integer distance d = nint(sqrt(s)).  FP64 sqrt gives floor(sqrt(s))
// to within one unit; integer corrections make it exact for s < 2^62.  Then
// sqrt(s) >= r + 1/2 exactly when s - r^2 > r (integers; never a tie).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t sq_dist(int32_t x1, int32_t y1, int32_t x2, int32_t y2)
{
    const int64_t dx = (int64_t)x1 - (int64_t)x2;
    const int64_t dy = (int64_t)y1 - (int64_t)y2;
    return dx * dx + dy * dy;
}

__device__ __forceinline__ int32_t nint_sqrt(int64_t s64)
{
    const uint64_t s = (uint64_t)s64;
    uint64_t r = (uint64_t)sqrt((double)s);
    while (r * r > s) --r;
    while ((r + 1) * (r + 1) <= s) ++r;
    return (int32_t)((s - r * r > r) ? r + 1 : r);
}

// ---------------------------------------------------------------------------
// Wave-level helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ int32_t read_lane_i32(int32_t v, int lane)
{
    return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ double read_lane_f64(double v, int lane)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int wave_incl_scan_i32(int v, int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Uniform grid over the bounding box: square cells of side `cell` (integer),
// gw x gh cells, cities bucketed by cell (row-major cell order) with their
// coordinates copied next to their index so that a run of cells in one grid
// row is one contiguous range of `pts`.
// ---------------------------------------------------------------------------
struct GridHdr {
    int32_t x0, y0;   // bounding-box minimum
    int32_t cell;     // cell side >= 1
    int32_t gw, gh;   // cells per row / column
    int32_t ncell;    // gw * gh
    int32_t n;        // cities
    int32_t cap;      // capacity of cell_start (>= ncell + 1)
};

struct GridView {
    GridHdr h;
    const int32_t *cell_start;   // [ncell + 1]
    const int4 *pts;             // [n] {x, y, city, 0} in cell order
};

// Byte layout of the grid buffer (offsets aligned to 256 bytes).
struct GridLayout {
    static constexpr size_t kAuxOffset = 128;   // 8-byte scratch slot inside the header block
    size_t hdr, cell_start, cursor, pts, total;
    static __host__ __device__ size_t align(size_t v) { return (v + 255) & ~(size_t)255; }
    static __host__ __device__ int64_t cap_for(int64_t n) { return 3 * n + 2; }
    __host__ __device__ explicit GridLayout(int64_t n)
    {
        const int64_t cap = cap_for(n);
        hdr = 0;
        cell_start = align(sizeof(GridHdr));
        cursor = align(cell_start + (size_t)(cap + 1) * 4);
        pts = align(cursor + (size_t)cap * 4);
        total = align(pts + (size_t)n * 16);
    }
};

__device__ __forceinline__ GridView grid_view(const void *grid)
{
    const char *b = (const char *)grid;
    GridView g;
    g.h = *(const GridHdr *)b;
    const GridLayout L(g.h.n);
    g.cell_start = (const int32_t *)(b + L.cell_start);
    g.pts = (const int4 *)(b + L.pts);
    return g;
}

__device__ __forceinline__ int cell_x(const GridHdr &h, int32_t x)
{
    return (int)(((int64_t)x - h.x0) / h.cell);
}
__device__ __forceinline__ int cell_y(const GridHdr &h, int32_t y)
{
    return (int)(((int64_t)y - h.y0) / h.cell);
}

// Smallest distance from (cx, cy) to any integer point outside the block of
// cells [gx-r, gx+r] x [gy-r, gy+r]; returns false when the block already
// covers the whole grid (nothing lies outside).
__device__ __forceinline__ bool outside_bound(const GridHdr &h, int32_t cx, int32_t cy, int gx,
                                              int gy, int r, int64_t &bound)
{
    bool any = false;
    int64_t b = INT64_MAX;
    if (gx - r > 0) {
        const int64_t v = (int64_t)cx - ((int64_t)h.x0 + (int64_t)(gx - r) * h.cell) + 1;
        b = v < b ? v : b;
        any = true;
    }
    if (gx + r < h.gw - 1) {
        const int64_t v = (int64_t)h.x0 + (int64_t)(gx + r + 1) * h.cell - cx;
        b = v < b ? v : b;
        any = true;
    }
    if (gy - r > 0) {
        const int64_t v = (int64_t)cy - ((int64_t)h.y0 + (int64_t)(gy - r) * h.cell) + 1;
        b = v < b ? v : b;
        any = true;
    }
    if (gy + r < h.gh - 1) {
        const int64_t v = (int64_t)h.y0 + (int64_t)(gy + r + 1) * h.cell - cy;
        b = v < b ? v : b;
        any = true;
    }
    bound = b;
    return any;
}

// Segment s of ring r around (gx, gy) as a range of cells in one grid row:
// s = 0, 1 are the bottom/top rows of the ring; s >= 2 the single side cells.
// Returns false if the segment lies outside the grid.
__device__ __forceinline__ bool ring_segment(const GridHdr &h, int gx, int gy, int r, int s,
                                             int &row, int &xa, int &xb)
{
    if (r == 0) {
        row = gy;
        xa = xb = gx;
    } else if (s < 2) {
        row = (s == 0) ? gy - r : gy + r;
        xa = gx - r;
        xb = gx + r;
    } else {
        const int q = s - 2;
        row = gy - r + 1 + (q >> 1);
        xa = xb = (q & 1) ? gx + r : gx - r;
    }
    xa = xa < 0 ? 0 : xa;
    xb = xb > h.gw - 1 ? h.gw - 1 : xb;
    return row >= 0 && row < h.gh && xa <= xb;
}

__device__ __forceinline__ int ring_segments(int r) { return r == 0 ? 1 : 4 * r; }

// Nearest unvisited city to (cx, cy) by key (d, city), searched ring by ring
// on the grid by the whole wave.  `visited(city)` tests the ant's bitmask.
// Rings stop once every point outside the searched block is provably farther
// than the best distance found (bound > d_best), so the result is exact.
// Returns (d << 32) | city, or ~0 if every city is visited.
template <class Visited>
__device__ uint64_t wave_nearest_unvisited(const GridView &g, int32_t cx, int32_t cy,
                                           const Visited &visited)
{
    const GridHdr &h = g.h;
    const int lane = lane_id();
    const int gx = cell_x(h, cx), gy = cell_y(h, cy);
    uint64_t best = ~0ull;
    for (int r = 0;; ++r) {
        const int nseg = ring_segments(r);
        for (int sb = 0; sb < nseg; sb += kWave) {
            const int s = sb + lane;
            int a = 0, b = 0, row, xa, xb;
            if (s < nseg && ring_segment(h, gx, gy, r, s, row, xa, xb)) {
                a = g.cell_start[(int64_t)row * h.gw + xa];
                b = g.cell_start[(int64_t)row * h.gw + xb + 1];
            }
            const int len = b - a;
            const int incl = wave_incl_scan_i32(len, lane);
            const int excl = incl - len;
            const int total = read_lane_i32(incl, kWave - 1);
            for (int base = 0; base < total; base += kWave) {
                const int idx = base + lane;
                // first lane whose inclusive end exceeds idx owns point idx
                int lo = 0;
#pragma unroll
                for (int step = kWave / 2; step > 0; step >>= 1) {
                    const int v = __shfl(incl, lo + step - 1);
                    if (v <= idx) lo += step;
                }
                const int pa = __shfl(a, lo);
                const int pe = __shfl(excl, lo);
                if (idx < total) {
                    const int4 pt = g.pts[pa + (idx - pe)];
                    if (!visited(pt.z)) {
                        const uint64_t key =
                            ((uint64_t)(uint32_t)nint_sqrt(sq_dist(cx, cy, pt.x, pt.y)) << 32) |
                            (uint32_t)pt.z;
                        best = key < best ? key : best;
                    }
                }
            }
        }
        best = wave_min_u64(best);
        int64_t bound;
        if (!outside_bound(h, cx, cy, gx, gy, r, bound)) break;
        if (best != ~0ull && bound > (int64_t)(best >> 32)) break;
    }
    return best;
}

}  // namespace aco
