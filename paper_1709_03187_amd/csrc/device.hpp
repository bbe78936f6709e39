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
// by the Weyl constants after every round.  The colony uses word 0 of each
// step's block; a PartialACO plan uses words 0-2 of the block of step 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1)
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
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1)
{
    return philox_block(c0, c1, c2, c3, k0, k1).x;
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

// Guards a kernel can trip on device data that the host cannot check before
// the launch.  A kernel that trips one keeps every access in range, finishes
// normally and ORs the bit into the device's error word; the next entry point
// that synchronises (or aco_device_error) reports it as ACO_ERR_DEVICE.
enum DeviceError : uint32_t {
    kErrNextCity = 1u,    // construction or NN tour: a next city out of range (internal)
    kErrLbestCity = 2u,   // a local best row is not a permutation of 0..n-1
    kErrLbestLen = 4u,    // a local best length that no tour can have, or a kept part's
                          // length that came out negative
    kErrTourCity = 8u,    // pheromone update: a tour holds a city out of range
    kErrLength = 16u,     // pheromone update: a length <= 0, or a deposit sum that could
                          // overflow int64 (m * quantum >= 2^63)
};

// Records a tripped guard in the device's error word (bits of DeviceError);
// err may be nullptr (no report).  Callers let one lane call it.
__device__ __forceinline__ void flag_error(uint32_t *err, uint32_t bit)
{
    if (err) atomicOr(err, bit);
}

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

// DPP move of a 64-bit value (both halves moved by the same pattern); lanes
// whose source is outside the row, or whose row is masked off, receive 0.
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, Ctrl, RowMask, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), Ctrl, RowMask, 0xF,
                                               true);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Inclusive prefix sum over lanes 0..width-1 (width a power of two <= 64,
// wave-uniform) with DPP: row shifts by 1, 2, 4, 8 inside each 16-lane row,
// then the row broadcasts of lane 15 and lane 31 carry totals across rows.
__device__ __forceinline__ double wave_incl_scan_f64(double v, int width)
{
    if (width > 1) v += dpp_f64<0x111, 0xF>(v);    // row_shr:1
    if (width > 2) v += dpp_f64<0x112, 0xF>(v);    // row_shr:2
    if (width > 4) v += dpp_f64<0x114, 0xF>(v);    // row_shr:4
    if (width > 8) v += dpp_f64<0x118, 0xF>(v);    // row_shr:8
    if (width > 16) v += dpp_f64<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    if (width > 32) v += dpp_f64<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

// Inclusive running maximum with the same DPP pattern (lanes shifted in read
// 0, which never exceeds a nonnegative value).
__device__ __forceinline__ double wave_incl_max_f64(double v, int width)
{
    if (width > 1) v = fmax(v, dpp_f64<0x111, 0xF>(v));
    if (width > 2) v = fmax(v, dpp_f64<0x112, 0xF>(v));
    if (width > 4) v = fmax(v, dpp_f64<0x114, 0xF>(v));
    if (width > 8) v = fmax(v, dpp_f64<0x118, 0xF>(v));
    if (width > 16) v = fmax(v, dpp_f64<0x142, 0xA>(v));
    if (width > 32) v = fmax(v, dpp_f64<0x143, 0xC>(v));
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
    int32_t kx;       // width of the extended neighbour table by city
    int32_t kxp;      // width of the extended neighbour table by position (0: none)
};

// Extended neighbour table: the kx = min(64, n - 1) nearest cities of every
// city in (d, index) order.  Its first k columns are the candidate list; the
// rest lets the fallback find the nearest unvisited city with one row read
// whenever one of those kx cities is still unvisited.
constexpr int kExtWidth = 64;
__host__ __device__ inline int ext_width(int64_t n) { return n - 1 < kExtWidth ? (int)(n - 1) : kExtWidth; }
// The single-instance construction keeps a wider table by position: the
// nearest unvisited city after the candidates is then found in the table far
// more often (a grid search costs many dependent reads, a table row a few).
constexpr int kExtPosWidth = 256;
__host__ __device__ inline int ext_pos_width(int64_t n)
{
    return n - 1 < kExtPosWidth ? (int)(n - 1) : kExtPosWidth;
}

// A city's position is its index in `pts` (cell order).  The single-instance
// construction works on positions, so that the cities of a run of cells in
// one grid row are one contiguous range of a position-indexed visited set.
struct GridView {
    GridHdr h;
    const int32_t *cell_start;   // [ncell + 1]
    const int4 *pts;             // [n] {x, y, city, 0} in cell order
    const int32_t *ext;          // [n][ext_stride], first kx entries of a row valid
    int32_t ext_stride;
    const int32_t *pinv;         // [n] position of each city (nullptr where not built)
    const int32_t *ext_pos;      // [n][ext_pos_stride]: the kxp nearest by position, entries
                                 // positions (nullptr where not built)
    int32_t ext_pos_stride;
};

// Byte layout of the grid buffer (offsets aligned to 256 bytes).
struct GridLayout {
    static constexpr size_t kAuxOffset = 128;   // 8-byte scratch slot inside the header block
    size_t hdr, cell_start, cursor, pts, ext, pinv, ext_pos, total;
    static __host__ __device__ size_t align(size_t v) { return (v + 255) & ~(size_t)255; }
    static __host__ __device__ int64_t cap_for(int64_t n) { return 3 * n + 2; }
    __host__ __device__ explicit GridLayout(int64_t n)
    {
        const int64_t cap = cap_for(n);
        hdr = 0;
        cell_start = align(sizeof(GridHdr));
        cursor = align(cell_start + (size_t)(cap + 1) * 4);
        pts = align(cursor + (size_t)cap * 4);
        ext = align(pts + (size_t)n * 16);
        pinv = align(ext + (size_t)n * ext_width(n) * 4);
        ext_pos = align(pinv + (size_t)n * 4);
        total = align(ext_pos + (size_t)n * ext_pos_width(n) * 4);
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
    g.ext = (const int32_t *)(b + L.ext);
    g.ext_stride = g.h.kx;
    g.pinv = (const int32_t *)(b + L.pinv);
    g.ext_pos = (const int32_t *)(b + L.ext_pos);
    g.ext_pos_stride = g.h.kxp;
    return g;
}

// Cell coordinates of a city: offsets from the box corner are below 2^30, so
// unsigned 32-bit division is exact (and much cheaper than 64-bit).
__device__ __forceinline__ int cell_x(const GridHdr &h, int32_t x)
{
    return (int)((uint32_t)(x - h.x0) / (uint32_t)h.cell);
}
__device__ __forceinline__ int cell_y(const GridHdr &h, int32_t y)
{
    return (int)((uint32_t)(y - h.y0) / (uint32_t)h.cell);
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

// Inclusive prefix sum of an int over all 64 lanes with DPP row shifts and
// row broadcasts (no LDS round trips).
__device__ __forceinline__ int wave_incl_scan_i32_dpp(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, true);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, true);   // row_bcast:31
    return v;
}

// Minimum of a 64-bit key over the wave; the result is valid in lane 63.
// Lanes whose DPP source is invalid (or whose row is masked) keep their own
// value, so the neutral element never has to be materialised.
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint64_t dpp_min_step_u64(uint64_t v)
{
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, Ctrl, RowMask, 0xF, false);
    const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, Ctrl, RowMask, 0xF, false);
    const uint64_t o = ((uint64_t)ohi << 32) | olo;
    return o < v ? o : v;
}

__device__ __forceinline__ uint64_t wave_min_u64_dpp(uint64_t v)
{
    v = dpp_min_step_u64<0x111, 0xF>(v);
    v = dpp_min_step_u64<0x112, 0xF>(v);
    v = dpp_min_step_u64<0x114, 0xF>(v);
    v = dpp_min_step_u64<0x118, 0xF>(v);
    v = dpp_min_step_u64<0x142, 0xA>(v);
    v = dpp_min_step_u64<0x143, 0xC>(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

// Slot s of the region searched when the block radius grows from rin to r
// (rin = -1 for the first pass): row y = gy - r + (s >> 1); rows farther than
// rin from gy contribute their full span [gx - r, gx + r] (side 0), rows of
// the inner block their left and right remainders (side 0 / side 1).  The
// cells of one grid row are consecutive, so each slot is one contiguous range
// of `pts`.  Returns false for an empty or off-grid slot.
__device__ __forceinline__ bool block_slot(const GridHdr &h, int gx, int gy, int rin, int r, int s,
                                           int &row, int &xa, int &xb)
{
    row = gy - r + (s >> 1);
    const int side = s & 1;
    const int dy = row > gy ? row - gy : gy - row;
    if (dy > rin) {
        if (side) return false;
        xa = gx - r;
        xb = gx + r;
    } else if (side == 0) {
        xa = gx - r;
        xb = gx - rin - 1;
    } else {
        xa = gx + rin + 1;
        xb = gx + r;
    }
    xa = xa < 0 ? 0 : xa;
    xb = xb > h.gw - 1 ? h.gw - 1 : xb;
    return row >= 0 && row < h.gh && xa <= xb;
}

// Largest block radius rho (in cells, around the cell of the point) whose
// cities are all closer than d_lo, or -1.  A city in the block of radius rho
// differs from the point by less than (rho + 1) cell in x and in y, so its
// s = dx^2 + dy^2 < 2 ((rho + 1) cell)^2; with 8 ((rho + 1) cell)^2 <=
// (2 d_lo - 1)^2 its rounded distance nint(sqrt(s)) is below d_lo.
__device__ __forceinline__ int closer_block_radius(const GridHdr &h, int64_t d_lo)
{
    if (d_lo <= 0 || d_lo > (1 << 29)) return -1;
    const int64_t q2 = (2 * d_lo - 1) * (2 * d_lo - 1);
    const int64_t cell = h.cell;
    auto fits = [&](int64_t t) { const int64_t e = t * cell; return 8 * e * e <= q2; };
    int64_t t = (int64_t)((double)(2 * d_lo - 1) / ((double)cell * 2.8284271247461903));
    while (t > 0 && !fits(t)) --t;
    while (fits(t + 1)) ++t;
    const int64_t lim = (int64_t)(h.gw > h.gh ? h.gw : h.gh);
    return (int)((t < lim ? t : lim) - 1);
}

// How the grid search sees the visited set.  By city: each point is tested
// by its city index.  By position: the set is indexed by position in `pts`,
// a point is tested by its position and a whole range of positions (the
// cities of a run of cells) can be found visited with a few word reads.
template <class Visited>
struct VisitedByCity {
    static constexpr bool kByPosition = false;   // a point's test needs its city index
    const Visited &visited;
    __device__ __forceinline__ bool test(int64_t, int32_t city) const { return visited(city); }
    __device__ __forceinline__ bool all_visited(int32_t, int32_t) const { return false; }
};
struct VisitedByPosition {
    static constexpr bool kByPosition = true;    // a point is tested before it is read
    const uint32_t *w;   // bit q: position q visited
    __device__ __forceinline__ bool test(int64_t q, int32_t) const
    {
        return (w[q >> 5] >> (q & 31)) & 1u;
    }
    // true when every position in [a, b) is visited (or the range is empty)
    __device__ __forceinline__ bool all_visited(int32_t a, int32_t b) const
    {
        for (int32_t q = a; q < b; q = (q | 31) + 1) {
            const uint32_t lo = q & 31;
            const uint32_t hi = (b - (q & ~31)) >= 32 ? 32u : (uint32_t)(b - (q & ~31));
            const uint32_t mask = (hi == 32u ? ~0u : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
            if (~w[q >> 5] & mask) return false;
        }
        return true;
    }
};

// Nearest unvisited city to (cx, cy) by key (d, city), searched by the whole
// wave over square blocks of cells: radius 1 first (or, given that no
// unvisited city is closer than d_lo, the first ring outside the block that
// holds only closer cities), then rings outward: one per pass, doubling (up to
// 16) after every pass that finds no unvisited city.  Each pass reads
// the new cells as contiguous row ranges of `pts`; ranges the visited set
// shows fully visited are dropped before any point is read; the rest are
// taken one point per lane (by position only the unvisited points are read,
// and a batch of 64 visited points reads nothing; by city every point is read
// and then tested), keeping a lane-local minimum (the distance is only
// rounded for cities that can beat it); one wave reduction per pass.  The
// search stops once every city outside the searched block is provably
// farther than the best distance found (bound > d_best), so the result is
// exact.  Returns (d << 32) | city, or ~0 if every city is visited.
#ifdef ACO_STEP_PROFILE
// Step profile build only: grid searches, their passes, their batches of 64
// points and the points in the searched ranges (added by lane 0 while
// g_grid_on is set; read
// back by the profile).  The counting is switched on for an iteration the
// clock profile does not time, since its atomics slow the searches down.
static __device__ unsigned long long g_grid_stats[4];
static __device__ int g_grid_on;
#define ACO_GRID_COUNTING const bool grid_count = g_grid_on != 0;
#define ACO_GRID_STAT(i, v)                                                                 \
    do {                                                                                    \
        if (grid_count && lane == 0) atomicAdd(&g_grid_stats[i], (unsigned long long)(v)); \
    } while (0)
#else
#define ACO_GRID_COUNTING
#define ACO_GRID_STAT(i, v) do { } while (0)
#endif

template <class Vis>
__device__ uint64_t wave_nearest_unvisited(const GridView &g, int32_t cx, int32_t cy,
                                           const Vis &vis, int64_t d_lo = 0)
{
    const GridHdr &h = g.h;
    const int lane = lane_id();
    const int gx = cell_x(h, cx), gy = cell_y(h, cy);
    uint64_t best = ~0ull;
    int64_t s_cut = INT64_MAX;   // cities with s > s_cut cannot beat this lane's best
    int rin = closer_block_radius(h, d_lo);
    int width = 1;   // rings per pass: doubles after every pass that finds nothing
    ACO_GRID_COUNTING
    ACO_GRID_STAT(0, 1);
    for (int r = rin < 0 ? 1 : rin + 1;; rin = r, r = r + width) {
        ACO_GRID_STAT(1, 1);
        const int nslots = 2 * (2 * r + 1);
        for (int sb = 0; sb < nslots; sb += kWave) {
            const int s = sb + lane;
            int a = 0, b = 0, row, xa, xb;
            if (s < nslots && block_slot(h, gx, gy, rin, r, s, row, xa, xb)) {
                a = g.cell_start[(int64_t)row * h.gw + xa];
                b = g.cell_start[(int64_t)row * h.gw + xb + 1];
                if (vis.all_visited(a, b)) b = a;
            }
            const int len = b - a;
            const int incl = wave_incl_scan_i32_dpp(len);
            const int excl = incl - len;
            const int total = read_lane_i32(incl, kWave - 1);
            ACO_GRID_STAT(3, total);
            int span = nslots - sb < kWave ? nslots - sb : kWave;   // slots in this batch
            int pw = 1;
            while (pw < span) pw <<= 1;
            for (int base = 0; base < total; base += kWave) {
                ACO_GRID_STAT(2, 1);
                const int idx = base + lane;
                // first slot whose inclusive end exceeds idx owns flat index idx
                int lo = 0;
                for (int step = pw >> 1; step > 0; step >>= 1) {
                    const int v = __shfl(incl, lo + step - 1);
                    if (v <= idx) lo += step;
                }
                const int pa = __shfl(a, lo);
                const int pe = __shfl(excl, lo);
                if constexpr (Vis::kByPosition) {
                    // by position the visited set is read first: only unvisited
                    // points are loaded, and a batch of visited points loads nothing
                    const int64_t q = pa + (idx - pe);
                    const bool unv = idx < total && !vis.test(q, 0);
                    if (__ballot(unv) == 0ull) continue;
                    if (unv) {
                        const int4 pt = g.pts[q];
                        const int64_t s2 = sq_dist(cx, cy, pt.x, pt.y);
                        if (s2 <= s_cut) {
                            const uint32_t d = (uint32_t)nint_sqrt(s2);
                            const uint64_t key = ((uint64_t)d << 32) | (uint32_t)pt.z;
                            if (key < best) {
                                best = key;
                                s_cut = (int64_t)d * d + d;
                            }
                        }
                    }
                } else if (idx < total) {
                    const int64_t q = pa + (idx - pe);
                    const int4 pt = g.pts[q];
                    const int64_t s2 = sq_dist(cx, cy, pt.x, pt.y);
                    if (s2 <= s_cut && !vis.test(q, pt.z)) {
                        const uint32_t d = (uint32_t)nint_sqrt(s2);
                        const uint64_t key = ((uint64_t)d << 32) | (uint32_t)pt.z;
                        if (key < best) {
                            best = key;
                            s_cut = (int64_t)d * d + d;   // nint(sqrt(s)) <= d  <=>  s <= d^2 + d
                        }
                    }
                }
            }
        }
        best = wave_min_u64_dpp(best);
        if (best != ~0ull) {
            const int64_t d = (int64_t)(best >> 32);
            s_cut = d * d + d;
            width = 1;
        } else if (width < 16) {
            width *= 2;
        }
        int64_t bound;
        if (!outside_bound(h, cx, cy, gx, gy, r, bound)) break;
        if (best != ~0ull && bound > (int64_t)(best >> 32)) break;
    }
    return best;
}

// The fallback of a step at city c when no unvisited candidate has positive
// weight: the first unvisited city of c's extended neighbour table is the
// nearest unvisited city (the table is in (d, index) order and holds every
// city closer than its last entry); only when all of them are visited is the
// grid searched, from outside the block that holds only closer cities.
template <class Visited>
__device__ int32_t fallback_city(const GridView &g, const int32_t *xy, int32_t c,
                                 const Visited &visited)
{
    const int lane = lane_id();
    const int kx = g.h.kx;
    bool unv = false;
    int32_t j = 0;
    if (lane < kx) {
        j = g.ext[(int64_t)c * g.ext_stride + lane];
        unv = !visited(j);
    }
    const uint64_t bal = __ballot(unv);
    if (bal) return read_lane_i32(j, __ffsll((unsigned long long)bal) - 1);
    // every city closer than the table's last entry is in the table, hence
    // visited: the answer is at least as far as that entry
    const int32_t cx = xy[2 * (int64_t)c], cy = xy[2 * (int64_t)c + 1];
    const int32_t jl = read_lane_i32(j, kx - 1);
    const int64_t d_lo = nint_sqrt(sq_dist(cx, cy, xy[2 * (int64_t)jl], xy[2 * (int64_t)jl + 1]));
    return (int32_t)(uint32_t)wave_nearest_unvisited(g, cx, cy, VisitedByCity<Visited>{visited}, d_lo);
}

// The position-indexed set read as the city-indexed one is: each point is
// loaded, then tested.  The NN tour's grid searches run faster this way (its
// searched ranges hold more unvisited points than an ant's do).
struct VisitedByPositionAfterLoad : VisitedByPosition {
    static constexpr bool kByPosition = false;
};

// The same fallback on positions: c and the result are positions in `pts`,
// `vis` is a view of the position-indexed visited set.  Ties still go to the
// lower city index (keys carry the city).
template <class VP>
__device__ __forceinline__ int32_t fallback_position(const GridView &g, int32_t c, const VP &vis)
{
    const int lane = lane_id();
    const int kxp = g.h.kxp;
    const int32_t *row = g.ext_pos + (int64_t)c * g.ext_pos_stride;
    int32_t j = 0;
    // the row in chunks of 64, nearest first: the first unvisited entry is the
    // nearest unvisited city
    for (int r0 = 0; r0 < kxp; r0 += kWave) {
        bool unv = false;
        if (r0 + lane < kxp) {
            j = row[r0 + lane];
            unv = !vis.test(j, 0);
        }
        const uint64_t bal = __ballot(unv);
        if (bal) return read_lane_i32(j, __ffsll((unsigned long long)bal) - 1);
    }
    const int4 me = g.pts[c];
    const int4 pl = g.pts[row[kxp - 1]];
    const int64_t d_lo = nint_sqrt(sq_dist(me.x, me.y, pl.x, pl.y));
    const uint64_t best = wave_nearest_unvisited(g, me.x, me.y, vis, d_lo);
    if (best == ~0ull) return -1;
    return g.pinv[(uint32_t)best];
}

}  // namespace aco
